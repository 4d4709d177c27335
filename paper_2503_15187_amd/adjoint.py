"""Differentiable EV-FDLB runs on top of the discrete-adjoint C ABI.

Rollout (a torch.autograd.Function) advances a state nsteps TVD-RK3 steps
and returns the final state together with the history of the mass flux
sum_k p_k F_k through one node after every step.  The forward pass keeps a
checkpoint every ceil(sqrt(nsteps)) steps.  The backward pass re-runs each
segment from its checkpoint with evlb_step_record (states and stage states
kept) and transposes it with evlb_adjoint_record, walking the segments in
reverse, the recomputation of the next segment on a second context and
stream overlapping the transposition of the current one; it returns the gradients with respect to the initial state and to
the parameters phi_sigma and sigma (the latter two enter as 0-d tensors whose
values must equal the context's; they only carry the gradient).

Equilibrium maps (n, u, T) fields to the initial reduced Maxwellian with
evlb_set_equilibrium; its backward uses evlb_equilibrium_adjoint.
"""
import math

import torch


class Equilibrium(torch.autograd.Function):
    @staticmethod
    def forward(ctx, n, u, T, solver):
        ctx.solver = solver
        ctx.save_for_backward(n, u, T)
        return solver.equilibrium(n.detach().contiguous(), u.detach().contiguous(), T.detach().contiguous())

    @staticmethod
    def backward(ctx, lam):
        n, u, T = ctx.saved_tensors
        g = ctx.solver.equilibrium_adjoint(n.contiguous(), u.contiguous(), T.contiguous(), lam.contiguous())
        return g[0], g[1], g[2], None


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f0, phi, sigma, solver, nsteps, flux_node, every=None):
        nsteps = int(nsteps)
        every = int(every) if every else max(1, int(math.ceil(math.sqrt(nsteps))))
        dev = f0.device
        vel = torch.tensor(solver.velocities, dtype=torch.float64, device=dev)
        rec = solver.record_buffer(every)
        R = rec.numel() // (every + 1)
        N = solver.n_tot
        # offsets of F_k(flux_node) inside a record, k = 0..q-1
        kofs = torch.arange(solver.q, device=dev) * N + flux_node
        f = f0.detach().contiguous()
        ckpt = {}
        flux = torch.empty(nsteps, dtype=torch.float64, device=dev)
        for start in range(0, nsteps, every):
            seg = min(every, nsteps - start)
            ckpt[start] = f.clone()
            solver.step_record(f, seg, rec)
            idx = (torch.arange(1, seg + 1, device=dev) * R)[:, None] + kofs[None, :]
            flux[start:start + seg] = rec[idx] @ vel
            f = solver.record_state(rec, seg).clone()
        ctx.solver, ctx.nsteps, ctx.every, ctx.flux_node = solver, nsteps, every, flux_node
        ctx.ckpt, ctx.vel = ckpt, vel
        return f, flux

    @staticmethod
    def backward(ctx, g_f, g_flux):
        solver, nsteps, every, node = ctx.solver, ctx.nsteps, ctx.every, ctx.flux_node
        lam = torch.zeros_like(ctx.ckpt[0]) if g_f is None else g_f.detach().clone().contiguous()
        obs = w = None
        if g_flux is not None:
            obs = torch.zeros_like(lam)
            obs[0, :, node] = ctx.vel
            w = g_flux.detach().contiguous()
        dparams = torch.zeros(2, dtype=torch.float64, device=lam.device)
        # The segments in reverse.  The recomputation of segment i + 1 (a
        # second context on a second stream, into the other record buffer)
        # runs while segment i is transposed: the two chains of small
        # launches fill the device together.
        starts = sorted(ctx.ckpt, reverse=True)
        recomp = getattr(solver, "_adjoint_twin", None)
        if recomp is None:
            recomp = solver._adjoint_twin = solver.twin()
        recs = [solver.record_buffer(every), solver.record_buffer(every)]
        main = torch.cuda.current_stream(lam.device)
        side = torch.cuda.Stream(device=lam.device)
        side.wait_stream(main)
        ready = [torch.cuda.Event() for _ in starts]
        freed = [torch.cuda.Event(), torch.cuda.Event()]

        def recompute(i):
            seg = min(every, nsteps - starts[i])
            if i >= 2:
                side.wait_event(freed[i % 2])  # segment i - 2 no longer reads this buffer
            recomp.step_record(ctx.ckpt[starts[i]], seg, recs[i % 2], stream=side)
            ready[i].record(side)

        recompute(0)
        if len(starts) > 1:
            recompute(1)
        for i, start in enumerate(starts):
            seg = min(every, nsteps - start)
            main.wait_event(ready[i])
            solver.adjoint_record(recs[i % 2], seg, lam, dparams, obs, None if w is None else w[start:start + seg],
                                  stream=main)
            freed[i % 2].record(main)
            if i + 2 < len(starts):
                recompute(i + 2)
        for r in recs:
            r.record_stream(side)
        return lam, dparams[0], dparams[1], None, None, None, None


def rollout(f0, phi, sigma, solver, nsteps, flux_node, every=None):
    return Rollout.apply(f0, phi, sigma, solver, nsteps, flux_node, every)


def slab_loss(n0, phi, sigma, solver, nsteps, flux_node, dt, dx, target, T0, every=None):
    """Time-integrated mass flux through flux_node plus the L2 misfit of the
    final density to a target: L = dt sum_n J(f^n) + 1/2 sum_i dx (n_i - n*_i)^2,
    differentiable in n0 (initial density, at rest, temperature T0), phi
    and sigma."""
    u0 = torch.zeros_like(n0)
    f0 = Equilibrium.apply(n0, u0, T0, solver)
    fN, flux = rollout(f0, phi, sigma, solver, nsteps, flux_node, every)
    nN = fN[0].sum(0)
    return dt * flux.sum() + 0.5 * dx * ((nN - target) ** 2).sum()
