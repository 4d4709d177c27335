"""Differentiable EV-FDLB runs on top of the discrete-adjoint C ABI.

Rollout (a torch.autograd.Function) advances a state nsteps TVD-RK3 steps
and returns the final state together with the history of the mass flux
sum_k p_k F_k through one node after every step.  Its backward pass walks the
steps in reverse with evlb_adjoint_step, recomputing the forward states of
each segment from checkpoints stored every ceil(sqrt(nsteps)) steps, and
returns the gradients with respect to the initial state and to the
parameters phi_sigma and sigma (the latter two enter as 0-d tensors whose
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
        vel = torch.tensor(solver.velocities, dtype=torch.float64, device=f0.device)
        f = f0.detach().clone().contiguous()
        ckpt = {0: f.clone()}
        flux = torch.empty(nsteps, dtype=torch.float64, device=f0.device)
        for s in range(1, nsteps + 1):
            solver.step(f, 1)
            flux[s - 1] = (vel * f[0, :, flux_node]).sum()
            if s % every == 0 and s < nsteps:
                ckpt[s] = f.clone()
        ctx.solver, ctx.nsteps, ctx.every, ctx.flux_node = solver, nsteps, every, flux_node
        ctx.ckpt, ctx.vel = ckpt, vel
        return f, flux

    @staticmethod
    def backward(ctx, g_f, g_flux):
        solver, nsteps, every, node = ctx.solver, ctx.nsteps, ctx.every, ctx.flux_node
        lam = torch.zeros_like(ctx.ckpt[0]) if g_f is None else g_f.detach().clone().contiguous()
        gfl = None if g_flux is None else g_flux.detach()
        dparams = torch.zeros(2, dtype=torch.float64, device=lam.device)
        for start in sorted(ctx.ckpt, reverse=True):
            end = min(start + every, nsteps)
            states = [ctx.ckpt[start]]
            f = ctx.ckpt[start].clone()
            for _ in range(start, end - 1):
                solver.step(f, 1)
                states.append(f.clone())
            for n in range(end - 1, start - 1, -1):
                if gfl is not None:
                    lam[0, :, node] += gfl[n] * ctx.vel
                lam = solver.adjoint_step(states[n - start], lam, dparams)
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
