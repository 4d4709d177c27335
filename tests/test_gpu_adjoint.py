"""Discrete adjoint of the EV-FDLB step (evlb_adjoint_step) against the
oracle: the transpose Jacobian of one TVD-RK3 step element by element from
complex-step columns of the oracle step, dot-product tests at larger sizes,
the parameter derivatives, the equilibrium adjoint, and gradients of the
slab loss through the checkpointed rollout."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads  # noqa: E402
from oracle import step1d, loss as oloss  # noqa: E402
from oracle.model import Params  # noqa: E402

pytestmark = pytest.mark.gpu

E = AD = None
H = 1e-30


def setup_module(module):
    global E, AD
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_15187_amd import evlb as _E, adjoint as _AD
    E, AD = _E, _AD


def td(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def state(N, Q, dx, seed=0, amp=0.2):
    rng = np.random.default_rng(seed)
    x = np.arange(N)
    n = 0.3 * (1 + amp * np.sin(2 * np.pi * x / N) + 0.02 * rng.standard_normal(N))
    u = 0.05 * np.cos(2 * np.pi * x / N)
    T = 0.6 * (1 + 0.05 * np.sin(4 * np.pi * x / N))
    return n, u, T, rng


def oracle_step(F, G, Q, dx, dt, **kw):
    tb = step1d.Tables(Params(Q=Q, dx=dx, dt=dt, **kw))
    return step1d.rk3_step(F, G, tb)


@pytest.mark.parametrize("mask", [1, 2, 4, 8, 15])
def test_adjoint_step_equals_transposed_jacobian(mask):
    """lam^n = (d f^{n+1} / d f^n)^T lam^{n+1}, every element, against
    complex-step columns of the oracle step (40 nodes, Q = 8)."""
    N, Q, dx, dt = 40, 8, 1 / 8, 0.005
    n, u, T, rng = state(N, Q, dx)
    tb = step1d.Tables(Params(Q=Q, dx=dx, dt=dt, term_mask=mask))
    F, G = step1d.initial_state(n, u, T, tb)
    F = F * (1 + 0.05 * rng.standard_normal(F.shape))
    G = G * (1 + 0.05 * rng.standard_normal(G.shape))
    lam = rng.standard_normal((2, Q, N))
    s = E.Solver(Q, dx, dt, N, term_mask=mask, adjoint=1)
    dpar = torch.zeros(2, dtype=torch.float64, device="cuda")
    got = s.adjoint_step(td(np.stack([F, G])), td(lam), dpar).cpu().numpy()
    ref = np.zeros((2, Q, N))
    for pl in range(2):
        for k in range(Q):
            for i in range(N):
                Fc, Gc = F.astype(complex), G.astype(complex)
                (Fc if pl == 0 else Gc)[k, i] += 1j * H
                F1, G1 = step1d.rk3_step(Fc, Gc, tb)
                ref[pl, k, i] = (np.sum(lam[0] * F1) + np.sum(lam[1] * G1)).imag / H
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"mask {mask}: max rel err {err:.2e}", flush=True)
    assert err < 1e-11
    # explicit parameter derivatives of <lam, f^{n+1}>
    dp = dpar.cpu().numpy()
    for which, idx in (("phi", 0), ("sigma", 1)):
        kw = {which: 1.0 + 1j * H}
        F1, G1 = oracle_step(F.astype(complex), G.astype(complex), Q, dx, dt, term_mask=mask, **kw)
        r = (np.sum(lam[0] * F1) + np.sum(lam[1] * G1)).imag / H
        assert abs(dp[idx] - r) <= 1e-10 * max(1.0, abs(r)), (which, dp[idx], r)


@pytest.mark.parametrize("Q,N,dx", [(16, 150, 1 / 8), (24, 130, 1 / 8), (16, 200, 1 / 4), (8, 140, 1 / 8)])
def test_adjoint_dot_product(Q, N, dx):
    """<J^T lam, v> (GPU adjoint) = <lam, J v> (oracle complex step along v)."""
    dt = 0.2 * dx / 8.6
    n, u, T, rng = state(N, Q, dx, seed=5)
    tb = step1d.Tables(Params(Q=Q, dx=dx, dt=dt))
    F, G = step1d.initial_state(n, u, T, tb)
    lam = rng.standard_normal((2, Q, N))
    v = rng.standard_normal((2, Q, N)) * np.concatenate([F, G]).reshape(2, Q, N)
    s = E.Solver(Q, dx, dt, N, adjoint=1)
    dpar = torch.zeros(2, dtype=torch.float64, device="cuda")
    got = s.adjoint_step(td(np.stack([F, G])), td(lam), dpar).cpu().numpy()
    F1, G1 = step1d.rk3_step(F + 1j * H * v[0], G + 1j * H * v[1], tb)
    ref = (np.sum(lam[0] * F1) + np.sum(lam[1] * G1)).imag / H
    lhs = np.sum(got * v)
    assert abs(lhs - ref) <= 1e-12 * np.sum(np.abs(got * v)), (lhs, ref)


def test_adjoint_ragged_batch_dot_product():
    """Several systems (multi-tile and shorter than a tile) in one state."""
    Q, dx = 16, 1 / 8
    dt = 0.2 * dx / 6.7
    nxs = [70, 33, 130]
    parts = [state(N, Q, dx, seed=i) for i, N in enumerate(nxs)]
    tb = step1d.Tables(Params(Q=Q, dx=dx, dt=dt))
    rng = np.random.default_rng(9)
    s = E.Solver(Q, dx, dt, nxs, adjoint=1)
    Fs = [step1d.initial_state(n, u, T, tb) for n, u, T, _ in parts]
    f = np.concatenate([np.stack(x) for x in Fs], axis=2)
    lam = rng.standard_normal(f.shape)
    v = rng.standard_normal(f.shape) * f
    dpar = torch.zeros(2, dtype=torch.float64, device="cuda")
    got = s.adjoint_step(td(f), td(lam), dpar).cpu().numpy()
    ref, off = 0.0, 0
    for (F, G), N in zip(Fs, nxs):
        F1, G1 = step1d.rk3_step(F + 1j * H * v[0, :, off:off + N], G + 1j * H * v[1, :, off:off + N], tb)
        ref += (np.sum(lam[0, :, off:off + N] * F1) + np.sum(lam[1, :, off:off + N] * G1)).imag / H
        off += N
    lhs = np.sum(got * v)
    assert abs(lhs - ref) <= 1e-12 * np.sum(np.abs(got * v))


def test_equilibrium_adjoint():
    Q, N, dx = 16, 64, 1 / 8
    n, u, T, rng = state(N, Q, dx, seed=2)
    tb = step1d.Tables(Params(Q=Q, dx=dx, dt=1e-3))
    lam = rng.standard_normal((2, Q, N))
    s = E.Solver(Q, dx, 1e-3, N)
    got = s.equilibrium_adjoint(td(n), td(u), td(T), td(lam)).cpu().numpy()
    for idx, base in enumerate((n, u, T)):
        dirv = rng.standard_normal(N)
        args = [n.astype(complex), u.astype(complex), T.astype(complex)]
        args[idx] = args[idx] + 1j * H * dirv
        F, G = step1d.initial_state(*args, tb)
        ref = (np.sum(lam[0] * F) + np.sum(lam[1] * G)).imag / H
        assert abs(np.sum(got[idx] * dirv) - ref) <= 1e-12 * np.sum(np.abs(got[idx] * dirv)) + 1e-14


def small_slab(nx=64, dx=1 / 8):
    c, n0, u, T = workloads.slab_1d(name="adjoint_slab_1d", nx=nx, dx=dx)
    c = dict(c)
    c["x0"] = 2.0
    x = workloads.grid(nx, dx)
    n0 = workloads.tanh_slab(x, c["n_l"], c["n_v"], c["x0"], 0.5)
    target = workloads.adjoint_target(dict(c, nx=nx, dx=dx), n0)
    i_f = nx // 2 + int(round(3.0 / dx))
    return c, n0, target, i_f


def test_slab_loss_gradients_match_complex_step():
    """Gradients of the slab loss (flux through x = 3 sigma plus the final
    misfit) over 20 steps at 64 nodes, dx = sigma/8, Q = 16, through the
    checkpointed rollout (checkpoint every 5 steps): d/dphi, d/dsigma and a
    random direction in the initial density, against complex step of the
    oracle loss."""
    c, n0, target, i_f = small_slab()
    Q, dx, T0 = 16, 1 / 8, c["T"]
    dt = 0.2 * dx / 6.6308782
    nsteps = 20
    s = E.Solver(Q, dx, dt, len(n0), adjoint=1)
    n0t = td(n0).requires_grad_(True)
    phi = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    sig = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    L = AD.slab_loss(n0t, phi, sig, s, nsteps, i_f, dt, dx, td(target), td(np.full(len(n0), T0)), every=5)
    gn, gphi, gsig = torch.autograd.grad(L, [n0t, phi, sig])
    L0 = oloss.slab_loss(n0, T0, Q, dx, dt, nsteps, i_f, target)
    assert abs(L.item() - L0) < 1e-12 * abs(L0)
    ref_phi = oloss.slab_loss(n0, T0, Q, dx, dt, nsteps, i_f, target, phi=1.0 + 1j * H).imag / H
    ref_sig = oloss.slab_loss(n0, T0, Q, dx, dt, nsteps, i_f, target, sigma=1.0 + 1j * H).imag / H
    dirv = np.random.default_rng(4).standard_normal(len(n0))
    ref_n = oloss.slab_loss(n0 + 1j * H * dirv, T0, Q, dx, dt, nsteps, i_f, target).imag / H
    print(f"dL/dphi {gphi.item():.12e} vs {ref_phi:.12e}; dL/dsigma {gsig.item():.12e} vs {ref_sig:.12e}", flush=True)
    assert abs(gphi.item() - ref_phi) <= 1e-9 * abs(ref_phi)
    assert abs(gsig.item() - ref_sig) <= 1e-9 * abs(ref_sig)
    gdir = float(np.sum(gn.cpu().numpy() * dirv))
    assert abs(gdir - ref_n) <= 1e-9 * np.sum(np.abs(gn.cpu().numpy() * dirv))


def test_full_size_adjoint_gradients_match_finite_differences():
    """Adjoint workload at full size (2048 nodes, dx = sigma/4, Q = 16, slab
    at 0.85 T_c, flux node x = 128 sigma) over its 2000 steps: adjoint gradients
    against finite differences of the GPU loss (central in phi_sigma and in a
    direction of the initial density; second-order backward in sigma, whose
    kernel has a node on the branch point |x' - x| = sigma, third order))."""
    c, n0, u0, T0 = workloads.slab_1d(name="adjoint_slab_1d")
    target = workloads.adjoint_target(c, n0)
    i_f = c["nx"] // 2 + int(round(c["x_flux"] / c["dx"]))
    nsteps = c["steps"]

    def loss(phi=1.0, sigma=1.0, dn=None, grad=False):
        s = E.Solver(c["Q"], c["dx"], c["dt"], c["nx"], phi_sigma=phi, sigma=sigma, adjoint=1)
        n = td(n0 if dn is None else n0 + dn)
        if grad:
            n.requires_grad_(True)
        ph = torch.tensor(phi, dtype=torch.float64, device="cuda", requires_grad=grad)
        sg = torch.tensor(sigma, dtype=torch.float64, device="cuda", requires_grad=grad)
        L = AD.slab_loss(n, ph, sg, s, nsteps, i_f, c["dt"], c["dx"], td(target), td(T0))
        if grad:
            return L.item(), torch.autograd.grad(L, [n, ph, sg])
        return L.item()

    L0, (gn, gphi, gsig) = loss(grad=True)
    h = 1e-5
    fd_phi = (loss(phi=1 + h) - loss(phi=1 - h)) / (2 * h)
    # third-order backward difference (the sigma derivative is one-sided)
    fd_sig = (11 * L0 - 18 * loss(sigma=1 - h) + 9 * loss(sigma=1 - 2 * h) - 2 * loss(sigma=1 - 3 * h)) / (6 * h)
    dirv = np.random.default_rng(11).standard_normal(len(n0)) * 1e-3
    fd_n = (loss(dn=h * dirv) - loss(dn=-h * dirv)) / (2 * h)
    gd = float(np.sum(gn.cpu().numpy() * dirv))
    print(f"phi {gphi.item():.10e} fd {fd_phi:.10e}; sigma {gsig.item():.10e} fd {fd_sig:.10e}; "
          f"n0 {gd:.10e} fd {fd_n:.10e}", flush=True)
    assert abs(gphi.item() - fd_phi) <= 1e-6 * abs(fd_phi)
    assert abs(gsig.item() - fd_sig) <= 1e-6 * abs(fd_sig)
    assert abs(gd - fd_n) <= 1e-6 * abs(fd_n)


def test_record_adjoint_matches_step_by_step():
    """evlb_adjoint_record over a recorded segment equals repeated
    evlb_adjoint_step calls (with the same per-step observable)."""
    Q, N, dx = 16, 90, 1 / 8
    dt = 0.2 * dx / 6.7
    n, u, T, rng = state(N, Q, dx, seed=8)
    s = E.Solver(Q, dx, dt, N, adjoint=1)
    f0 = s.equilibrium(td(n), td(u), td(T))
    nst = 6
    rec = s.record_buffer(nst)
    s.step_record(f0, nst, rec)
    fe = f0.clone()
    states = [fe.clone()]
    for _ in range(nst):
        s.step(fe, 1)
        states.append(fe.clone())
    last = s.record_state(rec, nst)
    assert ((last - states[-1]).abs().max() / states[-1].abs().max()).item() < 1e-13
    lam0 = td(rng.standard_normal((2, Q, N)))
    obs = td(rng.standard_normal((2, Q, N)))
    w = td(rng.standard_normal(nst))
    d1 = torch.zeros(2, dtype=torch.float64, device="cuda")
    d2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    la = lam0.clone()
    s.adjoint_record(rec, nst, la, d1, obs, w)
    lb = lam0.clone()
    for j in range(nst - 1, -1, -1):
        lb = lb + w[j] * obs
        lb = s.adjoint_step(states[j], lb, d2)
    assert ((la - lb).abs().max() / lb.abs().max()).item() < 1e-12
    assert torch.allclose(d1, d2, rtol=1e-12, atol=0)
