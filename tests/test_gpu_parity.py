"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerance: the method is FP64 throughout; the two sides differ only in
summation order (and the WENO-5 weights' common denominator), so one step
must agree to 1e-11 relative and 1000 steps to 1e-8 relative, measured as
max |gpu - oracle| / max |oracle| over each plane (F, G) of the state.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads  # noqa: E402
from oracle import step1d  # noqa: E402
from oracle.model import Params  # noqa: E402

from parity import check, rel  # noqa: E402

pytestmark = pytest.mark.gpu

E = None


def setup_module(module):
    global E
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_15187_amd import evlb as _E
    E = _E


DEV = "cuda"


def td(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)




def oracle_tables(c, **kw):
    return step1d.Tables(Params(Q=c["Q"], dx=c["dx"], dt=c["dt"], **kw))


def solver(c, nx=None, **kw):
    return E.Solver(c["Q"], c["dx"], c["dt"], nx if nx is not None else c["nx"], **kw)


def nonequilibrium(F, G, tb, seed=3):
    rng = np.random.default_rng(seed)
    scale = tb.w[:, None] / tb.w.max()
    return F * (1 + 0.03 * rng.standard_normal(F.shape) * scale), G * (1 + 0.03 * rng.standard_normal(G.shape) * scale)


def case_phase():
    c, n, u, T = workloads.phase_separation_1d()
    return c, n, u, T


def case_slab(nx=1024):
    c, n, u, T = workloads.slab_1d(nx=nx)
    return c, n, u, T


def test_equilibrium_and_moments_match_oracle():
    for c, n, u, T in (case_phase(), case_slab()):
        print(f"case Q={c['Q']} nx={c['nx']}", flush=True)
        tb = oracle_tables(c)
        F, G = step1d.initial_state(n, u, T, tb)
        s = solver(c)
        f = s.equilibrium(td(n), td(u), td(T)).cpu().numpy()
        check(f, [F, G], 1e-13)
        Fn, Gn = nonequilibrium(F, G, tb)
        mom = s.moments(td(np.stack([Fn, Gn]))).cpu().numpy()
        ref = step1d.moments(Fn, Gn, tb)
        for i in range(4):
            assert np.max(np.abs(mom[i] - ref[i])) <= 1e-13 * np.max(np.abs(ref[i])) + 1e-16, i


@pytest.mark.parametrize("tile", [16, 63, 64])
@pytest.mark.parametrize("mask", [1, 2, 4, 8, 15])
@pytest.mark.parametrize("which", ["phase", "slab"])
def test_rhs_matches_oracle_per_term(mask, which, tile):
    c, n, u, T = case_phase() if which == "phase" else case_slab()
    print(f"rhs case {which} mask={mask} tile={tile}", flush=True)
    tb = oracle_tables(c, term_mask=mask)
    F, G = nonequilibrium(*step1d.initial_state(n, u + 0.02 * np.sin(np.arange(len(n)) / 7.0), T, tb), tb)
    LF, LG = step1d.rhs(F, G, tb)
    s = solver(c, term_mask=mask, tile_nodes=tile)
    L = s.rhs(td(np.stack([F, G]))).cpu().numpy()
    check(L, [LF, LG], 1e-11)


@pytest.mark.parametrize("tile", [16, 63, 64])
@pytest.mark.parametrize("mode", [1, 2])
def test_one_and_ten_steps_match_oracle(mode, tile):
    for c, n, u, T in (case_phase(), case_slab()):
        print(f"steps case Q={c['Q']} nx={c['nx']} mode={mode} tile={tile}", flush=True)
        tb = oracle_tables(c)
        F, G = step1d.initial_state(n, u, T, tb)
        s = solver(c, exec_mode=mode, tile_nodes=tile)
        f = s.equilibrium(td(n), td(u), td(T))
        s.step(f, 1)
        F1, G1 = step1d.rk3_step(F, G, tb)
        check(f.cpu().numpy(), [F1, G1], 1e-11)
        s.step(f, 9)
        F10, G10 = step1d.run(F1, G1, tb, 9)
        check(f.cpu().numpy(), [F10, G10], 1e-10)
        assert s.status() == 0


@pytest.mark.parametrize("tile", [16, 63, 64])
def test_q8_rhs_and_steps_match_oracle(tile):
    """Q = 8 (two wavefronts per narrow tile, two MFMA chains on one of them):
    the phase-separation state on its own 8-node velocity set."""
    c, n, u, T = case_phase()
    c = dict(c, Q=8)
    print(f"q8 case nx={c['nx']} tile={tile}", flush=True)
    tb = oracle_tables(c)
    F, G = nonequilibrium(*step1d.initial_state(n, u + 0.02 * np.sin(np.arange(len(n)) / 7.0), T, tb), tb)
    LF, LG = step1d.rhs(F, G, tb)
    s = solver(c, tile_nodes=tile)
    L = s.rhs(td(np.stack([F, G]))).cpu().numpy()
    check(L, [LF, LG], 1e-11)
    for mode in (1, 2):
        F0, G0 = step1d.initial_state(n, u, T, tb)
        s = solver(c, exec_mode=mode, tile_nodes=tile)
        f = s.equilibrium(td(n), td(u), td(T))
        s.step(f, 1)
        F1, G1 = step1d.rk3_step(F0, G0, tb)
        check(f.cpu().numpy(), [F1, G1], 1e-11)
        s.step(f, 9)
        F10, G10 = step1d.run(F1, G1, tb, 9)
        check(f.cpu().numpy(), [F10, G10], 1e-10)
        assert s.status() == 0


def _smooth_state(N):
    """Smooth periodic density, velocity and temperature waves on N nodes."""
    x = np.arange(N) / N
    n = 0.3 * (1 + 0.1 * np.sin(2 * np.pi * x) + 0.05 * np.cos(6 * np.pi * x))
    u = 0.04 * np.sin(4 * np.pi * x)
    T = 0.6 * (1 + 0.05 * np.cos(2 * np.pi * x))
    return n, u, T


# force_model: EV1 = 0 (eq:F1 convolution), EV2 = 1 (eq:F2 local stencil), none = 2
@pytest.mark.parametrize("tile", [16, 63, 64])
@pytest.mark.parametrize("force", [1, 2])
def test_ev2_and_no_force_match_oracle(force, tile):
    """The EV2 force of eq:F2 and the force-free model (with a uniform
    external force) on a ragged 300-node grid: right-hand side per term, and
    1 and 10 steps in both launch modes."""
    Q, N, dx = 16, 300, 1 / 8
    dt = 0.2 * dx / 6.630878198393129
    kw = dict(force_model=force, g_ext=0.02 if force == 2 else 0.0)
    n, u, T = _smooth_state(N)
    c = dict(Q=Q, dx=dx, dt=dt)
    print(f"force case force={force} tile={tile}", flush=True)
    for mask in (2, 15):
        tb = oracle_tables(c, term_mask=mask, **kw)
        F, G = nonequilibrium(*step1d.initial_state(n, u, T, tb), tb)
        LF, LG = step1d.rhs(F, G, tb)
        L = solver(c, nx=N, term_mask=mask, tile_nodes=tile, **kw).rhs(td(np.stack([F, G]))).cpu().numpy()
        check(L, [LF, LG], 1e-11, what=repr(mask))
    tb = oracle_tables(c, **kw)
    F0, G0 = step1d.initial_state(n, u, T, tb)
    F1, G1 = step1d.rk3_step(F0, G0, tb)
    F10, G10 = step1d.run(F1, G1, tb, 9)
    for mode in (1, 2):
        s = solver(c, nx=N, exec_mode=mode, tile_nodes=tile, **kw)
        f = s.equilibrium(td(n), td(u), td(T))
        s.step(f, 1)
        check(f.cpu().numpy(), [F1, G1], 1e-11, what=repr(mode))
        s.step(f, 9)
        check(f.cpu().numpy(), [F10, G10], 1e-10, what=repr(mode))
        assert s.status() == 0


@pytest.mark.parametrize("tile", [16, 63, 64])
@pytest.mark.parametrize("force", [0, 1])
def test_widest_windows_match_oracle(force, tile):
    """The widest windows the kernels are built for: sigma/dx = 16 (the
    averaging window of eq:nbar, 33 nodes) and, for EV1, r_cut/dx = 64 (the
    force window of eq:F1, 129 nodes) at dx = sigma/16 with r_cut = 4 sigma,
    on a ragged 300-node grid: right-hand side and 1 and 10 steps."""
    Q, N, dx = 16, 300, 1 / 16
    dt = 0.2 * dx / 6.630878198393129
    kw = dict(force_model=force, r_cut=4.0)
    n, u, T = _smooth_state(N)
    c = dict(Q=Q, dx=dx, dt=dt)
    print(f"window case force={force} tile={tile}", flush=True)
    tb = oracle_tables(c, **kw)
    F, G = nonequilibrium(*step1d.initial_state(n, u, T, tb), tb)
    LF, LG = step1d.rhs(F, G, tb)
    L = solver(c, nx=N, tile_nodes=tile, **kw).rhs(td(np.stack([F, G]))).cpu().numpy()
    check(L, [LF, LG], 1e-11)
    F0, G0 = step1d.initial_state(n, u, T, tb)
    F1, G1 = step1d.rk3_step(F0, G0, tb)
    F10, G10 = step1d.run(F1, G1, tb, 9)
    for mode in (1, 2):
        s = solver(c, nx=N, exec_mode=mode, tile_nodes=tile, **kw)
        f = s.equilibrium(td(n), td(u), td(T))
        s.step(f, 1)
        check(f.cpu().numpy(), [F1, G1], 1e-11, what=repr(mode))
        s.step(f, 9)
        check(f.cpu().numpy(), [F10, G10], 1e-10, what=repr(mode))
        assert s.status() == 0


@pytest.mark.parametrize("tile", [16, 63, 64])
def test_tiny_systems_batch_matches_oracle(tile):
    """Systems shorter than the force window (r_cut/dx = 40 nodes each way):
    the smallest accepted length (8) and a few others, in one ragged batch,
    so that the density window and the WENO halo wrap round their periodic
    system several times.  1 and 10 steps, both launch modes, against
    independent oracle runs."""
    Q, dx = 16, 1 / 8
    dt = 0.2 * dx / 6.630878198393129
    nxs = [8, 9, 13, 31, 64, 65, 130]
    c = dict(Q=Q, dx=dx, dt=dt)
    tb = oracle_tables(c)
    parts, refs = [], []
    for i, N in enumerate(nxs):
        x = np.arange(N) / N
        n = 0.3 * (1 + 0.05 * np.sin(2 * np.pi * x + i))
        u = 0.03 * np.cos(2 * np.pi * x)
        T = 0.6 + 0.02 * np.sin(2 * np.pi * x)
        parts.append((n, u, T))
        F, G = step1d.initial_state(n, u, T, tb)
        F1, G1 = step1d.rk3_step(F, G, tb)
        refs.append(((F1, G1), step1d.run(F1, G1, tb, 9)))
    cat = [np.concatenate([p[k] for p in parts]) for k in range(3)]
    offs = np.cumsum([0] + nxs)
    print(f"tiny systems tile={tile}", flush=True)
    for mode in (1, 2):
        s = solver(c, nx=nxs, exec_mode=mode, tile_nodes=tile)
        f = s.equilibrium(*[td(a) for a in cat])
        s.step(f, 1)
        got1 = f.cpu().numpy()
        s.step(f, 9)
        got10 = f.cpu().numpy()
        assert s.status() == 0
        for i in range(len(nxs)):
            sl = slice(offs[i], offs[i + 1])
            check(got1[:, :, sl], refs[i][0], 1e-11, what=repr((mode, nxs[i])))
            check(got10[:, :, sl], refs[i][1], 1e-10, what=repr((mode, nxs[i])))


def test_phase_separation_1000_steps_match_oracle():
    """Full phase-separation workload: 256 nodes, Q = 16, 1000 steps."""
    c, n, u, T = case_phase()
    tb = oracle_tables(c)
    F, G = step1d.initial_state(n, u, T, tb)
    F, G = step1d.run(F, G, tb, c["steps"])
    s = solver(c)
    f = s.equilibrium(td(n), td(u), td(T))
    s.step(f, c["steps"])
    err, rerr = check(f.cpu().numpy(), [F, G], 1e-8, row_tol=1e-8)
    print(f"1000-step rel err {err:.3e}, per row {rerr:.3e}", flush=True)
    assert s.status() == 0


def test_exec_modes_agree_and_repeat_bitwise():
    c, n, u, T = case_slab(2048)
    out = []
    for mode, tile in ((1, 64), (2, 64), (1, 64), (1, 16), (2, 16), (1, 63), (2, 63)):
        s = solver(c, exec_mode=mode, tile_nodes=tile)
        f = s.equilibrium(td(n), td(u), td(T))
        s.step(f, 20)
        out.append(f.cpu().numpy())
    assert np.array_equal(out[0], out[2])
    for o in out[1:]:
        check(o, out[0], 1e-14)


def test_ragged_batch_matches_independent_oracle_runs():
    """Several periodic systems of uneven length in one state."""
    c, systems = workloads.batched_sweep_1d(n_sys=5, nx_max=700)
    nxs = c["nx_list"]
    tb = oracle_tables(c)
    n = np.concatenate([s[0] for s in systems])
    u = np.concatenate([s[1] for s in systems])
    T = np.concatenate([s[2] for s in systems])
    for mode, tile in ((1, 64), (2, 64), (1, 16), (2, 16), (1, 63), (2, 63)):
        s = solver(c, nx=nxs, exec_mode=mode, tile_nodes=tile)
        f = s.equilibrium(td(n), td(u), td(T))
        s.step(f, 5)
        got = f.cpu().numpy()
        off = 0
        for (ni, ui, Ti), nx in zip(systems, nxs):
            F, G = step1d.initial_state(ni, ui, Ti, tb)
            F, G = step1d.run(F, G, tb, 5)
            check(got[:, :, off:off + nx], [F, G], 1e-11, what=repr((mode, nx)))
            off += nx


def test_uniform_state_stationary_on_gpu():
    c, n, u, T = case_phase()
    s = solver(c)
    nn = np.full(c["nx"], 0.3)
    f = s.equilibrium(td(nn), td(0 * nn), td(0 * nn + 0.6))
    f0 = f.clone()
    s.step(f, 1000)
    assert (f - f0).abs().max().item() <= 1e-14 * f0.abs().max().item()


def test_conservation_on_gpu():
    c, n, u, T = case_slab(4096)
    s = solver(c)
    f = s.equilibrium(td(n), td(u), td(T))
    v = torch.tensor(s.velocities, dtype=torch.float64, device=DEV)[:, None]
    m0 = f[0].sum().item()
    scale = (v.abs() * f[0]).sum().item()
    s.step(f, 500)
    assert abs(f[0].sum().item() - m0) < 1e-13 * m0
    assert abs((v * f[0]).sum().item()) < 1e-13 * scale
    assert s.status() == 0


def test_slab_full_size_ten_steps_match_oracle():
    """Slab-evaporation workload at full size (4096 nodes, Q = 24)."""
    c, n, u, T = workloads.slab_1d()
    tb = oracle_tables(c)
    F, G = step1d.initial_state(n, u, T, tb)
    F, G = step1d.run(F, G, tb, 10)
    s = solver(c)
    f = s.equilibrium(td(n), td(u), td(T))
    s.step(f, 10)
    check(f.cpu().numpy(), [F, G], 1e-10)


@pytest.mark.timeout(900)
def test_slab_full_size_1000_steps_match_oracle():
    """Slab-evaporation workload at full size (4096 nodes, Q = 24, the
    bench's launch shape) over 1000 steps against the oracle: 1e-8."""
    c, n, u, T = workloads.slab_1d()
    tb = oracle_tables(c)
    F, G = step1d.initial_state(n, u, T, tb)
    F, G = step1d.run(F, G, tb, 1000)
    s = solver(c)
    f = s.equilibrium(td(n), td(u), td(T))
    s.step(f, 1000)
    err, rerr = check(f.cpu().numpy(), [F, G], 1e-8, row_tol=1e-8)
    print(f"slab 1000-step rel err {err:.3e}, per row {rerr:.3e}", flush=True)
    assert s.status() == 0


@pytest.mark.timeout(900)
def test_adjoint_workload_forward_1000_steps_match_oracle():
    """The adjoint workload's forward step at its own parameters (2048
    nodes, dx = sigma/4, Q = 16, slab at T = 0.85 T_c) over 1000 steps."""
    c, n, u, T = workloads.slab_1d(name="adjoint_slab_1d")
    tb = oracle_tables(c)
    F, G = step1d.initial_state(n, u, T, tb)
    F, G = step1d.run(F, G, tb, 1000)
    s = solver(c)
    f = s.equilibrium(td(n), td(u), td(T))
    s.step(f, 1000)
    err, rerr = check(f.cpu().numpy(), [F, G], 1e-8, row_tol=1e-8)
    print(f"adjoint-slab 1000-step rel err {err:.3e}, per row {rerr:.3e}", flush=True)
    assert s.status() == 0


@pytest.mark.parametrize("force", [0, 1])
@pytest.mark.parametrize("which", ["sec3b", "sec3c"])
def test_paper_parameter_runs_match_oracle(which, force):
    """The paper's own numerical parameters (Sec. III: dx = sigma/10,
    dt = 5e-3, Q = 16, r_cut/dx = 50) on its own initial states: the four
    phase-separation runs of eq:rho_init_takata (Sec. III B) or the four
    evaporating slabs of eq:tan (Sec. III C), as one batch, EV1 or EV2;
    1 and 20 steps against independent oracle runs."""
    c, systems = workloads.paper_sec3b() if which == "sec3b" else workloads.paper_sec3c()
    print(f"paper parameters {which} force={force}", flush=True)
    nxs = [len(x[0]) for x in systems]
    tb = oracle_tables(c, force_model=force)
    s = solver(c, nx=nxs, force_model=force)
    f = s.equilibrium(*[td(np.concatenate([x[k] for x in systems])) for k in range(3)])
    s.step(f, 1)
    got1 = f.cpu().numpy()
    s.step(f, 19)
    got20 = f.cpu().numpy()
    assert s.status() == 0
    offs = np.cumsum([0] + nxs)
    for i, (n, u, T) in enumerate(systems):
        F, G = step1d.initial_state(n, u, T, tb)
        F1, G1 = step1d.rk3_step(F, G, tb)
        F20, G20 = step1d.run(F1, G1, tb, 19)
        sl = slice(offs[i], offs[i + 1])
        check(got1[:, :, sl], [F1, G1], 1e-11, what=repr((which, i)))
        check(got20[:, :, sl], [F20, G20], 1e-11, steps=20, what=repr((which, i)))


def _ev1_ev2_density_gap(which, steps):
    """Runs the paper's Sec. III B or III C batch with the EV1 and with the
    EV2 force; returns max|n_EV1 - n_EV2| / max n_EV1 per run."""
    c, systems = workloads.paper_sec3b() if which == "sec3b" else workloads.paper_sec3c()
    nxs = [len(x[0]) for x in systems]
    cat = [td(np.concatenate([x[k] for x in systems])) for k in range(3)]
    dens = []
    for force in (0, 1):
        s = solver(c, nx=nxs, force_model=force)
        f = s.equilibrium(*cat)
        s.step(f, steps)
        assert s.status() == 0
        dens.append(s.moments(f)[0].cpu().numpy())
    offs = np.cumsum([0] + nxs)
    gap = []
    for i in range(len(nxs)):
        a, b = dens[0][offs[i]:offs[i + 1]], dens[1][offs[i]:offs[i + 1]]
        gap.append(np.max(np.abs(a - b)) / np.max(a))
    return c, np.array(gap)


def test_ev1_and_ev2_agree_on_smooth_profiles():
    """Sec. III B reports that the EV1 (eq:F1) and EV2 (eq:F2) forces give
    matching profiles at t = 100 from the sinusoidal state of
    eq:rho_init_takata, for the lowest and the highest temperature, because
    the density gradients stay small; Sec. III C that on the evaporating slab
    they agree at T = 0.74 and that EV2 departs at the lowest temperature,
    where the interface is sharpest.  Both batches run with each force at the
    paper's parameters (Sec. III B to t = 100, 20000 steps; Sec. III C to
    t = 75, 15000 steps).  Bars: the paper's figures show the two curves
    overlapping at plot resolution, taken as 3% of the largest density; the
    gap must shrink as T rises towards T_c (smoother profiles), and on the
    slab be larger at T = 0.6 than at T = 0.74.  Part of every gap is not
    the gradient expansion: EV1's kernel is truncated at r_cut = 5 sigma, so
    its attraction parameter is 0.4% below the untruncated a = 4 pi / 3 that
    EV2 uses."""
    c, gap_b = _ev1_ev2_density_gap("sec3b", 20000)
    temps_b = [p[0] for p in c["pairs"]]
    c, gap_c = _ev1_ev2_density_gap("sec3c", 15000)
    temps_c = c["T"]
    print("Sec. III B t = 100, EV1-EV2 density gap by T:",
          ", ".join(f"{t}: {g:.2e}" for t, g in zip(temps_b, gap_b)), flush=True)
    print("Sec. III C t = 75, EV1-EV2 density gap by T:",
          ", ".join(f"{t}: {g:.2e}" for t, g in zip(temps_c, gap_c)), flush=True)
    assert np.all(gap_b < 3e-2)
    order = np.argsort(temps_b)
    assert np.all(np.diff(gap_b[order]) < 0)          # smaller gap at higher T
    assert gap_c[int(np.argmin(temps_c))] > gap_c[int(np.argmax(temps_c))]
    assert gap_c[int(np.argmax(temps_c))] < 3e-2


def test_nonfinite_state_is_reported():
    c, n, u, T = case_phase()
    s = solver(c)
    f = s.equilibrium(td(n), td(u), td(T))
    f[0, :, 17] = float("nan")
    s.step(f, 1)
    assert s.status() == E.EVLB_ENONFINITE
    assert s.status() == 0   # latch cleared
