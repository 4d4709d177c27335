"""Parity of the 2D HIP path (dim = 2, through the C ABI) with the 2D oracle.

Tolerance as in 1D: FP64 on both sides, differing only in summation order
(the disc sums, the Dp contractions on the matrix cores, the WENO-5 weights'
common denominator), so one right-hand side or one step agrees to 1e-11
relative, max |gpu - oracle| / max |oracle| over each plane family (F, G).

Full size (1024 x 1024, the 2D phase-separation workload): the oracle runs
on windows cut from the periodic domain.  Every operation of a stage reaches
at most r_cut/dx = 20 nodes (the force), so a window with a margin of 24
nodes reproduces the right-hand side of its centre exactly, and a margin of
64 nodes the whole three-stage step.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads  # noqa: E402
from oracle import step2d  # noqa: E402
from oracle.model import Params, TERM_ADV, TERM_FORCE, TERM_J0, TERM_J1, FORCE_NONE  # noqa: E402

from parity import check, rel  # noqa: E402

pytestmark = pytest.mark.gpu

E = None
DEV = "cuda"


def setup_module(module):
    global E
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_15187_amd import evlb as _E
    E = _E


def td(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def tstate(F, G):
    """The node-major device state of the oracle's planes F, G (q, q, ny, nx)."""
    return E.Solver.from_planes(td(np.stack([F, G])))


def planes(f):
    """A device state or right-hand side as host planes (2, q, q, ny, nx)."""
    return E.Solver.planes(f).cpu().numpy()




def tables(c, **kw):
    return step2d.Tables2D(Params(Q=16, dx=c["dx"], dt=c["dt"], **kw))


def solver(c, nx, ny, **kw):
    return E.Solver(16, c["dx"], c["dt"], nx, ny=ny, **kw)


def perturbation_at(yi, xi):
    """Deterministic non-equilibrium factor
    1 + 0.03 w_k w_l / w_max^2 sin(0.37 x + 0.61 y + 1.3 k + 0.7 l + 2.1 d)
    at node indices (yi, xi); perturbation_torch evaluates the same
    expression on the device for full-size states."""
    from oracle.quadrature import gauss_hermite
    w = gauss_hermite(16)[1]
    wn = w / w.max()
    d = np.arange(2)[:, None, None, None, None]
    k = np.arange(16)[None, :, None, None, None]
    l = np.arange(16)[None, None, :, None, None]
    y = np.asarray(yi, dtype=np.float64)[None, None, None, :, None]
    x = np.asarray(xi, dtype=np.float64)[None, None, None, None, :]
    s = np.sin(0.37 * x + 0.61 * y + 1.3 * k + 0.7 * l + 2.1 * d)
    return 1.0 + 0.03 * wn[k] * wn[l] * s


def perturbation(shape):
    return perturbation_at(np.arange(shape[0]), np.arange(shape[1]))


def perturbation_torch(ny, nx):
    from oracle.quadrature import gauss_hermite
    w = gauss_hermite(16)[1]
    wn = torch.tensor(w / w.max(), dtype=torch.float64, device=DEV)
    d = torch.arange(2, device=DEV, dtype=torch.float64)[:, None, None, None, None]
    kk = torch.arange(16, device=DEV)
    k = kk.to(torch.float64)[None, :, None, None, None]
    l = kk.to(torch.float64)[None, None, :, None, None]
    y = torch.arange(ny, device=DEV, dtype=torch.float64)[None, None, None, :, None]
    x = torch.arange(nx, device=DEV, dtype=torch.float64)[None, None, None, None, :]
    s = torch.sin(0.37 * x + 0.61 * y + 1.3 * k + 0.7 * l + 2.1 * d)
    return 1.0 + 0.03 * wn[kk][None, :, None, None, None] * wn[kk][None, None, :, None, None] * s


def small_case(nx, ny, seed=None):
    c, n, ux, uy, T = workloads.phase_separation_2d(nx=nx, ny=ny, seed=seed)
    # a weak flow so that every J1 and Shakhov term is exercised
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ux = 0.03 * np.sin(2 * np.pi * xx / nx) * np.cos(2 * np.pi * yy / ny)
    uy = -0.02 * np.cos(2 * np.pi * 2 * xx / nx)
    T = T * (1 + 0.02 * np.sin(2 * np.pi * yy / ny))
    return c, n, ux, uy, T


def oracle_state(c, n, ux, uy, T, tb, perturb=True):
    F, G = step2d.initial_state(n, ux, uy, T, tb)
    if perturb:
        P = perturbation(n.shape)
        F, G = F * P[0], G * P[1]
    return F, G


def test_equilibrium_and_moments_2d():
    c, n, ux, uy, T = small_case(40, 24)
    tb = tables(c)
    F, G = step2d.initial_state(n, ux, uy, T, tb)
    s = solver(c, 40, 24)
    f = planes(s.equilibrium(td(n), td(np.stack([ux, uy])), td(T)))
    check(f, [F, G], 1e-13)
    Fp, Gp = oracle_state(c, n, ux, uy, T, tb)
    mom = s.moments(tstate(Fp, Gp)).cpu().numpy()
    ref = step2d.moments(Fp, Gp, tb)
    for i in range(6):
        assert np.max(np.abs(mom[i] - ref[i].ravel())) <= 1e-13 * np.max(np.abs(ref[i])) + 1e-16, i


@pytest.mark.parametrize("mask", [TERM_ADV, TERM_FORCE, TERM_J0, TERM_J1, 15])
@pytest.mark.parametrize("nx,ny", [(72, 40), (24, 8)])
def test_rhs_terms_2d(mask, nx, ny):
    """Each term alone and all together; (72, 40) has ragged tiles in every
    kernel, (24, 8) is narrower than one tile and the smallest ny."""
    print(f"rhs mask={mask} nx={nx} ny={ny}", flush=True)
    c, n, ux, uy, T = small_case(nx, ny)
    kw = dict(term_mask=mask, g_ext=0.01 if mask == TERM_FORCE else 0.0)
    tb = tables(c, **kw)
    F, G = oracle_state(c, n, ux, uy, T, tb)
    LF, LG = step2d.rhs(F, G, tb)
    s = solver(c, nx, ny, **kw)
    L = planes(s.rhs(tstate(F, G)))
    check(L, [LF, LG], 1e-11)


def test_rhs_force_model_none_2d():
    c, n, ux, uy, T = small_case(40, 16)
    kw = dict(force_model=FORCE_NONE, g_ext=0.02)
    tb = tables(c, **kw)
    F, G = oracle_state(c, n, ux, uy, T, tb)
    LF, LG = step2d.rhs(F, G, tb)
    L = planes(solver(c, 40, 16, force_model=2, g_ext=0.02).rhs(tstate(F, G)))
    check(L, [LF, LG], 1e-11)


@pytest.mark.timeout(900)
def test_100_steps_2d_small_periodic_grid():
    """100 steps on a 24 x 20 periodic grid (shorter than the force
    window, so the density and force windows wrap several times; ragged in
    x against the 16-column strips) against the oracle."""
    nx, ny, nsteps = 24, 20, 100
    c, n, ux, uy, T = small_case(nx, ny)
    tb = tables(c)
    F, G = oracle_state(c, n, ux, uy, T, tb)
    Fo, Go = step2d.run(F, G, tb, nsteps)
    s = solver(c, nx, ny)
    f = tstate(F, G)
    s.step(f, nsteps)
    assert s.status() == E.EVLB_OK
    err, rerr = check(planes(f), [Fo, Go], 1e-11, steps=nsteps)
    print(f"2D 100-step rel err {err:.3e}, per row {rerr:.3e}", flush=True)


@pytest.mark.parametrize("nsteps", [1, 4])
def test_steps_2d(nsteps):
    nx, ny = 72, 40
    print(f"steps={nsteps}", flush=True)
    c, n, ux, uy, T = small_case(nx, ny)
    tb = tables(c)
    F, G = oracle_state(c, n, ux, uy, T, tb)
    Fo, Go = step2d.run(F, G, tb, nsteps)
    s = solver(c, nx, ny)
    f = tstate(F, G)
    s.step(f, nsteps)
    assert s.status() == E.EVLB_OK
    check(planes(f), [Fo, Go], 1e-11, steps=nsteps)


@pytest.mark.parametrize("nx,ny,nsteps", [(37, 53, 2), (9, 8, 3)])
def test_steps_2d_ragged_strips_and_segments(nx, ny, nsteps):
    """Grids that the fused stage's 8-column strips and row segments do not
    divide: 37 x 53 has a last strip of 5 columns and three row segments of
    18, 18 and 17 rows; 9 x 8 has a strip of one column whose halo wraps
    onto itself, at the smallest ny.  Right-hand side and steps against the
    oracle."""
    print(f"ragged 2d nx={nx} ny={ny} steps={nsteps}", flush=True)
    c, n, ux, uy, T = small_case(nx, ny)
    tb = tables(c)
    F, G = oracle_state(c, n, ux, uy, T, tb)
    s = solver(c, nx, ny)
    LF, LG = step2d.rhs(F, G, tb)
    check(planes(s.rhs(tstate(F, G))), [LF, LG], 1e-11, what="rhs")
    Fo, Go = step2d.run(F, G, tb, nsteps)
    f = tstate(F, G)
    s.step(f, nsteps)
    assert s.status() == E.EVLB_OK
    check(planes(f), [Fo, Go], 1e-11, steps=nsteps, what="steps")


def test_uniform_state_stationary_2d():
    c, n, ux, uy, T = workloads.phase_separation_2d(nx=48, ny=32)
    s = solver(c, 48, 32)
    f = s.equilibrium(td(np.full((32, 48), 0.3)), td(np.zeros((2, 32, 48))), td(np.full((32, 48), c["T"])))
    f0 = f.clone()
    s.step(f, 20)
    assert torch.max(torch.abs(f - f0)).item() <= 1e-14 * torch.max(f0).item()


def test_conservation_2d():
    """Mass and both momentum components conserved over 10 steps."""
    c, n, ux, uy, T = small_case(64, 48)
    tb = tables(c)
    F, G = oracle_state(c, n, ux, uy, T, tb)
    s = solver(c, 64, 48)
    f = tstate(F, G)
    fp = E.Solver.planes(f)  # a view: follows the steps
    v = torch.tensor(tb.v, dtype=torch.float64, device=DEV)
    mass0 = fp[0].sum().item()
    px0 = (v[:, None, None, None] * fp[0]).sum().item()
    py0 = (v[None, :, None, None] * fp[0]).sum().item()
    scale = (v.abs()[:, None, None, None] * fp[0]).sum().item()
    s.step(f, 10)
    assert abs(fp[0].sum().item() - mass0) < 1e-13 * mass0
    assert abs((v[:, None, None, None] * fp[0]).sum().item() - px0) < 1e-13 * scale
    assert abs((v[None, :, None, None] * fp[0]).sum().item() - py0) < 1e-13 * scale


def test_nonfinite_status_2d():
    c, n, ux, uy, T = small_case(32, 16)
    s = solver(c, 32, 16)
    f = s.equilibrium(td(n), td(np.stack([ux, uy])), td(T))
    f[0, 3, 5] = -1.0  # every velocity of F at node (y, x) = (3, 5)
    s.step(f, 1)
    assert s.status() == E.EVLB_ENONFINITE
    assert s.status() == E.EVLB_OK  # cleared


def _window(a, y0, x0, h, w):
    ny, nx = a.shape[-2:]
    yi = (y0 + np.arange(h)) % ny
    xi = (x0 + np.arange(w)) % nx
    return a[..., yi[:, None], xi[None, :]]


@pytest.fixture(scope="module")
def full_state():
    """The 1024 x 1024 workload on the device with the non-equilibrium
    factor, and its node fields on the host."""
    c, n, ux, uy, T = workloads.phase_separation_2d()
    s = solver(c, c["nx"], c["ny"])
    f = s.equilibrium(td(n), td(np.stack([ux, uy])), td(T))
    f.mul_(E.Solver.from_planes(perturbation_torch(c["ny"], c["nx"])))
    return c, n, ux, uy, T, s, f


SAMPLES = [(0, 0), (517, 300), (1000, 1010)]


def test_full_size_rhs_sampled(full_state):
    c, n, ux, uy, T, s, f = full_state
    print("full-size rhs", flush=True)
    L = s.rhs(f)
    tb = tables(c)
    m, b = 24, 16
    for (yc, xc) in SAMPLES:
        y0, x0 = yc - m, xc - m
        h = w = b + 2 * m
        Fw, Gw = step2d.initial_state(_window(n, y0, x0, h, w), _window(ux, y0, x0, h, w),
                                      _window(uy, y0, x0, h, w), _window(T, y0, x0, h, w), tb)
        yi = (y0 + np.arange(h)) % c["ny"]
        xi = (x0 + np.arange(w)) % c["nx"]
        P = perturbation_at(yi, xi)
        LF, LG = step2d.rhs(Fw * P[0], Gw * P[1], tb)
        cy = slice(m, m + b)
        ys = torch.tensor((yc + np.arange(b)) % c["ny"], device=DEV)
        xs = torch.tensor((xc + np.arange(b)) % c["nx"], device=DEV)
        got = E.Solver.planes(L).index_select(3, ys).index_select(4, xs).cpu().numpy()
        check(got, [LF[:, :, cy, cy], LG[:, :, cy, cy]], 1e-11, what=repr((yc, xc)))


def test_full_size_step_sampled(full_state):
    """One full-size step (the launch sequence the bench times), checked on
    a 16 x 16 block against the oracle on a window with a 64-node margin."""
    c, n, ux, uy, T, s, f = full_state
    print("full-size step", flush=True)
    g = f.clone()
    s.step(g, 1)
    assert s.status() == E.EVLB_OK
    tb = tables(c)
    m, b = 64, 16
    yc, xc = 700, 130
    y0, x0 = yc - m, xc - m
    h = w = b + 2 * m
    yi = (y0 + np.arange(h)) % c["ny"]
    xi = (x0 + np.arange(w)) % c["nx"]
    Fw, Gw = step2d.initial_state(_window(n, y0, x0, h, w), _window(ux, y0, x0, h, w),
                                  _window(uy, y0, x0, h, w), _window(T, y0, x0, h, w), tb)
    P = perturbation_at(yi, xi)
    Fo, Go = step2d.rk3_step(Fw * P[0], Gw * P[1], tb)
    got = E.Solver.planes(g)[:, :, :, yc:yc + b, xc:xc + b].cpu().numpy()
    check(got, [Fo[:, :, m:m + b, m:m + b], Go[:, :, m:m + b, m:m + b]], 1e-11)
