"""Isothermal mode (Sec. III A: the fluid temperature is kept constant).

Parity of the HIP path with the oracle's isothermal mode (1D right-hand
side per term and 10 steps, 2D right-hand side and one step), and the
stationary planar interfaces of Sec. III A at the paper's own parameters:
five temperatures T in {0.55, 0.6, 0.65, 0.7, 0.74}, the domain
[-100 sigma, 100 sigma] at dx = sigma/10, Q = 16, dt = 5e-3, the tanh
profile of eq:tanh with x0 = 50 sigma at the Maxwell densities.  After 1e5
steps (t = 500; the paper runs 1e6) the bulk densities lie on the Maxwell
construction of eq:EOSS (Fig. 2) to 1e-3 in n sigma^3; a is the discrete
kernel's attraction parameter at dx = sigma/10.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads  # noqa: E402
from oracle import model, step1d, step2d  # noqa: E402
from oracle.model import Params  # noqa: E402

pytestmark = pytest.mark.gpu

E = None


def setup_module(module):
    global E
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_15187_amd import evlb as _E
    E = _E


def td(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def rel(got, ref):
    return max(np.max(np.abs(got[i] - ref[i])) / np.max(np.abs(ref[i])) for i in range(2))


def _state_1d(T_iso):
    c, n, u, T = workloads.phase_separation_1d()
    x = np.arange(c["nx"]) / c["nx"]
    u = 0.05 * np.sin(2 * np.pi * x)
    T = T * (1 + 0.05 * np.cos(2 * np.pi * x))  # moment temperature away from T_iso
    tb = step1d.Tables(Params(Q=16, dx=c["dx"], dt=c["dt"], T_iso=T_iso))
    F, G = step1d.initial_state(n, u, T, tb)
    rng = np.random.default_rng(9)
    scale = tb.w[:, None] / tb.w.max()
    return c, tb, F * (1 + 0.02 * rng.standard_normal(F.shape) * scale), G


@pytest.mark.parametrize("mask", [4, 8, 15])
def test_isothermal_rhs_1d(mask):
    T_iso = 0.55
    c, tb, F, G = _state_1d(T_iso)
    tb = step1d.Tables(Params(Q=16, dx=c["dx"], dt=c["dt"], T_iso=T_iso, term_mask=mask))
    LF, LG = step1d.rhs(F, G, tb)
    s = E.Solver(16, c["dx"], c["dt"], c["nx"], T_iso=T_iso, term_mask=mask)
    L = s.rhs(td(np.stack([F, G]))).cpu().numpy()
    assert rel(L, [LF, LG]) < 1e-11


@pytest.mark.parametrize("tile", [16, 63])
def test_isothermal_steps_1d(tile):
    T_iso = 0.55
    c, tb, F, G = _state_1d(T_iso)
    Fo, Go = step1d.run(F, G, tb, 10)
    s = E.Solver(16, c["dx"], c["dt"], c["nx"], T_iso=T_iso, exec_mode=1, tile_nodes=tile)
    f = td(np.stack([F, G]))
    s.step(f, 10)
    assert s.status() == E.EVLB_OK
    assert rel(f.cpu().numpy(), [Fo, Go]) < 1e-10


def test_isothermal_2d_rhs_and_step():
    T_iso = 0.55
    c, n, ux, uy, T = workloads.phase_separation_2d(nx=40, ny=24)
    yy, xx = np.meshgrid(np.arange(24), np.arange(40), indexing="ij")
    ux = 0.03 * np.sin(2 * np.pi * xx / 40)
    T = T * (1 + 0.03 * np.cos(2 * np.pi * yy / 24))
    tb = step2d.Tables2D(Params(Q=16, dx=c["dx"], dt=c["dt"], T_iso=T_iso))
    F, G = step2d.initial_state(n, ux, uy, T, tb)
    LF, LG = step2d.rhs(F, G, tb)
    s = E.Solver(16, c["dx"], c["dt"], 40, ny=24, T_iso=T_iso)
    L = s.rhs(td(np.stack([F, G]))).cpu().numpy()
    assert rel(L, [LF, LG]) < 1e-11
    Fo, Go = step2d.rk3_step(F, G, tb)
    f = td(np.stack([F, G]))
    s.step(f, 1)
    assert rel(f.cpu().numpy(), [Fo, Go]) < 1e-11


TEMPS = (0.55, 0.6, 0.65, 0.7, 0.74)
STEPS_3A = 100000


def test_stationary_interfaces_sec3a_on_maxwell_construction():
    dx, dt, nx, x0 = 0.1, 5e-3, 2000, 50.0
    a = model.attraction_parameter_discrete(Params(Q=16, dx=dx, dt=dt))
    Tc = model.critical_point(a)[1]
    x = workloads.grid(nx, dx)
    for T in TEMPS:
        nv, nl = model.maxwell_construction(T, a)
        xi = np.sqrt(3.0 / (4 * np.pi * np.sqrt(3) * (Tc - T)))
        n = nl + (nv - nl) / 2 * (1 + np.tanh((np.abs(x) - x0) / xi))
        s = E.Solver(16, dx, dt, nx, T_iso=T)
        f = s.equilibrium(td(n), td(np.zeros(nx)), td(np.full(nx, T)))
        for _ in range(4):
            s.step(f, STEPS_3A // 4)
        assert s.status() == E.EVLB_OK
        mom = s.moments(f).cpu().numpy()
        print(f"T {T}: n_l {mom[0][nx // 2]:.6f} (Maxwell {nl:.6f})  n_v {mom[0][0]:.6f} (Maxwell {nv:.6f})",
              flush=True)
        assert abs(mom[0][nx // 2] - nl) < 1e-3, (T, mom[0][nx // 2], nl)
        assert abs(mom[0][0] - nv) < 1e-3, (T, mom[0][0], nv)
