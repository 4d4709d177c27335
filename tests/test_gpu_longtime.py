"""Long-time pin (P15): bulk coexistence densities against the Maxwell
construction of the equation of state.

Sec. III A runs stationary planar interfaces for a long time and finds the
bulk liquid and vapour densities on the Maxwell construction of eq:EOSS
(Fig. 2).  Here four periodic 64 sigma systems (dx = sigma/8, Q = 16) start
from the tanh profile of eq:tanh at the Maxwell densities of T/T_c = 0.6,
0.7, 0.8, 0.9 (T_c and a of the discrete kernel) and run 2e5 thermal TVD-RK3
steps in one batched launch sequence.  The fluid is thermal, so the
interface settles at a slightly different temperature; the densities at the
centres of the two bulk phases are compared with the Maxwell construction at
the final mean temperature, to 1e-3 in n sigma^3.  The oracle is far too slow
for 2e5 steps; the equation of state and the Maxwell construction come from
it.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads  # noqa: E402
from oracle import model  # noqa: E402

pytestmark = pytest.mark.gpu

NX, X0, STEPS = 512, 16.0, 200000
TR = (0.6, 0.7, 0.8, 0.9)


def test_long_time_coexistence_matches_maxwell_construction():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_15187_amd import evlb as E
    c = workloads.constants()["phase_separation_1d"]
    a, Tc, dx, dt = c["a_disc"], c["Tc_disc"], c["dx"], c["dt"]
    x = workloads.grid(NX, dx)
    ns, Ts = [], []
    for tr in TR:
        T = tr * Tc
        nv, nl = model.maxwell_construction(T, a)
        xi = np.sqrt(3.0 / (4 * np.pi * np.sqrt(3) * (Tc - T)))
        ns.append(nl + (nv - nl) / 2 * (1 + np.tanh((np.abs(x) - X0) / xi)))
        Ts.append(np.full(NX, T))
    td = lambda v: torch.tensor(np.concatenate(v), dtype=torch.float64, device="cuda")
    s = E.Solver(16, dx, dt, [NX] * len(TR))
    f = s.equilibrium(td(ns), td([np.zeros(NX)] * len(TR)), td(Ts))
    for _ in range(4):
        s.step(f, STEPS // 4)
        print("steps", flush=True)
    assert s.status() == E.EVLB_OK
    mom = s.moments(f).cpu().numpy()
    for i, tr in enumerate(TR):
        sl = slice(i * NX, (i + 1) * NX)
        n, T = mom[0, sl], mom[2, sl]
        Tm = T.mean()
        assert T.max() - T.min() < 5e-3, (tr, T.min(), T.max())
        nv, nl = model.maxwell_construction(Tm, a)
        print(f"T/Tc {tr}: T {Tm:.6f}  n_l {n[NX // 2]:.6f} (Maxwell {nl:.6f})  n_v {n[0]:.6f} (Maxwell {nv:.6f})",
              flush=True)
        assert abs(n[NX // 2] - nl) < 1e-3, (tr, n[NX // 2], nl)
        assert abs(n[0] - nv) < 1e-3, (tr, n[0], nv)
