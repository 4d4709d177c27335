"""Write workloads/constants.json: the derived constants of the synthetic
workloads (temperatures from T/T_c, coexistence densities, time steps).

Every number comes from the CPU oracle (equation of state eq:EOSS with the
discrete kernel's attraction parameter, Maxwell construction, Gauss-Hermite
nodes), so that neither the oracle's inputs nor its expected values ever
come from the HIP path.  Run:  python tests/golden/make_workload_constants.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import model, step2d  # noqa: E402
from oracle.quadrature import gauss_hermite  # noqa: E402


def tc_disc(dx):
    a = model.attraction_parameter_discrete(model.Params(Q=16, dx=dx, dt=1.0))
    return a, model.critical_point(a)[1]


def main():
    vmax = {Q: float(gauss_hermite(Q)[0][-1]) for Q in (16, 24)}
    a8, tc8 = tc_disc(1 / 8)
    a4, tc4 = tc_disc(1 / 4)
    out = {"_doc": "derived by tests/golden/make_workload_constants.py from the CPU oracle"}

    T1 = 0.7 * tc8
    out["phase_separation_1d"] = dict(
        Q=16, dx=0.125, nx=256, T=T1, n0=0.25, noise=0.01, steps=1000, seed=2503152,
        dt=0.2 * 0.125 / vmax[16], a_disc=a8, Tc_disc=tc8)

    T2 = 0.8 * tc8
    nv2, nl2 = model.maxwell_construction(T2, a8)
    out["slab_evaporation_1d"] = dict(
        Q=24, dx=0.125, nx=4096, T=T2, n_l=nl2, n_v=nv2, x0=32.0, width=2.0, steps=20000,
        dt=0.2 * 0.125 / vmax[24], a_disc=a8, Tc_disc=tc8)

    out["batched_sweep_1d"] = dict(
        Q=16, dx=0.125, n_sys=512, nx_min=256, nx_max=8192, t_over_tc=[0.6, 0.95],
        n0=[0.15, 0.35], noise=0.01, steps=5000, seed=2503155,
        dt=0.2 * 0.125 / vmax[16], a_disc=a8, Tc_disc=tc8)

    # 2D: attraction parameter of the cell-centre disc kernel at dx = sigma/4
    a2d = step2d.attraction_parameter_2d(step2d.Tables2D(model.Params(Q=16, dx=0.25, dt=1.0)))
    tc2d = model.critical_point(a2d)[1]
    out["phase_separation_2d"] = dict(
        Q=16, dx=0.25, nx=1024, ny=1024, T=0.75 * tc2d, n0=0.3, noise=0.01, steps=2000, seed=2503154,
        dt=0.2 * 0.25 / vmax[16], a_disc=a2d, Tc_disc=tc2d)

    # the paper's own runs (Sec. III B and III C): dx = sigma/10, dt = 5e-3,
    # Q = 16, absolute temperatures, a of the discrete kernel at sigma/10
    a10, tc10 = tc_disc(0.1)
    pairs = [[0.7, 0.4], [0.65, 0.55], [0.6, 0.65], [0.55, 0.7]]
    amp = []
    for T, _ in pairs:
        nv, nl = model.maxwell_construction(T, a10)
        amp.append(0.5 * (nl + nv))
    out["paper_sec3b_phase_separation"] = dict(
        Q=16, dx=0.1, dt=5e-3, L=100.0, nx=1000, pairs=pairs, A=amp, t_end=5000.0, steps=1000000,
        a_disc=a10, Tc_disc=tc10, table1_ev1_s=1.8e4, table1_ev2_s=6e3)
    temps = [0.6, 0.65, 0.7, 0.74]
    coex = [list(model.maxwell_construction(T, a10)) for T in temps]
    out["paper_sec3c_evaporation"] = dict(
        Q=16, dx=0.1, dt=5e-3, nx=4000, x0=25.0, width=2.0, T=temps, n_v=[c[0] for c in coex],
        n_l=[c[1] for c in coex], t_end=75.0, steps=15000, a_disc=a10, Tc_disc=tc10,
        table1_ev1_s=3.4e3, table1_ev2_s=9e2)

    T5 = 0.85 * tc4
    nv5, nl5 = model.maxwell_construction(T5, a4)
    out["adjoint_slab_1d"] = dict(
        Q=16, dx=0.25, nx=2048, T=T5, n_l=nl5, n_v=nv5, x0=32.0, width=2.0, steps=2000,
        x_flux=128.0, target_seed=2503156, target_modes=8, target_amp=0.01,
        dt=0.2 * 0.25 / vmax[16], a_disc=a4, Tc_disc=tc4)

    path = os.path.join(ROOT, "workloads", "constants.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
