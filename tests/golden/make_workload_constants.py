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
