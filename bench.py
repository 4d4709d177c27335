"""Throughput of the EV-FDLB time step on one MI355X.

One bench step = one TVD-RK3 time step (three stages, every part of the
method) of the slab-evaporation workload: 4096 nodes, Q = 24 Gauss-Hermite
velocities, dx = sigma/8, liquid slab 64 sigma wide (eq:tan) at the
coexistence densities of T/T_c = 0.8.  The metric counts site-velocity
updates per second: nodes x velocities x 3 stages x steps / GPU time.

Prints one JSON line (see the fields below).  The state is resident in HBM
before the timed region; timing uses HIP events on the stream the kernels run
on.  The CPU baseline is the oracle timed on a bounded number of steps of
the same workload on one host core.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE_STEP = 128.0   # per site-velocity per RK3 step (F and G)


def cpu_baseline(c, n, u, T, target_s=12.0):
    """Oracle (numpy FP64, one thread) on a bounded sample of steps."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle import step1d
    from oracle.model import Params
    ctxm = threadpool_limits(1) if threadpool_limits else None
    try:
        tb = step1d.Tables(Params(Q=c["Q"], dx=c["dx"], dt=c["dt"]))
        F, G = step1d.initial_state(n, u, T, tb)
        t0 = time.perf_counter()
        F, G = step1d.rk3_step(F, G, tb)
        t1 = time.perf_counter() - t0
        steps = max(1, int(target_s / max(t1, 1e-6)))
        t0 = time.perf_counter()
        for _ in range(steps):
            F, G = step1d.rk3_step(F, G, tb)
        el = time.perf_counter() - t0
    finally:
        if ctxm is not None:
            ctxm.__exit__(None, None, None)
    rate = c["nx"] * c["Q"] * 3 * steps / el
    return {"value": rate, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} RK3 steps of the {c['nx']}x{c['Q']} slab workload ({el:.1f} s, numpy FP64, 1 thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed RK3 steps (default: the workload's 20000)")
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--exec-mode", type=int, default=0, help="0 auto, 1 per stage, 2 persistent")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU (domain-decomposed) path is "
              "not part of it. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2503_15187_amd import evlb as E

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    c, n, u, T = workloads.slab_1d()
    steps = args.steps if args.steps is not None else c["steps"]
    s = E.Solver(c["Q"], c["dx"], c["dt"], c["nx"], device=dev, exec_mode=args.exec_mode)
    td = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    f = s.equilibrium(td(n), td(u), td(T))
    stream = torch.cuda.current_stream()
    if args.warmup:
        s.step(f, args.warmup)
    torch.cuda.synchronize()
    if s.status() != 0:
        raise RuntimeError("non-finite state during warm-up")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    s.step(f, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    status = s.status()
    if status != 0:
        raise RuntimeError(f"device status {status} after the timed run")

    updates = c["nx"] * c["Q"] * 3 * steps
    value = updates / gpu_s
    # dominant kernel: the whole step loop runs in one persistent launch (auto
    # mode for this size), so one launch moves 128 B per site-velocity per step
    persistent = args.exec_mode == 2 or (args.exec_mode == 0 and (c["nx"] + 63) // 64 <= 2 * 256)
    if persistent:
        launches = 1
        kernel = "persistent_kernel<24,8>"
    else:
        launches = 3 * steps
        kernel = "stage_kernel<24,8>"
    alg_bytes = BYTES_PER_UPDATE_STEP * c["nx"] * c["Q"] * steps / launches
    dur = gpu_s / launches
    achieved = alg_bytes / dur / 1e9
    out = {
        "metric": "site-velocity updates/s per RK stage (FP64)",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_s * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "slab_evaporation_1d", "nx": c["nx"], "q": c["Q"], "dx": c["dx"],
                   "dt": c["dt"], "T": c["T"], "exec": "persistent" if persistent else "per_stage"},
        "roofline": {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "hbm_peak_frac": achieved / HBM_PEAK_GBS,
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, n, u, T)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
