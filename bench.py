"""Throughput of the EV-FDLB time step on one MI355X.

Headline: the 2D phase-separation workload, the largest configuration and
the one bound by HBM bandwidth: 1024 x 1024 periodic nodes, dx = sigma/4,
16 x 16 tensor Gauss-Hermite velocities (plus the reduced z-energy G), T =
0.75 T_c of the disc kernel, n0 = 0.3 with 1% Gaussian noise.  One bench
step = one TVD-RK3 time step (three stages, every part of the method).  The
metric counts site-velocity updates per second: nodes x velocities x 3
stages x steps / GPU time.

Secondary entries: the slab-evaporation workload (4096 nodes, Q = 24, the
latency-bound case), the batched sweep (512 independent periodic systems of
log-uniform length in [256, 8192], Q = 16, about 1.1M nodes), the
adjoint/forward time ratio of the differentiable slab workload, and the
paper's own Sec. III B / III C runs (context for Table I).

Prints one JSON line.  The state is resident in HBM before the timed region;
timing uses HIP events on the stream the kernels run on.  The CPU baseline
is the 2D oracle timed on periodic 128 x 128 windows of the headline
workload, on one host core and on every core the process may use (one
window per worker process), before the GPU is touched.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per site-velocity per RK3 step (F and G together):
# stage 1 reads f^n and writes f^(1) (16 + 16 B), stages 2 and 3 each read
# f^(s-1) and f^n and write f^(s) (48 B); node fields and halo re-reads excluded
BYTES_PER_UPDATE_STEP = 128.0
KERNEL_NAMES = {16: "stage_kernel<{q},16,{q}>", 63: "stage_kernel_col<{q}>", 64: "stage_kernel<{q},64,8>"}


def cpu_baseline(c, n, u, T, target_s=8.0):
    """Oracle (numpy FP64, one thread) on a bounded sample of steps of a 1D
    workload."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle import step1d
    from oracle.model import Params
    lim = threadpool_limits(1) if threadpool_limits else None
    try:
        tb = step1d.Tables(Params(Q=c["Q"], dx=c["dx"], dt=c["dt"]))
        F, G = step1d.initial_state(n, u, T, tb)
        F, G = step1d.rk3_step(F, G, tb)           # warm caches
        t0 = time.perf_counter()
        for _ in range(3):
            F, G = step1d.rk3_step(F, G, tb)
        per = (time.perf_counter() - t0) / 3
        steps = max(3, int(target_s / per))
        t0 = time.perf_counter()
        for _ in range(steps):
            F, G = step1d.rk3_step(F, G, tb)
        el = time.perf_counter() - t0
    finally:
        if lim is not None:
            lim.__exit__(None, None, None)
    rate = c["nx"] * c["Q"] * 3 * steps / el
    return {"value": rate, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} RK3 steps of the {c['nx']}-node Q={c['Q']} slab workload "
                      f"({el:.1f} s, numpy FP64, 1 thread)",
            "host": host_cpu()}


def _oracle_2d_window(args):
    """One worker of the 2D CPU baseline: `steps` RK3 steps of the oracle on
    a periodic w x w window of the headline workload (window index i picks
    its position).  Returns (seconds, updates)."""
    i, w, steps = args
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(1)
    except ImportError:  # pragma: no cover
        lim = None
    import workloads
    from oracle import step2d
    from oracle.model import Params
    c, n, ux, uy, T = workloads.phase_separation_2d()
    y0 = (i * w) % c["ny"]
    x0 = ((i * w) // c["ny"] * w) % c["nx"]
    cut = lambda a: np.ascontiguousarray(a[y0:y0 + w, x0:x0 + w])
    tb = step2d.Tables2D(Params(Q=c["Q"], dx=c["dx"], dt=c["dt"]))
    F, G = step2d.initial_state(cut(n), cut(ux), cut(uy), cut(T), tb)
    t0 = time.perf_counter()
    for _ in range(steps):
        F, G = step2d.rk3_step(F, G, tb)
    el = time.perf_counter() - t0
    if lim is not None:
        lim.__exit__(None, None, None)
    return el, w * w * c["Q"] * c["Q"] * 3 * steps


def cpu_baseline_2d(w=128, steps=3, max_workers=16):
    """The 2D oracle (numpy FP64) on periodic w x w windows cut from the
    headline workload: one worker on one core, then one worker per core the
    process may use (at most max_workers), each on its own window, all
    started together; the rate is total updates over the slowest worker's
    time.  Worker processes are forked before this process touches the
    GPU."""
    import multiprocessing as mp
    el1, up1 = _oracle_2d_window((0, w, steps))
    cores = max(1, min(max_workers, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_2d_window, [(i, w, steps) for i in range(cores)])
    el_all = max(r[0] for r in res)
    up_all = sum(r[1] for r in res)
    return {"value": up_all / el_all, "unit": "updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} RK3 steps of the 2D oracle (numpy FP64, one thread per process) on each of "
                      f"{cores} periodic {w}x{w} windows of the 1024x1024 16x16-velocity workload, one "
                      f"window per process, all cores together ({el_all:.1f} s)",
            "value_1core": up1 / el1,
            "sample_1core": f"{steps} RK3 steps on one {w}x{w} window, one process, one thread ({el1:.1f} s)",
            "host": host_cpu()}


def host_cpu():
    """CPU model and the logical CPUs this process may run on."""
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "cpus": len(os.sched_getaffinity(0))}


TRAFFIC_SOURCE = ("profiles/hbm_traffic.txt: rocprofv3 FETCH_SIZE + WRITE_SIZE per launch from committed counter "
                  "runs, used while the kernel source's sha256 matches (null otherwise); not counted in this run")


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed counter runs (profiles/
    hbm_traffic.txt), or None when the kernel's source file changed since."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "hbm_traffic.txt")) as fh:
            rec = json.load(fh)
        e = rec["entries"].get(f"{workload}/{kernel}")
        if e is None:
            return None
        src = e.get("source", rec.get("source"))
        with open(os.path.join(ROOT, src), "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
    except (OSError, ValueError, KeyError):
        return None
    if sha != e.get("source_sha256", rec.get("source_sha256")):
        return None
    return e["bytes_per_launch"]


def _kernel_names(raw):
    """The full name (template arguments without spaces) and the family
    (no template arguments) of a kernel name as rocprofv3 prints it."""
    n = raw.replace("(anonymous namespace)::", "")
    if n.startswith("void "):
        n = n[5:]
    depth, cut = 0, len(n)
    for i, ch in enumerate(n):  # the argument list: the first '(' outside <>
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    n = n[:cut].replace(" ", "")
    n = n.split("::")[-1] if "<" not in n else n[:n.index("<")].split("::")[-1] + n[n.index("<"):]
    return n, n.split("<")[0]


def write_traffic(workload, fetch_csv, write_csv, commands):
    """Per-launch HBM bytes of every kernel of one workload's counter runs
    (rocprofv3 --pmc FETCH_SIZE, resp. WRITE_SIZE, of bench.py with
    --calibrate-copy, whose last device copy moves 256 MiB and calibrates
    both counters) into profiles/hbm_traffic.txt, keyed workload/kernel for
    the full name and for the family (the mean over its variants)."""
    import csv
    import hashlib
    from collections import defaultdict

    def per_kernel(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        per = defaultdict(lambda: defaultdict(float))
        order = []
        for r in rows:
            per[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
            order.append((int(r["Dispatch_Id"]), r["Kernel_Name"]))
        copies = sorted(d for d, k in order if "copyBuffer" in k)
        if not copies:
            raise SystemExit(f"{path}: no device copy to calibrate against (run with --calibrate-copy)")
        last = copies[-1]
        cal = next(v[str(last)] for k, v in per.items() if str(last) in v)
        return per, cal

    fetch, fcal = per_kernel(fetch_csv, "FETCH_SIZE")
    write, wcal = per_kernel(write_csv, "WRITE_SIZE")
    sf, sw = 262144.0 / fcal, 262144.0 / wcal
    acc = defaultdict(lambda: [0.0, 0.0, 0])
    two_d = workload.endswith("_2d")
    for raw, vals in fetch.items():
        # the library's kernels of this dimension (2D: namespace evlb2d)
        if raw.startswith("__amd") or "at::" in raw or ("evlb2d::" in raw) != two_d:
            continue
        full, fam = _kernel_names(raw)
        wv = write.get(raw, {})
        for d, v in vals.items():
            for key in {full, fam}:
                a = acc[key]
                a[0] += v * 1024.0 * sf
                a[1] += wv.get(d, 0.0) * 1024.0 * sw
                a[2] += 1
    src = "paper_2503_15187_amd/csrc/" + ("evlb2d.hip" if workload.endswith("_2d") else "evlb.hip")
    with open(os.path.join(ROOT, src), "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        rec = {"entries": {}, "commands": {}}
    if not isinstance(rec.get("commands"), dict):
        rec["commands"] = {}
    rec["entries"] = {k: v for k, v in rec["entries"].items() if not k.startswith(workload + "/")}
    for key, (fb, wb, n) in sorted(acc.items()):
        rec["entries"][f"{workload}/{key}"] = {
            "bytes_per_launch": (fb + wb) / n, "fetch_bytes": fb / n, "write_bytes": wb / n, "launches": n,
            "source": src, "source_sha256": sha}
    rec["calibration"] = {"copy_bytes": 256 * 1024 * 1024, "scale_fetch": sf, "scale_write": sw,
                          "copy_fetch_kib": fcal, "copy_write_kib": wcal}
    rec["commands"][workload] = commands
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    for key, (fb, wb, n) in sorted(acc.items()):
        print(f"{workload}/{key}: {(fb + wb) / n:.4g} B per launch ({n} launches)")


def copy_bandwidth(torch, dev, mib=1024, reps=10):
    """Context for the roofline: the rate of a plain device-to-device copy of
    `mib` MiB (read + write bytes over the copy time, HIP events on the
    current stream), next to the published 8 TB/s peak."""
    n = mib * 1024 * 1024 // 8
    x = torch.ones(n, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    gbs = 2 * n * 8 / s / 1e9
    del x, y
    return {"GB_per_s": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS, "bytes": 2 * n * 8,
            "what": f"torch copy_ of {mib} MiB FP64, device to device"}


def default_tile(nx, cus=256):
    """The library's automatic tile choice: column tiles when they give at
    least four wavefronts per CU, else narrow 16-node tiles."""
    nxs = [nx] if isinstance(nx, int) else list(nx)
    return 63 if sum((v + 62) // 63 for v in nxs) >= 4 * cus else 16


def measure(E, torch, dev, q, dx, dt, nx, n, u, T, steps, warmup, mode=None, tile=None, graph=True):
    """Times `steps` RK3 steps.  Per-stage launches are replayed from a
    captured HIP graph of up to 500 steps (graph=True) or launched one by
    one; the persistent mode is one launch either way."""
    from paper_2503_15187_amd import autotune
    td = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    n_tot = int(np.sum(nx))
    if mode is None or tile is None:
        probe = E.Solver(q, dx, dt, nx, device=dev)
        f0 = probe.equilibrium(td(n), td(u), td(T))
        mode, tile, _ = autotune.tune(q, dx, dt, nx, f0, steps=max(5, min(50, steps // 20)), use_cache=False)
        del probe
    s = E.Solver(q, dx, dt, nx, device=dev, exec_mode=mode, tile_nodes=tile)
    f = s.equilibrium(td(n), td(u), td(T))
    stream = torch.cuda.current_stream()
    persistent = mode == E.EVLB_EXEC_PERSISTENT
    use_graph = graph and not persistent
    if use_graph:
        g = autotune.GraphStepper(s, f, chunk=max(1, min(steps, 500)))
        advance = g.step
    else:
        advance = lambda k: s.step(f, k)  # noqa: E731
    if warmup:
        advance(warmup)
    torch.cuda.synchronize()
    if s.status() != 0:
        raise RuntimeError("non-finite state during warm-up")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    advance(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    if s.status() != 0:
        raise RuntimeError("device status not ok after the timed run")
    updates = n_tot * q * 3 * steps
    launches = 1 if persistent else 3 * steps
    kname = KERNEL_NAMES[tile].format(q=q)
    if persistent:
        kname = f"persistent_kernel<{kname}>"
    alg_bytes = BYTES_PER_UPDATE_STEP * n_tot * q * steps / launches
    achieved = alg_bytes / (gpu_s / launches) / 1e9
    return {
        "value": updates / gpu_s, "gpu_s": gpu_s, "wall_s": wall, "ms_per_step": gpu_s * 1e3 / steps,
        "exec": "persistent" if persistent else ("per_stage_graph" if use_graph else "per_stage"), "tile_nodes": tile,
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": alg_bytes, "avg_launch_us": gpu_s / launches * 1e6},
    }


KERNELS_2D = ("fields_kernel", "fused_kernel")


def measure_2d(E, torch, dev, steps, warmup):
    """2D phase separation: 1024 x 1024 periodic nodes, dx = sigma/4, 16 x 16
    tensor Gauss-Hermite velocities plus the reduced z-energy, T = 0.75 T_c
    of the disc kernel, n0 = 0.3 with 1% Gaussian noise.  One RK stage is two
    launches (node fields, then the fused stage kernel), and one raw-sums
    launch starts each evlb_step call; the roofline is taken over the stage:
    algorithmic bytes per stage / stage time."""
    import workloads
    c, n, ux, uy, T = workloads.phase_separation_2d()
    td = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    s = E.Solver(c["Q"], c["dx"], c["dt"], c["nx"], ny=c["ny"], device=dev)
    f = s.equilibrium(td(n), td(np.stack([ux, uy])), td(T))
    stream = torch.cuda.current_stream()
    if warmup:
        s.step(f, warmup)
    torch.cuda.synchronize()
    if s.status() != 0:
        raise RuntimeError("non-finite 2D state during warm-up")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    s.step(f, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    if s.status() != 0:
        raise RuntimeError("device status not ok after the timed 2D run")
    n_tot = c["nx"] * c["ny"]
    nvel = c["Q"] * c["Q"]
    stage_s = gpu_s / (3 * steps)
    alg_stage = BYTES_PER_UPDATE_STEP / 3 * n_tot * nvel
    achieved = alg_stage / stage_s / 1e9
    traffic = [measured_traffic("phase_separation_2d", k) for k in KERNELS_2D]
    return {"config": {"workload": "phase_separation_2d", "nx": c["nx"], "ny": c["ny"], "q": f"{c['Q']}x{c['Q']}",
                       "dx": c["dx"], "dt": c["dt"], "T": c["T"]},
            "steps": steps, "value": n_tot * nvel * 3 * steps / gpu_s, "unit": "updates/s",
            "ms_per_step": gpu_s * 1e3 / steps,
            "roofline": {"bound": "hbm", "kernel": "stage = " + " + ".join(KERNELS_2D), "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": None if None in traffic else sum(traffic), "traffic_source": TRAFFIC_SOURCE,
                         "bytes_per_stage": alg_stage, "avg_stage_us": stage_s * 1e6}}


def paper_runs(E, torch, dev, steps_3b=None):
    """The paper's own runs at its parameters (dx = sigma/10, dt = 5e-3,
    Q = 16), timed end to end for comparison with the single-core runtimes of
    Table I (context, not a target): Sec. III B, the four phase-separation
    runs of eq:rho_init_takata to t = 5000 (1e6 steps; steps_3b shortens
    them and the time per run is scaled to the paper's step count), and
    Sec. III C, the four evaporation runs to t = 75 (15000 steps), each set
    as one batched launch sequence, with EV1 and with EV2."""
    import workloads
    td = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    out = []
    for name, make in (("paper_sec3b_phase_separation", workloads.paper_sec3b),
                       ("paper_sec3c_evaporation", workloads.paper_sec3c)):
        c, systems = make()
        steps = c["steps"] if (steps_3b is None or name.endswith("evaporation")) else steps_3b
        n = np.concatenate([x[0] for x in systems])
        u = np.concatenate([x[1] for x in systems])
        T = np.concatenate([x[2] for x in systems])
        nxs = [len(x[0]) for x in systems]
        for fm, label, paper_s in ((E.EVLB_FORCE_EV1, "EV1", c["table1_ev1_s"]),
                                   (E.EVLB_FORCE_EV2, "EV2", c["table1_ev2_s"])):
            s = E.Solver(c["Q"], c["dx"], c["dt"], nxs, device=dev, force_model=fm)
            f = s.equilibrium(td(n), td(u), td(T))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(f, steps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            if s.status() != 0:
                raise RuntimeError(f"device status not ok in {name} {label}")
            out.append({"config": {"workload": name, "force": label, "runs": len(systems), "nx": nxs[0],
                                   "q": c["Q"], "dx": c["dx"], "dt": c["dt"], "steps": steps,
                                   "t_end": steps * c["dt"]},
                        "metric": "wall time of the batched runs", "value": wall, "unit": "s",
                        "higher_is_better": False,
                        "updates_per_s": sum(nxs) * c["Q"] * 3 * steps / wall,
                        # per run at the paper's step count (scaled per step when the timed run is shorter)
                        "s_per_run_at_paper_steps": wall / len(systems) * c["steps"] / steps,
                        "paper_steps": c["steps"],
                        "paper_single_core_s_per_run": paper_s})
            del s, f
    return out


def adjoint_ratio(E, torch, dev, nsteps):
    """Adjoint workload: 2048 nodes, dx = sigma/4, Q = 16, slab at T = 0.85
    T_c; loss = time-integrated flux through x = 128 sigma + final misfit.
    Times the forward rollout (per-step flux recorded, sqrt(N) checkpoints)
    and the backward pass (segment recompute + discrete adjoint steps)."""
    import workloads
    from paper_2503_15187_amd import adjoint as AD
    c, n0, u0, T0 = workloads.slab_1d(name="adjoint_slab_1d")
    target = workloads.adjoint_target(c, n0)
    i_f = c["nx"] // 2 + int(round(c["x_flux"] / c["dx"]))
    s = E.Solver(c["Q"], c["dx"], c["dt"], c["nx"], device=dev, adjoint=1)
    td = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    n0t = td(n0).requires_grad_(True)
    phi = torch.tensor(1.0, dtype=torch.float64, device=dev, requires_grad=True)
    sig = torch.tensor(1.0, dtype=torch.float64, device=dev, requires_grad=True)
    # warm-up
    L = AD.slab_loss(n0t, phi, sig, s, 20, i_f, c["dt"], c["dx"], td(target), td(T0))
    torch.autograd.grad(L, [n0t, phi, sig])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L = AD.slab_loss(n0t, phi, sig, s, nsteps, i_f, c["dt"], c["dx"], td(target), td(T0))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g = torch.autograd.grad(L, [n0t, phi, sig])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    f = s.equilibrium(td(n0), td(u0), td(T0))
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    s.step(f, nsteps)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    if s.status() != 0:
        raise RuntimeError("device status not ok in the adjoint workload")
    # the transposed step alone: evlb_adjoint_record over a recorded segment
    # (no recomputation) against evlb_step, per step, on HIP events
    seg = int(np.ceil(np.sqrt(nsteps)))
    reps = max(1, nsteps // seg)
    rec = s.record_buffer(seg)
    s.step_record(f, seg, rec)
    lam0 = torch.full_like(f, 1e-3)
    lam = lam0.clone()
    dpar = torch.zeros(2, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    s.adjoint_record(rec, seg, lam, dpar)
    e[0].record(stream)
    for _ in range(reps):
        s.adjoint_record(rec, seg, lam, dpar)
    e[1].record(stream)
    e[2].record(stream)
    s.step(f, reps * seg)
    e[3].record(stream)
    torch.cuda.synchronize()
    adj_step = e[0].elapsed_time(e[1]) / (reps * seg)
    fwd_step = e[2].elapsed_time(e[3]) / (reps * seg)
    return {"config": {"workload": "adjoint_slab_1d", "nx": c["nx"], "q": c["Q"], "dx": c["dx"], "steps": nsteps,
                       "checkpoint_every": int(np.ceil(np.sqrt(nsteps)))},
            "metric": "adjoint/forward time", "value": (t2 - t1) / (t1 - t0), "unit": "ratio",
            "forward_s": t1 - t0, "backward_s": t2 - t1, "plain_forward_s": t4 - t3,
            "ratio_vs_plain_forward": (t2 - t1) / (t4 - t3),
            "adjoint_step_ms": adj_step, "forward_step_ms": fwd_step, "adjoint_step_over_forward_step": adj_step / fwd_step,
            "grad": {"dL_dphi": g[1].item(), "dL_dsigma": g[2].item(), "dL_dn0_norm": g[0].norm().item()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed RK3 steps of the 2D headline workload")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--slab-steps", type=int, default=20000, help="timed RK3 steps of the slab workload")
    ap.add_argument("--slab-warmup", type=int, default=200)
    ap.add_argument("--exec-mode", type=int, default=None, help="slab: 1 per stage, 2 persistent (default: autotune)")
    ap.add_argument("--tile", type=int, default=None, help="slab: 16, 63 or 64 (default: autotune)")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--no-slab", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-paper-runs", action="store_true")
    ap.add_argument("--paper-3b-steps", type=int, default=20000,
                    help="steps of the Sec. III B runs (the paper's 1e6 take about 20 s; the default times "
                         "20000 and scales per step)")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--no-graph", action="store_true",
                    help="launch per-stage kernels one by one instead of replaying a captured HIP graph")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default launch shape (one kernel per stage) instead of timing candidates")
    ap.add_argument("--traffic-from", nargs=3, metavar=("WORKLOAD", "FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/hbm_traffic.txt entries of WORKLOAD from rocprofv3 counter runs and exit "
                         "(no device use); the commands that made them follow as --traffic-command")
    ap.add_argument("--traffic-command", action="append", default=[])
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, run one 256 MiB device-to-device copy (a reference for HBM byte counters)")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(*args.traffic_from, args.traffic_command)
        return
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only; a multi-GPU (domain-decomposed) path is "
              "not implemented. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    # the CPU baseline forks its workers before anything touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline_2d()

    import torch
    import workloads
    from paper_2503_15187_amd import evlb as E

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    head = measure_2d(E, torch, dev, args.steps, args.warmup)
    out = {
        "metric": "site-velocity updates/s per RK stage (FP64)",
        "value": head["value"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "hbm_peak_frac": head["roofline"]["frac"],
        "secondary": [],
    }
    if not args.no_slab:
        c, n, u, T = workloads.slab_1d()
        mode, tile = args.exec_mode, args.tile
        if args.no_autotune:
            mode, tile = E.EVLB_EXEC_PER_STAGE, default_tile(c["nx"])
        m = measure(E, torch, dev, c["Q"], c["dx"], c["dt"], c["nx"], n, u, T, args.slab_steps, args.slab_warmup,
                    mode, tile, graph=not args.no_graph)
        ent = {"config": {"workload": "slab_evaporation_1d", "nx": c["nx"], "q": c["Q"], "dx": c["dx"],
                          "dt": c["dt"], "T": c["T"], "exec": m["exec"], "tile_nodes": m["tile_nodes"]},
               "steps": args.slab_steps, "value": m["value"], "unit": "updates/s", "ms_per_step": m["ms_per_step"],
               "roofline": dict(m["roofline"], traffic=measured_traffic("slab_evaporation_1d", m["roofline"]["kernel"]),
                                traffic_source=TRAFFIC_SOURCE)}
        if not args.no_cpu_baseline:
            ent["cpu_baseline_1core"] = cpu_baseline(c, n, u, T)
        out["secondary"].append(ent)
    if not args.no_batch:
        cb, systems = workloads.batched_sweep_1d()
        nb = np.concatenate([x[0] for x in systems])
        ub = np.concatenate([x[1] for x in systems])
        Tb = np.concatenate([x[2] for x in systems])
        bmode = btile = None
        if args.no_autotune:
            bmode, btile = E.EVLB_EXEC_PER_STAGE, default_tile(cb["nx_list"])
        mb = measure(E, torch, dev, cb["Q"], cb["dx"], cb["dt"], cb["nx_list"], nb, ub, Tb,
                     args.batch_steps, 5, bmode, btile, graph=not args.no_graph)
        out["secondary"].append({
            "config": {"workload": "batched_sweep_1d", "n_sys": cb["n_sys"], "n_tot": int(len(nb)), "q": cb["Q"],
                       "dx": cb["dx"], "exec": mb["exec"], "tile_nodes": mb["tile_nodes"]},
            "steps": args.batch_steps, "value": mb["value"], "unit": "updates/s", "ms_per_step": mb["ms_per_step"],
            "roofline": dict(mb["roofline"], traffic=measured_traffic("batched_sweep_1d", mb["roofline"]["kernel"]),
                             traffic_source=TRAFFIC_SOURCE)})
    if not args.no_adjoint:
        out["secondary"].append(adjoint_ratio(E, torch, dev, args.adjoint_steps))
    if not args.no_paper_runs:
        out["secondary"] += paper_runs(E, torch, dev, args.paper_3b_steps)
    out["hbm_copy"] = copy_bandwidth(torch, dev)
    if args.calibrate_copy:
        x = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
