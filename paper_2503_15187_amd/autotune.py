"""Launch-shape autotuner and graph-captured stepping.

The stage kernel comes in three tile shapes (16-node narrow tiles with one
velocity per thread, 63-node column tiles with one node per thread, 64-node
tiles with velocity groups) and two launch modes (one kernel per stage, or one
persistent cooperative kernel for all steps).  Which is fastest depends on
the grid size: the autotuner times every candidate for a few steps on the
caller's problem and caches the winner per problem signature.

GraphStepper captures a fixed number of steps of the chosen per-stage
launches in a HIP graph (through torch.cuda.graph) and replays it, so a long
run costs one graph launch per chunk.
"""
import json
import os
import time

import torch

from . import evlb as E

CANDIDATES = [(E.EVLB_EXEC_PER_STAGE, 16), (E.EVLB_EXEC_PER_STAGE, 63), (E.EVLB_EXEC_PER_STAGE, 64),
              (E.EVLB_EXEC_PERSISTENT, 16), (E.EVLB_EXEC_PERSISTENT, 63)]

_CACHE_PATH = os.environ.get("EVLB_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "evlb_tune.json"))
_memo = {}


def signature(q, nx, **kw):
    nxs = [int(nx)] if isinstance(nx, int) else [int(v) for v in nx]
    return f"q{q}-n{sum(nxs)}-s{len(nxs)}-max{max(nxs)}-" + "-".join(f"{k}{v}" for k, v in sorted(kw.items()))


def _load_cache():
    try:
        with open(_CACHE_PATH) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(d):
    try:
        os.makedirs(os.path.dirname(_CACHE_PATH), exist_ok=True)
        with open(_CACHE_PATH, "w") as fh:
            json.dump(d, fh, indent=1)
    except OSError:
        pass


def tune(q, dx, dt, nx, f0, steps=10, candidates=CANDIDATES, use_cache=True, verbose=False, **kw):
    """Returns (exec_mode, tile_nodes, seconds per step) of the fastest
    candidate on this problem.  f0: a representative state (not modified)."""
    sig = signature(q, nx, **{k: v for k, v in kw.items() if k in ("force_model", "term_mask")})
    if use_cache:
        if sig in _memo:
            return _memo[sig]
        cache = _load_cache()
        if sig in cache:
            _memo[sig] = tuple(cache[sig])
            return _memo[sig]
    best = None
    for mode, tile in candidates:
        s = E.Solver(q, dx, dt, nx, device=f0.device, exec_mode=mode, tile_nodes=tile, **kw)
        f = f0.clone()
        s.step(f, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(f, steps)
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / steps
        if s.status() != 0:
            continue
        if verbose:
            print(f"  autotune {sig}: mode={mode} tile={tile} {dt_s * 1e6:.1f} us/step", flush=True)
        if best is None or dt_s < best[2]:
            best = (mode, tile, dt_s)
        del s
    if best is None:
        raise RuntimeError("no launch shape ran cleanly")
    _memo[sig] = best
    if use_cache:
        cache = _load_cache()
        cache[sig] = list(best)
        _store_cache(cache)
    return best


class GraphStepper:
    """Steps a Solver through a captured HIP graph of `chunk` steps.

    The graph binds the state tensor it was captured with; step() runs
    nsteps = m * chunk + r steps as m graph replays plus r eager steps."""

    def __init__(self, solver, f, chunk=50):
        if solver.params.exec_mode == E.EVLB_EXEC_PERSISTENT:
            raise ValueError("graph capture is for per-stage launches")
        self.solver = solver
        self.f = f
        self.chunk = int(chunk)
        # warm-up outside capture, then capture on torch's side stream
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            solver.step(f, 0)
        torch.cuda.current_stream().wait_stream(s)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            solver.step(f, self.chunk)

    def step(self, nsteps):
        m, r = divmod(int(nsteps), self.chunk)
        for _ in range(m):
            self.graph.replay()
        if r:
            self.solver.step(self.f, r)
        return self.f
