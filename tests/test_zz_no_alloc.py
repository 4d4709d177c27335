"""The allocation-free context (evlb_init_noalloc) against a context on a
caller workspace: the same steps, right-hand side and moments, on two
noalloc contexts in a row on one device (the second smaller, so that it
re-initialises the shared static workspace over the first one's contents),
in 1D and in 2D."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads  # noqa: E402

from parity import rel  # noqa: E402

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


def _run(noalloc, c, n, u, T, nx, steps, **kw):
    s = E.Solver(c["Q"], c["dx"], c["dt"], nx, noalloc=noalloc, **kw)
    f = s.equilibrium(td(n), td(u), td(T))
    s.step(f, steps)
    L = s.rhs(f)
    m = s.moments(f)
    torch.cuda.synchronize()
    assert s.status() == E.EVLB_OK
    out = f.cpu().numpy(), L.cpu().numpy(), m.cpu().numpy()
    del s
    return out


def _same(got, ref, what):
    for name, a, b in zip(("state", "rhs", "moments"), got, ref):
        err = rel(a, b)
        print(f"{what} {name}: rel err {err:.3e}, bit-identical {np.array_equal(a, b)}", flush=True)
        assert err <= 1e-13, (what, name, err)


def test_noalloc_context_matches_workspace_context_two_calls():
    # first call: the 4096-node evaporation slab (3.3 MiB of workspace)
    c, n, u, T = workloads.slab_1d()
    print("noalloc: slab 1d, 4096 nodes", flush=True)
    ref = _run(False, c, n, u, T, c["nx"], 5)
    got = _run(True, c, n, u, T, c["nx"], 5)
    _same(got, ref, "slab")
    # second call, smaller: the 256-node phase-separation box
    c, n, u, T = workloads.phase_separation_1d()
    print("noalloc: phase separation 1d, 256 nodes", flush=True)
    ref = _run(False, c, n, u, T, c["nx"], 5)
    got = _run(True, c, n, u, T, c["nx"], 5)
    _same(got, ref, "box")


def test_noalloc_context_2d():
    c, n, ux, uy, T = workloads.phase_separation_2d(nx=40, ny=24)
    print("noalloc: 2d 40 x 24", flush=True)
    u = np.stack([ux, uy])
    ref = _run(False, c, n, u, T, 40, 3, ny=24)
    got = _run(True, c, n, u, T, 40, 3, ny=24)
    _same(got, ref, "2d")
