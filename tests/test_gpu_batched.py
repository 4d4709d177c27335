"""Batched sweeps of many independent 1D systems: graph-captured stepping,
autotuned launch shapes, and the full-size batch checked against the oracle
on sampled systems and by per-system conservation."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads  # noqa: E402
from oracle import step1d  # noqa: E402
from oracle.model import Params  # noqa: E402

from parity import check, rel  # noqa: E402

pytestmark = pytest.mark.gpu

E = AT = None


def setup_module(module):
    global E, AT
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_15187_amd import evlb as _E, autotune as _AT
    E, AT = _E, _AT


def td(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")




def batch(n_sys, nx_max=None):
    c, systems = workloads.batched_sweep_1d(n_sys=n_sys, nx_max=nx_max)
    n = np.concatenate([s[0] for s in systems])
    u = np.concatenate([s[1] for s in systems])
    T = np.concatenate([s[2] for s in systems])
    return c, systems, n, u, T


@pytest.mark.parametrize("tile", [16, 63])
def test_graph_replays_match_eager_steps(tile):
    c, systems, n, u, T = batch(24, 1500)
    s = E.Solver(c["Q"], c["dx"], c["dt"], c["nx_list"], exec_mode=1, tile_nodes=tile)
    f_eager = s.equilibrium(td(n), td(u), td(T))
    f_graph = f_eager.clone()
    f_one = f_eager.clone()
    # each evlb_step call starts from the moments of its input state, so the
    # graph (three calls of 10 steps) is compared with three eager calls
    for _ in range(3):
        s.step(f_eager, 10)
    s.step(f_one, 30)
    g = AT.GraphStepper(s, f_graph, chunk=10)
    ref_after = []
    for i in range(3):
        g.graph.replay()
        # eager work and a synchronisation between replays
        ref_after.append(s.moments(f_graph)[0].sum().item())
        torch.cuda.synchronize()
    assert torch.equal(f_graph, f_eager)
    assert ((f_one - f_eager).abs().max() / f_one.abs().max()).item() < 1e-13
    assert s.status() == 0


def test_graph_replays_single_system_slab():
    """The headline path: one system (no tile descriptors), Q = 24, narrow
    tiles.  Every replay of a 5-step graph, with eager work and a
    synchronisation in between, equals five eager steps bit for bit."""
    c, n, u, T = workloads.slab_1d(nx=1024)
    s = E.Solver(c["Q"], c["dx"], c["dt"], c["nx"], exec_mode=1, tile_nodes=16)
    f_eager = s.equilibrium(td(n), td(u), td(T))
    f_graph = f_eager.clone()
    g = AT.GraphStepper(s, f_graph, chunk=5)
    for i in range(4):
        g.graph.replay()
        s.step(f_eager, 5)
        _ = s.moments(f_graph)[0].sum().item()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(f_graph, f_eager), i
    assert s.status() == 0


def test_graph_stepper_remainder():
    c, systems, n, u, T = batch(8, 900)
    s = E.Solver(c["Q"], c["dx"], c["dt"], c["nx_list"], exec_mode=1, tile_nodes=16)
    fa = s.equilibrium(td(n), td(u), td(T))
    fb = fa.clone()
    for k in (10, 10, 3):
        s.step(fa, k)
    AT.GraphStepper(s, fb, chunk=10).step(23)
    torch.cuda.synchronize()
    assert torch.equal(fa, fb)


def test_autotune_picks_a_working_shape():
    c, systems, n, u, T = batch(16, 1200)
    probe = E.Solver(c["Q"], c["dx"], c["dt"], c["nx_list"])
    f0 = probe.equilibrium(td(n), td(u), td(T))
    mode, tile, sec = AT.tune(c["Q"], c["dx"], c["dt"], c["nx_list"], f0, steps=3, use_cache=False)
    assert (mode, tile) in AT.CANDIDATES and sec > 0


@pytest.mark.timeout(900)
def test_full_batch_all_systems_match_oracle():
    """All 512 systems (about 1.1M nodes) in the launch shape the bench uses
    (column tiles, one kernel per stage), 3 steps; every system is
    recomputed by the oracle."""
    c, systems, n, u, T = batch(None)
    nxs = c["nx_list"]
    s = E.Solver(c["Q"], c["dx"], c["dt"], nxs, exec_mode=1, tile_nodes=63)
    f = s.equilibrium(td(n), td(u), td(T))
    s.step(f, 3)
    assert s.status() == 0
    got = f.cpu().numpy()
    offs = np.concatenate([[0], np.cumsum(nxs)])
    tb = step1d.Tables(Params(Q=c["Q"], dx=c["dx"], dt=c["dt"]))
    for i in range(len(nxs)):
        ni, ui, Ti = systems[i]
        F, G = step1d.initial_state(ni, ui, Ti, tb)
        F, G = step1d.run(F, G, tb, 3)
        check(got[:, :, offs[i]:offs[i + 1]], [F, G], 1e-11, steps=3, what=repr((i, nxs[i])))


def test_full_batch_per_system_mass_conservation():
    c, systems, n, u, T = batch(None)
    nxs = c["nx_list"]
    s = E.Solver(c["Q"], c["dx"], c["dt"], nxs, exec_mode=1, tile_nodes=63)
    f = s.equilibrium(td(n), td(u), td(T))
    offs = torch.tensor(np.concatenate([[0], np.cumsum(nxs)]), device="cuda")
    seg = torch.repeat_interleave(torch.arange(len(nxs), device="cuda"), torch.tensor(nxs, device="cuda"))

    def per_system_mass(f):
        m = f[0].sum(0)
        return torch.zeros(len(nxs), dtype=torch.float64, device="cuda").index_add_(0, seg, m)

    m0 = per_system_mass(f)
    s.step(f, 50)
    m1 = per_system_mass(f)
    assert s.status() == 0
    assert torch.max(torch.abs(m1 - m0) / m0).item() < 1e-13
