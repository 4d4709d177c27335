"""Host-side checks of the C ABI: the library loads, exports every entry
point declared in include/evlb.h, and validates parameters on the host
(no device call is made by any of these)."""
import ctypes
import os
import re

import pytest

import paper_2503_15187_amd as P
from paper_2503_15187_amd import evlb as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DT16 = 0.2 * 0.125 / 6.630878198393129


def declared_functions():
    src = open(os.path.join(ROOT, "include", "evlb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(evlb_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported():
    names = declared_functions()
    assert len(names) >= 10
    L = P.lib()
    for name in names:
        assert hasattr(L, name), name


def test_validate_accepts_workload_parameters():
    assert P.evlb_validate(P.make_params(16, 0.125, DT16, 256)) == E.EVLB_OK
    assert P.evlb_validate(P.make_params(16, 0.1, 5e-3, [2000] * 5, T_iso=0.6)) == E.EVLB_OK
    assert P.evlb_validate(P.make_params(24, 0.125, 0.2 * 0.125 / 8.5078, 4096)) == E.EVLB_OK
    assert P.evlb_validate(P.make_params(16, 0.25, 0.2 * 0.25 / 6.6309, [256, 300, 8192])) == E.EVLB_OK


@pytest.mark.parametrize("kw,code", [
    (dict(q=12), E.EVLB_EUNSUPPORTED),
    (dict(dt=0.1), E.EVLB_ECFL),
    (dict(dt=-1.0), E.EVLB_EINVAL),
    (dict(dx=0.3), E.EVLB_EINVAL),            # sigma/dx not an even integer
    (dict(r_cut=5.125), E.EVLB_EINVAL),       # r_cut/dx odd
    (dict(r_cut=9.0), E.EVLB_EINVAL),         # window above the built maximum
    (dict(nx=4), E.EVLB_EINVAL),
    (dict(nx=[256, 0]), E.EVLB_EINVAL),
    (dict(gamma=2.5), E.EVLB_EINVAL),
    (dict(force_model=E.EVLB_FORCE_EV2, gamma=4.5), E.EVLB_EINVAL),
    (dict(force_model=7), E.EVLB_EINVAL),
    (dict(term_mask=16), E.EVLB_EINVAL),
    (dict(weno_eps=0.0), E.EVLB_EINVAL),
    (dict(exec_mode=9), E.EVLB_EINVAL),
    (dict(sigma=-1.0), E.EVLB_EINVAL),
    (dict(T_iso=-0.5), E.EVLB_EINVAL),
    (dict(T_iso=0.6, adjoint=1), E.EVLB_EUNSUPPORTED),
    (dict(nx=[256, 300], T_iso_sys=[0.6, -0.1]), E.EVLB_EINVAL),
    (dict(nx=[256, 300], T_iso_sys=[0.6, float("nan")]), E.EVLB_EINVAL),
    (dict(nx=[256, 300], T_iso_sys=[0.0, 0.6], adjoint=1), E.EVLB_EUNSUPPORTED),
])
def test_validate_rejects(kw, code):
    base = dict(q=16, dx=0.125, dt=DT16, nx=256)
    base.update(kw)
    p = P.make_params(**base)
    assert P.evlb_validate(p) == code
    assert P.evlb_workspace_bytes(p) == 0


def test_abi_version_checked():
    p = P.make_params(16, 0.125, DT16, 256)
    p.abi_version = 99
    assert P.evlb_validate(p) == E.EVLB_EINVAL


def test_workspace_size_scales_with_nodes():
    a = P.evlb_workspace_bytes(P.make_params(16, 0.125, DT16, 1024))
    b = P.evlb_workspace_bytes(P.make_params(16, 0.125, DT16, 2048))
    # two stage buffers [2][q][n] and two moment buffers [4][n] per node
    per_node = 2 * 2 * 16 * 8 + 2 * 4 * 8
    assert abs((b - a) - 1024 * per_node) < 4096


def test_init_rejects_missing_workspace_before_device_work():
    p = P.make_params(16, 0.125, DT16, 256)
    out = ctypes.c_void_p()
    L = P.lib()
    assert L.evlb_init(ctypes.byref(p), None, 0, None, ctypes.byref(out)) == E.EVLB_EWORKSPACE
    assert L.evlb_init(ctypes.byref(p), ctypes.c_void_p(256), 16, None, ctypes.byref(out)) == E.EVLB_EWORKSPACE
    assert L.evlb_init(ctypes.byref(p), ctypes.c_void_p(257), 1 << 30, None, ctypes.byref(out)) == E.EVLB_EWORKSPACE
    assert out.value is None


def test_null_context_rejected():
    L = P.lib()
    assert L.evlb_step(None, None, 1, None) == E.EVLB_EINVAL
    assert L.evlb_moments(None, None, None, None, None, None, None) == E.EVLB_EINVAL
    assert L.evlb_status(None, None, 0) == E.EVLB_EINVAL


def test_strerror():
    for code in (0, -1, -2, -3, -4, -5, -6, -77):
        assert isinstance(P.strerror(code), str) and P.strerror(code)


# ---------------------------------------------------------------------------
# dim = 2
# ---------------------------------------------------------------------------
DT2D = 0.2 * 0.25 / 6.630878198393129


def _p2(**kw):
    base = dict(q=16, dx=0.25, dt=DT2D, nx=1024, ny=1024)
    base.update(kw)
    return P.make_params(**base)


def test_validate_accepts_2d_workload():
    p = _p2()
    assert p.dim == 2
    assert P.evlb_validate(p) == E.EVLB_OK
    assert P.evlb_validate(_p2(nx=40, ny=24)) == E.EVLB_OK
    assert P.evlb_validate(_p2(force_model=E.EVLB_FORCE_NONE)) == E.EVLB_OK


@pytest.mark.parametrize("kw,code", [
    (dict(q=8), E.EVLB_EUNSUPPORTED),
    (dict(gamma=8.0), E.EVLB_EUNSUPPORTED),
    (dict(force_model=E.EVLB_FORCE_EV2), E.EVLB_EUNSUPPORTED),
    (dict(adjoint=1), E.EVLB_EUNSUPPORTED),
    (dict(exec_mode=E.EVLB_EXEC_PERSISTENT), E.EVLB_EUNSUPPORTED),
    (dict(tile_nodes=64), E.EVLB_EINVAL),
    (dict(ny=4), E.EVLB_EINVAL),
    (dict(nx=[64, 64]), E.EVLB_EINVAL),
    (dict(r_cut=5.1), E.EVLB_EINVAL),       # r_cut/dx not an integer
    (dict(r_cut=7.0), E.EVLB_EINVAL),       # force disc above the built maximum
    (dict(dt=0.2), E.EVLB_ECFL),
    (dict(dt=0.6 * 0.25 / 6.630878198393129), E.EVLB_ECFL),  # 1D limit met, 2D sum exceeded
    (dict(T_iso=float("nan")), E.EVLB_EINVAL),
    (dict(T_iso_sys=[0.6]), E.EVLB_EUNSUPPORTED),
])
def test_validate_rejects_2d(kw, code):
    p = _p2(**kw)
    assert P.evlb_validate(p) == code
    assert P.evlb_workspace_bytes(p) == 0


def test_workspace_2d_scales_with_nodes():
    a = P.evlb_workspace_bytes(_p2(nx=256, ny=256))
    b = P.evlb_workspace_bytes(_p2(nx=256, ny=512))
    # two stage buffers [2][256][n], moments [6][n], raw velocity sums
    # [11][n] and node fields [18][n]
    per_node = 2 * 2 * 256 * 8 + 6 * 8 + 11 * 8 + 18 * 8
    assert abs((b - a) - 256 * 256 * per_node) < 4096


def test_init_2d_rejects_missing_workspace_before_device_work():
    p = _p2(nx=64, ny=64)
    out = ctypes.c_void_p()
    L = P.lib()
    assert L.evlb_init(ctypes.byref(p), None, 0, None, ctypes.byref(out)) == E.EVLB_EWORKSPACE
    assert L.evlb_init(ctypes.byref(p), ctypes.c_void_p(256), 16, None, ctypes.byref(out)) == E.EVLB_EWORKSPACE
    assert out.value is None


def test_per_system_isothermal_temperatures():
    """T_iso_sys: accepted with zeros (thermal) and positive entries, also with
    the adjoint when every entry is 0; one double per node more workspace; one
    value per system required by the binding."""
    nxs = [2000, 1500, 1000]
    base = P.make_params(16, 0.1, 5e-3, nxs)
    p = P.make_params(16, 0.1, 5e-3, nxs, T_iso_sys=[0.55, 0.0, 0.7])
    assert P.evlb_validate(p) == E.EVLB_OK
    grow = P.evlb_workspace_bytes(p) - P.evlb_workspace_bytes(base)
    assert 8 * sum(nxs) <= grow < 8 * sum(nxs) + 256
    assert P.evlb_validate(P.make_params(16, 0.1, 5e-3, nxs, adjoint=1, T_iso_sys=[0.0] * 3)) == E.EVLB_OK
    with pytest.raises(ValueError):
        P.make_params(16, 0.1, 5e-3, nxs, T_iso_sys=[0.6, 0.6])


def test_noalloc_rejects_oversized_workspace_on_host():
    """evlb_init_noalloc checks the static workspace limit before any device
    call: a 256 x 256 2D system needs more than EVLB_NOALLOC_MAX_BYTES."""
    p = P.make_params(16, 0.25, DT2D, 256, ny=256)
    assert P.evlb_workspace_bytes(p) > E.EVLB_NOALLOC_MAX_BYTES
    out = ctypes.c_void_p()
    assert P.lib().evlb_init_noalloc(ctypes.byref(p), None, ctypes.byref(out)) == E.EVLB_EWORKSPACE
    assert out.value is None
    cfl = P.make_params(16, 0.125, 0.1, 256)
    assert P.lib().evlb_init_noalloc(ctypes.byref(cfl), None, ctypes.byref(out)) == E.EVLB_ECFL
