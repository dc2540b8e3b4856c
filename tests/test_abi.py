"""The C-ABI library loads, exports every symbol its header declares, and
rejects bad arguments before touching the device (no GPU needed)."""
import ctypes
import math

import pytest

from paper_1007_3432_amd import hub
from tests import hubtest


@pytest.fixture(scope="module")
def lib():
    hubtest.ensure_built()
    return hub.load()


def test_header_declares_the_api():
    names = set(hub.declared_symbols())
    assert {"hub_links_from_sigma", "hub_apply_M", "hub_apply_MtM", "hub_cg_solve",
            "hub_apply_cheb", "hub_apply_cheb_noalloc", "hub_pcg_solve",
            "hub_hmc_force", "hub_md_trajectory", "hub_hmc_trajectory", "hub_serve_create", "hub_serve_submit", "hub_serve_poll",
            "hub_serve_destroy", "hub_solver_release", "hub_last_error"} <= names


def test_every_declared_symbol_is_exported(lib):
    for name in hub.declared_symbols():
        assert hasattr(lib, name), name


def _call_apply(lib, lat, link=hub.F64, vec=hub.F64, x=16, y=32, links=48):
    return lib.hub_apply_MtM(ctypes.byref(lat), ctypes.c_void_p(links), link, vec,
                             ctypes.c_void_p(x), ctypes.c_void_p(y), None)


@pytest.mark.parametrize("bad", [dict(d=0), dict(d=4), dict(nx=1), dict(nt=1),
                                 dict(U=0.5), dict(dtau=0.0), dict(t_hop=-1.0),
                                 dict(mu=math.nan), dict(nx=2 ** 11, d=3)])
def test_invalid_lattice_rejected(lib, bad):
    kw = dict(d=1, nx=8, nt=8, t_hop=1.0, dtau=0.05, U=-2.0, mu=0.0)
    kw.update(bad)
    lat = hub.lattice(**kw)
    assert _call_apply(lib, lat) == hub.HUB_E_INVALID
    assert hub.last_error()


def test_reserved_must_be_zero(lib):
    lat = hub.lattice(1, 8, 8)
    lat.reserved = 1
    assert _call_apply(lib, lat) == hub.HUB_E_INVALID


@pytest.mark.parametrize("link,vec", [(hub.F32, hub.F64), (hub.F16, hub.F64),
                                      (hub.F64, hub.F32), (hub.F16, hub.F16), (7, 0)])
def test_bad_precision_pair_rejected(lib, link, vec):
    assert _call_apply(lib, hub.lattice(1, 8, 8), link=link, vec=vec) == hub.HUB_E_INVALID


def test_null_misaligned_and_aliased_pointers(lib):
    lat = hub.lattice(1, 8, 8)
    assert _call_apply(lib, lat, x=0) == hub.HUB_E_INVALID
    assert "x" in hub.last_error()
    assert _call_apply(lib, lat, x=20) == hub.HUB_E_INVALID
    assert "aligned" in hub.last_error()
    assert _call_apply(lib, lat, x=64, y=64) == hub.HUB_E_INVALID


def test_cg_options_validated(lib):
    lat = hub.lattice(1, 8, 8)
    st = hub.CGStats()
    for opts in (hub.cg_opts(tol=0.0), hub.cg_opts(tol=1.5), hub.cg_opts(max_iter=0),
                 hub.cg_opts(bulk=hub.F32, reliable_every=0),
                 hub.CGOpts(hub.F64, hub.F16, 1e-10, 10, 50),
                 hub.CGOpts(hub.F16, hub.F16, 1e-10, 10, 50)):
        s = lib.hub_cg_solve(ctypes.byref(lat), ctypes.c_void_p(16), ctypes.c_void_p(32),
                             ctypes.c_void_p(48), ctypes.byref(opts), ctypes.byref(st), None)
        assert s == hub.HUB_E_INVALID


@pytest.mark.parametrize("cheb", [hub.ChebOpts(0, 0, 0.01, 0.0), hub.ChebOpts(257, 0, 0.01, 0.0),
                                  hub.ChebOpts(4, 1, 0.01, 0.0), hub.ChebOpts(4, 0, 0.0, 0.0),
                                  hub.ChebOpts(4, 0, 1.0, 0.0),
                                  hub.ChebOpts(4, 0, 0.01, math.inf)])
def test_cheb_options_validated(lib, cheb):
    lat = hub.lattice(1, 8, 8)
    assert lib.hub_apply_cheb(ctypes.byref(lat), ctypes.c_void_p(16), ctypes.c_void_p(32),
                              ctypes.c_void_p(48), ctypes.byref(cheb), None) == hub.HUB_E_INVALID
    st = hub.CGStats()
    assert lib.hub_pcg_solve(ctypes.byref(lat), ctypes.c_void_p(16), ctypes.c_void_p(32),
                             ctypes.c_void_p(48), ctypes.byref(hub.cg_opts()),
                             ctypes.byref(cheb), ctypes.byref(st), None) == hub.HUB_E_INVALID
    assert lib.hub_apply_cheb(ctypes.byref(lat), ctypes.c_void_p(16), ctypes.c_void_p(32),
                              None, ctypes.byref(hub.cheb_opts(4, 0.01)), None) == hub.HUB_E_INVALID
    assert lib.hub_apply_cheb(ctypes.byref(lat), ctypes.c_void_p(16), ctypes.c_void_p(32),
                              ctypes.c_void_p(32), ctypes.byref(hub.cheb_opts(4, 0.01)),
                              None) == hub.HUB_E_INVALID


def test_cheb_noalloc_rejects_oversize_before_launch(lib):
    """More sites than the fixed 64 MiB workspace holds: HUB_E_NOMEM from the
    host-side check, before any device call."""
    for lat in (hub.lattice(1, 4096, 2050),          # 8 396 800 sites, fused plan
                hub.lattice(2, 1448, 3)):            # 6 290 112 sites, two-pass plan
        s = lib.hub_apply_cheb_noalloc(ctypes.byref(lat), ctypes.c_void_p(16),
                                       ctypes.c_void_p(32), ctypes.c_void_p(48),
                                       ctypes.byref(hub.cheb_opts(4, 0.01)), None)
        assert s == hub.HUB_E_NOMEM
        assert "64 MiB" in hub.last_error() or "workspace" in hub.last_error()


@pytest.mark.parametrize("opts", [hub.MDOpts(0, 0, 0.1, hub.cg_opts()),
                                  hub.MDOpts(4, 1, 0.1, hub.cg_opts()),
                                  hub.MDOpts(4, 0, 0.0, hub.cg_opts()),
                                  hub.MDOpts(4, 0, math.nan, hub.cg_opts()),
                                  hub.MDOpts(4, 0, 0.1, hub.cg_opts(tol=0.0)),
                                  hub.MDOpts(4, 0, 0.1, hub.CGOpts(hub.F16, hub.F16, 1e-10, 9, 50))])
def test_md_options_validated(lib, opts):
    lat = hub.lattice(1, 8, 8)
    st = hub.MDStats()
    assert lib.hub_md_trajectory(ctypes.byref(lat), ctypes.c_void_p(16), ctypes.c_void_p(32),
                                 ctypes.c_void_p(48), ctypes.byref(opts), ctypes.byref(st),
                                 None) == hub.HUB_E_INVALID
    assert lib.hub_hmc_trajectory(ctypes.byref(lat), ctypes.c_void_p(16), ctypes.c_void_p(32),
                                  ctypes.c_void_p(48), ctypes.c_double(0.5), ctypes.byref(opts),
                                  ctypes.byref(st), None) == hub.HUB_E_INVALID


def test_hmc_pointer_checks(lib):
    lat = hub.lattice(1, 8, 8)
    st = hub.MDStats()
    good = hub.md_opts(2, 0.1)
    assert lib.hub_hmc_force(ctypes.byref(lat), ctypes.c_void_p(16), ctypes.c_void_p(32),
                             ctypes.c_void_p(16), None) == hub.HUB_E_INVALID
    assert lib.hub_hmc_force(ctypes.byref(lat), ctypes.c_void_p(16), ctypes.c_void_p(40),
                             ctypes.c_void_p(64), None) == hub.HUB_E_INVALID
    assert lib.hub_md_trajectory(ctypes.byref(lat), ctypes.c_void_p(16), ctypes.c_void_p(16),
                                 ctypes.c_void_p(48), ctypes.byref(good), ctypes.byref(st),
                                 None) == hub.HUB_E_INVALID
    assert lib.hub_hmc_trajectory(ctypes.byref(lat), ctypes.c_void_p(16), ctypes.c_void_p(32),
                                  ctypes.c_void_p(48), ctypes.c_double(math.inf),
                                  ctypes.byref(good), ctypes.byref(st), None) == hub.HUB_E_INVALID


def test_pcg_requires_fp64(lib):
    lat = hub.lattice(1, 8, 8)
    st = hub.CGStats()
    for opts in (hub.cg_opts(bulk=hub.F32), hub.cg_opts(bulk=hub.F32, link=hub.F16)):
        assert lib.hub_pcg_solve(ctypes.byref(lat), ctypes.c_void_p(16), ctypes.c_void_p(32),
                                 ctypes.c_void_p(48), ctypes.byref(opts),
                                 ctypes.byref(hub.cheb_opts(4, 0.01)), ctypes.byref(st),
                                 None) == hub.HUB_E_INVALID
        assert "F64" in hub.last_error()


def test_last_error_empty_after_success_path_is_thread_local(lib):
    import threading
    lat = hub.lattice(0, 8, 8)
    assert _call_apply(lib, lat) == hub.HUB_E_INVALID
    seen = []
    th = threading.Thread(target=lambda: seen.append(hub.last_error()))
    th.start()
    th.join()
    assert seen == [""]
    assert hub.last_error() != ""


def test_solver_release_before_any_solve_is_a_no_op(lib):
    """Nothing cached yet on this thread: the release touches no device."""
    assert lib.hub_solver_release() == hub.HUB_OK
    assert lib.hub_solver_release() == hub.HUB_OK
    assert hub.last_error() == ""
