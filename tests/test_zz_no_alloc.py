"""hub_apply_cheb_noalloc (the Chebyshev preconditioner with its workspace in
the library's fixed per-GPU array) against hub_apply_cheb, through the C ABI.

Both run the same sweeps with the same factor order, so the results must be
bitwise equal.  The calls come in a row with shrinking inputs (the largest
lattice the fixed array holds, a smaller fused one, then a two-pass lattice
that uses the array for two vectors), so stale contents of the shared array
from the previous call cannot go unnoticed; the last test records the call
into a HIP graph and replays it.
"""
import numpy as np
import pytest
import torch

from paper_1007_3432_amd import hub, inputs
from tests import hubtest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    hubtest.ensure_built()


def _inputs(shape, seed):
    d, nx, nt = shape
    lat = hub.lattice(d, nx, nt)
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=seed)
    links = hubtest.empty(lat.volume, hub.F64)
    hub.hub_links_from_sigma(lat, hubtest.to_dev(sigma), links, hub.F64)
    r = hubtest.to_dev(inputs.random_vector(lat.volume, seed + 1))
    return lat, links, r


SEQUENCE = [(3, 32, 256), (3, 16, 160), (1, 300, 37), (2, 20, 30)]


def test_noalloc_matches_allocating_call_in_a_row():
    cheb = hub.cheb_opts(6, 0.01)
    for k, shape in enumerate(SEQUENCE):
        hubtest.log_case(f"cheb noalloc {shape}")
        lat, links, r = _inputs(shape, 40 + k)
        z_ref = hubtest.empty(lat.volume, hub.F64)
        z = hubtest.empty(lat.volume, hub.F64).fill_(np.nan)
        hub.hub_apply_cheb(lat, links, r, z_ref, cheb)
        hub.hub_apply_cheb_noalloc(lat, links, r, z, cheb)
        a, b = z.cpu().numpy(), z_ref.cpu().numpy()
        assert np.all(np.isfinite(a)), shape
        assert np.array_equal(a, b), (shape, np.max(np.abs(a - b)))


def test_noalloc_rejects_lattice_beyond_the_array():
    lat = hub.lattice(1, 4096, 4098)   # 16.8M sites: 128 MiB of workspace
    links = hubtest.empty(16, hub.F64)
    with pytest.raises(hub.HubError) as e:
        hub.load()
        import ctypes
        s = hub.load().hub_apply_cheb_noalloc(ctypes.byref(lat), links.data_ptr(),
                                              links.data_ptr() + 64, links.data_ptr() + 128,
                                              ctypes.byref(hub.cheb_opts(4, 0.01)), None)
        hub._check(s, "hub_apply_cheb_noalloc")
    assert e.value.status == hub.HUB_E_NOMEM


def test_noalloc_under_graph_capture():
    """Recorded once into a HIP graph and replayed three times, with eager
    calls of the allocating variant on other inputs in between: every replay
    gives the eager result."""
    cheb = hub.cheb_opts(4, 0.003)
    lat, links, r = _inputs((1, 2048, 64), 60)
    lat2, links2, r2 = _inputs((3, 8, 40), 61)
    z_ref = hubtest.empty(lat.volume, hub.F64)
    hub.hub_apply_cheb(lat, links, r, z_ref, cheb)
    z = hubtest.empty(lat.volume, hub.F64)
    hub.hub_apply_cheb_noalloc(lat, links, r, z, cheb)     # first call: symbol lookup
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        hub.hub_apply_cheb_noalloc(lat, links, r, z, cheb)
    want = z_ref.cpu().numpy()
    for rep in range(3):
        z.fill_(np.nan)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(z.cpu().numpy(), want), rep
        z2 = hubtest.empty(lat2.volume, hub.F64)
        hub.hub_apply_cheb_noalloc(lat2, links2, r2, z2, cheb)
        torch.cuda.synchronize()
