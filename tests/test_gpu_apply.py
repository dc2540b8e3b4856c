"""Parity of the HIP link precompute, M, M^T and the fused M^T M sweep with
the CPU oracle, through the C ABI, on seeded inputs.

Tolerances (norm-wise relative, |gpu - oracle| / |oracle|):
  FP64            1e-13  (each output is a sum of at most ~30 O(1) terms;
                          FMA contraction and summation order move it by a
                          few ulps)
  FP32            2e-6   (same sums in FP32, u = 6e-8, <= ~30 roundings)
  FP16 sin(sigma) 2e-6   against the oracle fed the same FP16-rounded links;
                          2e-3 against the exact FP64 operator (|d sin| <=
                          2^-12, |dA| <= b 2^-12 ~ 1.1e-4 relative to A ~ 1)
"""
import numpy as np
import pytest

import oracle
from paper_1007_3432_amd import hub, inputs
from tests import hubtest

pytestmark = pytest.mark.gpu

SHAPES = [
    (1, 32, 64), (1, 2, 2), (1, 2, 3), (1, 3, 2), (1, 5, 7), (1, 37, 9), (1, 64, 8),
    (1, 255, 17), (1, 256, 16), (1, 300, 20), (1, 1000, 13), (1, 2048, 512),
    (1, 65, 6), (1, 129, 5), (1, 130, 6), (1, 258, 4), (1, 642, 3),
    # 2^19 sites and more take the marching d=1 tile (8 slices per wavefront):
    # a 6-site last strip and a 3-slice last tile; a one-pair last strip
    # (nx = 2 mod 128); a one-slice last tile
    (1, 1030, 515), (1, 2050, 260), (1, 4096, 129), (1, 130, 4100), (1, 300, 1800),
    (2, 2, 2), (2, 5, 4), (2, 8, 6),
    (3, 2, 2), (3, 3, 5), (3, 4, 6), (3, 8, 80), (3, 5, 3), (3, 16, 160),
]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    hubtest.ensure_built()
    oracle.set_threads(16)


def _lat(d, nx, nt, **kw):
    o = oracle.Lattice(d, nx, nt, **kw)
    return o, hub.lattice(d, nx, nt, o.t_hop, o.dtau, o.U, o.mu)


def _f16_links_reference(olat, sigma):
    """A from FP16-rounded sin(sigma_{s-1}), evaluated in FP64: the operator
    the FP16-link kernels apply."""
    vs, nt = olat.vs, olat.nt
    sig = sigma.reshape(nt, vs)
    s16 = np.sin(np.roll(sig, 1, axis=0)).astype(np.float16).astype(np.float64)
    b = oracle.hs_coupling(olat.dtau, olat.U)
    l = np.exp(olat.dtau * olat.mu) * (1 + b * s16)
    l[1:] *= -1
    return l.reshape(-1)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "d%d_%dx%d" % s)
def test_links_parity(shape):
    d, nx, nt = shape
    olat, lat = _lat(d, nx, nt, mu=0.1)
    hubtest.log_case(f"links {shape}")
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=1)
    A_ref = oracle.links(olat, sigma)
    sig_d = hubtest.to_dev(sigma)
    for link in (hub.F64, hub.F32):
        out = hubtest.empty(lat.volume, link)
        hub.hub_links_from_sigma(lat, sig_d, out, link)
        got = out.double().cpu().numpy()
        # sin() may differ by 1 ulp between libm and the device library, and
        # the device may contract 1 + b sin into an FMA: a few ulps in all.
        tol = 1e-15 if link == hub.F64 else 1.2e-7
        assert np.max(np.abs(got - A_ref) / np.abs(A_ref)) <= tol
    out = hubtest.empty(lat.volume, hub.F16)
    hub.hub_links_from_sigma(lat, sig_d, out, hub.F16)
    vs = nx ** d
    expect = np.sin(np.roll(sigma.reshape(nt, vs), 1, axis=0)).reshape(-1).astype(np.float16)
    np.testing.assert_array_equal(out.cpu().numpy(), expect)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "d%d_%dx%d" % s)
def test_apply_fp64_parity(shape):
    d, nx, nt = shape
    olat, lat = _lat(d, nx, nt)
    hubtest.log_case(f"apply fp64 {shape}")
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=2)
    x = inputs.random_vector(olat.volume, 3)
    A = oracle.links(olat, sigma)
    A_d, x_d = hubtest.to_dev(A), hubtest.to_dev(x)
    y_d = hubtest.empty(lat.volume, hub.F64)
    hub.hub_apply_M(lat, A_d, hub.F64, hub.F64, x_d, y_d, 0)
    assert hubtest.rel_err(y_d.cpu().numpy(), oracle.apply_M(olat, A, x)) <= 1e-13
    hub.hub_apply_M(lat, A_d, hub.F64, hub.F64, x_d, y_d, 1)
    assert hubtest.rel_err(y_d.cpu().numpy(), oracle.apply_Mt(olat, A, x)) <= 1e-13
    hub.hub_apply_MtM(lat, A_d, hub.F64, hub.F64, x_d, y_d)
    z_ref = oracle.apply_MtM(olat, A, x)
    z = y_d.cpu().numpy()
    assert hubtest.rel_err(z, z_ref) <= 1e-13
    # element-wise as well: no site may be far off while the norm hides it
    assert np.max(np.abs(z - z_ref)) <= 1e-13 * np.max(np.abs(z_ref))


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "d%d_%dx%d" % s)
def test_apply_fp32_and_fp16_links(shape):
    d, nx, nt = shape
    olat, lat = _lat(d, nx, nt, mu=-0.05)
    hubtest.log_case(f"apply fp32/fp16 {shape}")
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=4)
    x = inputs.random_vector(olat.volume, 5)
    A = oracle.links(olat, sigma)
    A16 = _f16_links_reference(olat, sigma)
    sig_d = hubtest.to_dev(sigma)
    x32 = hubtest.to_dev(x.astype(np.float32))
    xr = x32.double().cpu().numpy()  # the FP32 input exactly
    out = hubtest.empty(lat.volume, hub.F32)
    for link, Aref, tol_exact in ((hub.F32, A, 2e-6), (hub.F16, A16, 2e-3)):
        links = hubtest.empty(lat.volume, link)
        hub.hub_links_from_sigma(lat, sig_d, links, link)
        for transpose, ref in ((0, oracle.apply_M), (1, oracle.apply_Mt)):
            hub.hub_apply_M(lat, links, link, hub.F32, x32, out, transpose)
            got = out.double().cpu().numpy()
            assert hubtest.rel_err(got, ref(olat, Aref, xr)) <= 2e-6
        hub.hub_apply_MtM(lat, links, link, hub.F32, x32, out)
        got = out.double().cpu().numpy()
        assert hubtest.rel_err(got, oracle.apply_MtM(olat, Aref, xr)) <= 2e-6
        assert hubtest.rel_err(got, oracle.apply_MtM(olat, A, xr)) <= tol_exact


def test_apply_full_size_c3_fp64():
    """d=3, 32^3 x 256 (8.4M sites) in the launch configuration the benchmark
    uses, against the oracle on every site."""
    d, nx, nt = 3, 32, 256
    olat, lat = _lat(d, nx, nt)
    hubtest.log_case("apply fp64 c3 full")
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=0)
    x = inputs.random_vector(olat.volume, 6)
    A = oracle.links(olat, sigma)
    A_d, x_d = hubtest.to_dev(A), hubtest.to_dev(x)
    z_d = hubtest.empty(lat.volume, hub.F64)
    hub.hub_apply_MtM(lat, A_d, hub.F64, hub.F64, x_d, z_d)
    assert hubtest.rel_err(z_d.cpu().numpy(), oracle.apply_MtM(olat, A, x)) <= 1e-13


@pytest.mark.parametrize("shape", [(3, 32, 256), (3, 64, 16)], ids=["32x256", "64x16"])
def test_apply_d3_unrolled_march(shape):
    """Lattices on which every block of the bare FP64 product marches exactly
    16 slices take the completely unrolled march with two slices in flight:
    element-wise against the oracle on every site."""
    d, nx, nt = shape
    olat, lat = _lat(d, nx, nt, mu=0.02)
    hubtest.log_case(f"apply fp64 unrolled march {shape}")
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=9)
    x = inputs.random_vector(olat.volume, 10)
    A = oracle.links(olat, sigma)
    z_d = hubtest.empty(lat.volume, hub.F64)
    hub.hub_apply_MtM(lat, hubtest.to_dev(A), hub.F64, hub.F64, hubtest.to_dev(x), z_d)
    z, z_ref = z_d.cpu().numpy(), oracle.apply_MtM(olat, A, x)
    assert hubtest.rel_err(z, z_ref) <= 1e-13
    assert np.max(np.abs(z - z_ref)) <= 1e-13 * np.max(np.abs(z_ref))


@pytest.mark.parametrize("vec", [hub.F64, hub.F32], ids=["f64", "f32"])
def test_apply_d3_nx64(vec):
    """d=3, 64^3 x 4 (1 048 576 sites): the default 64 x 4 x 4 tile of the
    fused d = 3 sweep, element-wise against the oracle."""
    d, nx, nt = 3, 64, 4
    olat, lat = _lat(d, nx, nt)
    hubtest.log_case(f"apply d3 nx64 vec={vec}")
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=11)
    x = inputs.random_vector(olat.volume, 12)
    A = oracle.links(olat, sigma)
    if vec == hub.F64:
        A_d, x_d, xr, tol = hubtest.to_dev(A), hubtest.to_dev(x), x, 1e-13
    else:
        A_d = hubtest.to_dev(A.astype(np.float32))
        x_d = hubtest.to_dev(x.astype(np.float32))
        xr = x.astype(np.float32).astype(np.float64)
        A = A.astype(np.float32).astype(np.float64)
        tol = 2e-6
    z_d = hubtest.empty(lat.volume, vec)
    hub.hub_apply_MtM(lat, A_d, vec, vec, x_d, z_d)
    z = z_d.double().cpu().numpy()
    z_ref = oracle.apply_MtM(olat, A, xr)
    assert hubtest.rel_err(z, z_ref) <= tol
    assert np.max(np.abs(z - z_ref)) <= tol * np.max(np.abs(z_ref))


def test_special_cases():
    """U = 0 (free fermions), t = 0 (decoupled sites), large mu."""
    for kw in (dict(U=0.0), dict(t_hop=0.0), dict(mu=2.0), dict(dtau=0.2, U=-7.915)):
        for shape in ((1, 40, 6), (3, 4, 4)):
            olat, lat = _lat(*shape, **kw)
            hubtest.log_case(f"special {shape} {kw}")
            sigma, _ = inputs.sigma_eta(*shape, seed=8)
            x = inputs.random_vector(olat.volume, 9)
            A = oracle.links(olat, sigma)
            links = hubtest.empty(lat.volume, hub.F64)
            hub.hub_links_from_sigma(lat, hubtest.to_dev(sigma), links, hub.F64)
            z = hubtest.empty(lat.volume, hub.F64)
            hub.hub_apply_MtM(lat, links, hub.F64, hub.F64, hubtest.to_dev(x), z)
            assert hubtest.rel_err(z.cpu().numpy(), oracle.apply_MtM(olat, A, x)) <= 1e-13


def test_repeated_calls_are_deterministic():
    olat, lat = _lat(1, 2048, 512)
    sigma, _ = inputs.sigma_eta(1, 2048, 512, seed=0)
    links = hubtest.empty(lat.volume, hub.F64)
    hub.hub_links_from_sigma(lat, hubtest.to_dev(sigma), links, hub.F64)
    x = hubtest.to_dev(inputs.random_vector(olat.volume, 1))
    z1 = hubtest.empty(lat.volume, hub.F64)
    z2 = hubtest.empty(lat.volume, hub.F64)
    hub.hub_apply_MtM(lat, links, hub.F64, hub.F64, x, z1)
    for _ in range(3):
        hub.hub_apply_MtM(lat, links, hub.F64, hub.F64, x, z2)
    assert bool((z1 == z2).all())
