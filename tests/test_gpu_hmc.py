"""Parity of the HMC pieces (Sec. 4.1, phi-algorithm) with the oracle, through
the C ABI: the force kernel, the leapfrog MD trajectory and the HMC
trajectory with its Metropolis step.

Tolerances:
  force      1e-13 relative (norm-wise and element-wise against max|F|): the
             same stencil sums plus one sin/cos per site, FMA contraction and
             1-ulp differences of the device sin/cos;
  MD / HMC   every force evaluation solves Q x = phi to the same true
             residual on both sides but not to the same bits (CG iterates
             depend on rounding order), so the solutions differ by up to
             ~2 cond(Q) tol relative; at tol = 1e-12 and these lattices that
             moves pi and sigma by < 1e-9 over a trajectory (checked at 1e-8)
             and H by < 1e-9 relative.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1007_3432_amd import hub, inputs
from tests import hubtest

pytestmark = pytest.mark.gpu

FORCE_SHAPES = [(1, 32, 64), (1, 2, 2), (1, 300, 37), (2, 6, 10), (3, 2, 2), (3, 5, 7),
                (3, 8, 20), (1, 2048, 512)]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    hubtest.ensure_built()
    oracle.set_threads(16)


def _lat(d, nx, nt, **kw):
    o = oracle.Lattice(d, nx, nt, **kw)
    return o, hub.lattice(d, nx, nt, o.t_hop, o.dtau, o.U, o.mu)


def _draw(V, seed):
    rng = np.random.default_rng(seed)
    sigma = rng.uniform(-math.pi, math.pi, V)
    eta = rng.standard_normal(V) / math.sqrt(2.0)
    pi = rng.standard_normal(V)
    return sigma, eta, pi


@pytest.mark.parametrize("shape", FORCE_SHAPES, ids=lambda s: "d%d_%dx%d" % s)
def test_force_parity(shape):
    d, nx, nt = shape
    olat, lat = _lat(d, nx, nt, mu=0.05)
    hubtest.log_case(f"hmc force {shape}")
    sigma, _, _ = _draw(olat.volume, 31)
    x = inputs.random_vector(olat.volume, 32)
    F_d = hubtest.empty(lat.volume, hub.F64)
    hub.hub_hmc_force(lat, hubtest.to_dev(sigma), hubtest.to_dev(x), F_d)
    F = F_d.cpu().numpy()
    F_ref = oracle.force(olat, sigma, x)
    assert hubtest.rel_err(F, F_ref) <= 1e-13
    assert np.max(np.abs(F - F_ref)) <= 1e-13 * np.max(np.abs(F_ref))


def test_force_full_size_c3():
    olat, lat = _lat(3, 32, 256)
    hubtest.log_case("hmc force c3 full")
    sigma, _, _ = _draw(olat.volume, 33)
    x = inputs.random_vector(olat.volume, 34)
    F_d = hubtest.empty(lat.volume, hub.F64)
    hub.hub_hmc_force(lat, hubtest.to_dev(sigma), hubtest.to_dev(x), F_d)
    assert hubtest.rel_err(F_d.cpu().numpy(), oracle.force(olat, sigma, x)) <= 1e-13


MD_CASES = [((1, 32, 16), 0.02, 8), ((3, 4, 8), 0.02, 6), ((1, 6, 2), 0.05, 5)]


@pytest.mark.parametrize("shape,eps,n", MD_CASES, ids=["d1_32x16", "d3_4x8", "d1_6x2"])
def test_md_trajectory_matches_oracle(shape, eps, n):
    olat, lat = _lat(*shape)
    hubtest.log_case(f"md {shape} eps={eps} n={n}")
    sigma, eta, pi = _draw(olat.volume, 41)
    A = oracle.links(olat, sigma)
    phi = oracle.apply_Mt(olat, A, eta)
    s_ref, p_ref, r_ref = oracle.md(olat, sigma, pi, phi, eps, n, tol=1e-12)
    sig_d, pi_d = hubtest.to_dev(sigma), hubtest.to_dev(pi)
    st = hub.hub_md_trajectory(lat, sig_d, pi_d, hubtest.to_dev(phi),
                               hub.md_opts(n, eps, hub.cg_opts(hub.F64, tol=1e-12)))
    assert st["status"] == "HUB_OK" and st["solves"] == n + 1 == r_ref.solves
    assert np.max(np.abs(sig_d.cpu().numpy() - s_ref)) <= 1e-8
    assert np.max(np.abs(pi_d.cpu().numpy() - p_ref)) <= 1e-8
    assert st["h_start"] == pytest.approx(r_ref.h_start, rel=1e-9)
    assert st["h_end"] == pytest.approx(r_ref.h_end, rel=1e-9)
    assert abs(st["delta_h"] - r_ref.delta_h) <= 1e-8 * max(1.0, abs(r_ref.h_start))
    assert abs(st["cg_iters"] - r_ref.cg_iters) <= 0.05 * r_ref.cg_iters + 3 * (n + 1)


def test_md_trajectory_mixed_precision_solves():
    """Force evaluations by the mixed-precision solver (FP32 bulk, FP64 true
    residual): the same trajectory as the oracle's FP64 one, to the accuracy
    of a 1e-10 solve."""
    olat, lat = _lat(1, 64, 32)
    sigma, eta, pi = _draw(olat.volume, 43)
    A = oracle.links(olat, sigma)
    phi = oracle.apply_Mt(olat, A, eta)
    s_ref, p_ref, r_ref = oracle.md(olat, sigma, pi, phi, 0.02, 6, tol=1e-10)
    sig_d, pi_d = hubtest.to_dev(sigma), hubtest.to_dev(pi)
    st = hub.hub_md_trajectory(lat, sig_d, pi_d, hubtest.to_dev(phi),
                               hub.md_opts(6, 0.02, hub.cg_opts(hub.F32, hub.F32)))
    assert st["status"] == "HUB_OK"
    assert np.max(np.abs(sig_d.cpu().numpy() - s_ref)) <= 1e-6
    assert np.max(np.abs(pi_d.cpu().numpy() - p_ref)) <= 1e-6
    assert abs(st["delta_h"] - r_ref.delta_h) <= 1e-6 * abs(r_ref.h_start)


def test_md_trajectory_is_reversible_on_gpu():
    olat, lat = _lat(3, 4, 6)
    sigma, eta, pi = _draw(olat.volume, 47)
    A = oracle.links(olat, sigma)
    phi_d = hubtest.to_dev(oracle.apply_Mt(olat, A, eta))
    sig_d, pi_d = hubtest.to_dev(sigma), hubtest.to_dev(pi)
    opts = hub.md_opts(10, 0.03, hub.cg_opts(hub.F64, tol=1e-13))
    st1 = hub.hub_md_trajectory(lat, sig_d, pi_d, phi_d, opts)
    assert np.max(np.abs(sig_d.cpu().numpy() - sigma)) > 1e-3
    pi_d.neg_()
    st2 = hub.hub_md_trajectory(lat, sig_d, pi_d, phi_d, opts)
    assert np.max(np.abs(sig_d.cpu().numpy() - sigma)) <= 1e-9
    assert np.max(np.abs(pi_d.cpu().numpy() + pi)) <= 1e-9
    assert st2["h_end"] == pytest.approx(st1["h_start"], rel=1e-11)


@pytest.mark.parametrize("shape", [(1, 16, 12), (3, 3, 6)], ids=["d1_16x12", "d3_3x6"])
def test_hmc_trajectory_matches_oracle(shape):
    olat, lat = _lat(*shape)
    hubtest.log_case(f"hmc trajectory {shape}")
    sigma, eta, pi = _draw(olat.volume, 53)
    eps, n = 0.05, 6
    opts = hub.md_opts(n, eps, hub.cg_opts(hub.F64, tol=1e-12))
    s_ref, r_ref = oracle.hmc(olat, sigma, eta, pi, 0.0, eps, n, tol=1e-12)
    assert r_ref.accepted
    sig_d = hubtest.to_dev(sigma)
    eta_d, pi_d = hubtest.to_dev(eta), hubtest.to_dev(pi)
    st = hub.hub_hmc_trajectory(lat, sig_d, eta_d, pi_d, 0.0, opts)
    assert st["accepted"] and st["status"] == "HUB_OK"
    assert np.max(np.abs(sig_d.cpu().numpy() - s_ref)) <= 1e-8
    assert abs(st["delta_h"] - r_ref.delta_h) <= 1e-8 * max(1.0, abs(r_ref.h_start))
    # pi0 and eta are inputs only
    np.testing.assert_array_equal(pi_d.cpu().numpy(), pi)
    np.testing.assert_array_equal(eta_d.cpu().numpy(), eta)
    # Metropolis: u just above exp(-dH) rejects (field untouched, bitwise),
    # u just below accepts; for dH <= 0 every u < 1 accepts.
    boltz = math.exp(-r_ref.delta_h)
    sig2 = hubtest.to_dev(sigma)
    if boltz < 1.0:
        st2 = hub.hub_hmc_trajectory(lat, sig2, eta_d, pi_d, min(1.0, boltz * 1.001), opts)
        assert not st2["accepted"]
        np.testing.assert_array_equal(sig2.cpu().numpy(), sigma)
    else:
        st2 = hub.hub_hmc_trajectory(lat, sig2, eta_d, pi_d, 0.999, opts)
        assert st2["accepted"]


def test_hmc_failed_solve_leaves_field_untouched():
    olat, lat = _lat(1, 32, 16)
    sigma, eta, pi = _draw(olat.volume, 59)
    sig_d = hubtest.to_dev(sigma)
    opts = hub.md_opts(3, 0.02, hub.cg_opts(hub.F64, max_iter=3))
    st = hub.hub_hmc_trajectory(lat, sig_d, hubtest.to_dev(eta), hubtest.to_dev(pi), 0.0, opts,
                                raise_on_noconv=False)
    assert st["status"] == "HUB_E_NOCONV" and not st["accepted"]
    np.testing.assert_array_equal(sig_d.cpu().numpy(), sigma)
