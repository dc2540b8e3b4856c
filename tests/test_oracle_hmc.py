"""Pins of the oracle's Hybrid Monte Carlo pieces (Sec. 4.1, the
phi-algorithm): the force dS_p/dsigma, the pseudofermion action, the leapfrog
MD trajectory and the Metropolis step.

What fixes them independently of the oracle's own code:
  * the force is the gradient of S_p(sigma) = phi^T Q(sigma)^{-1} phi; central
    finite differences of S_p with Q built densely from the operator and a
    numpy solve must reproduce it (a wrong slice, sign, factor or cos/sin
    fails);
  * with phi = M^T eta, S_p = eta^T M Q^{-1} M^T eta = eta . eta exactly;
  * leapfrog is time-reversible: integrating from (sigma_1, -pi_1) retraces
    the path back to (sigma_0, -pi_0);
  * leapfrog's energy error over a fixed trajectory length is O(eps^2);
  * Metropolis keeps the end point iff u < exp(-dH), else restores sigma.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1007_3432_amd import inputs
from tests import dense


def _setup(shape, seed=0, **kw):
    lat = oracle.Lattice(*shape, **kw)
    rng = np.random.default_rng(seed)
    sigma = rng.uniform(-math.pi, math.pi, lat.volume)
    eta = rng.standard_normal(lat.volume) / math.sqrt(2.0)
    pi = rng.standard_normal(lat.volume)
    return lat, sigma, eta, pi


def _dense_M(lat, sigma):
    A = oracle.links(lat, sigma)
    return dense.dense_from_apply(lambda v: oracle.apply_M(lat, A, v), lat.volume)


def _action(lat, sigma, phi):
    M = _dense_M(lat, sigma)
    return float(phi @ np.linalg.solve(M.T @ M, phi))


@pytest.mark.parametrize("shape,kw", [((1, 4, 5), {}), ((1, 3, 4), dict(mu=0.3)),
                                      ((2, 3, 3), {}), ((3, 2, 3), dict(U=-4.0))],
                         ids=["d1_4x5", "d1_3x4_mu", "d2_3x3", "d3_2x3_U4"])
def test_force_is_gradient_of_action(shape, kw):
    lat, sigma, eta, _ = _setup(shape, seed=3, **kw)
    M = _dense_M(lat, sigma)
    phi = M.T @ eta
    x = np.linalg.solve(M.T @ M, phi)
    F = oracle.force(lat, sigma, x)
    h = 1e-5
    fd = np.empty(lat.volume)
    for j in range(lat.volume):
        sp, sm = sigma.copy(), sigma.copy()
        sp[j] += h
        sm[j] -= h
        fd[j] = (_action(lat, sp, phi) - _action(lat, sm, phi)) / (2 * h)
    assert np.max(np.abs(F - fd)) <= 1e-6 * np.max(np.abs(fd)), np.max(np.abs(F - fd))
    # every site carries a force: no component is silently dropped
    assert np.all(np.abs(F) > 0)


def test_force_vanishes_without_coupling():
    lat, sigma, eta, _ = _setup((1, 6, 4), U=0.0)
    x = inputs.random_vector(lat.volume, 1)
    assert np.all(oracle.force(lat, sigma, x) == 0.0)


def test_action_of_heatbath_field_is_eta_squared():
    lat, sigma, eta, _ = _setup((1, 16, 8), seed=5)
    A = oracle.links(lat, sigma)
    phi = oracle.apply_Mt(lat, A, eta)
    _, _, res = oracle.md(lat, sigma, np.zeros(lat.volume), phi, 0.0, 1, tol=1e-13)
    # with pi = 0, H_start = S_p
    assert res.h_start == pytest.approx(float(eta @ eta), rel=1e-10)


@pytest.mark.parametrize("shape", [(1, 8, 6), (3, 3, 4)], ids=["d1_8x6", "d3_3x4"])
def test_leapfrog_is_reversible(shape):
    lat, sigma, eta, pi = _setup(shape, seed=7)
    A = oracle.links(lat, sigma)
    phi = oracle.apply_Mt(lat, A, eta)
    s1, p1, r1 = oracle.md(lat, sigma, pi, phi, 0.02, 10, tol=1e-13)
    assert r1.solves == 11 and not r1.failed
    assert np.max(np.abs(s1 - sigma)) > 1e-3          # it moved
    s2, p2, r2 = oracle.md(lat, s1, -p1, phi, 0.02, 10, tol=1e-13)
    assert np.max(np.abs(s2 - sigma)) <= 1e-9
    assert np.max(np.abs(p2 + pi)) <= 1e-9
    # H is a function of the phase-space point only
    assert r2.h_start == pytest.approx(r1.h_end, rel=1e-12)
    assert r2.h_end == pytest.approx(r1.h_start, rel=1e-12)


def test_energy_error_is_second_order_in_step():
    lat, sigma, eta, pi = _setup((1, 8, 8), seed=11)
    A = oracle.links(lat, sigma)
    phi = oracle.apply_Mt(lat, A, eta)
    T = 0.5
    dh = []
    for n in (10, 20, 40):
        _, _, r = oracle.md(lat, sigma, pi, phi, T / n, n, tol=1e-13)
        dh.append(abs(r.delta_h))
    assert dh[0] > 1e-6            # large enough to be above solver noise
    for a, b in zip(dh, dh[1:]):
        assert 0.18 <= b / a <= 0.32, dh


def test_metropolis_accepts_below_and_rejects_above_boltzmann_factor():
    lat, sigma, eta, pi = _setup((1, 6, 6), seed=13)
    eps, n = 0.2, 4
    s_acc, r = oracle.hmc(lat, sigma, eta, pi, 0.0, eps, n, tol=1e-12)
    assert r.accepted
    A = oracle.links(lat, sigma)
    phi = oracle.apply_Mt(lat, A, eta)
    s_end, _, r_md = oracle.md(lat, sigma, pi, phi, eps, n, tol=1e-12)
    np.testing.assert_array_equal(s_acc, s_end)
    assert r.delta_h == r_md.delta_h
    boltz = math.exp(-r.delta_h)
    if boltz < 1.0:
        s_rej, r2 = oracle.hmc(lat, sigma, eta, pi, boltz * (1 + 1e-9), eps, n, tol=1e-12)
        assert not r2.accepted
        np.testing.assert_array_equal(s_rej, sigma)
        _, r3 = oracle.hmc(lat, sigma, eta, pi, boltz * (1 - 1e-9), eps, n, tol=1e-12)
        assert r3.accepted
    else:
        _, r2 = oracle.hmc(lat, sigma, eta, pi, 0.999999, eps, n, tol=1e-12)
        assert r2.accepted
