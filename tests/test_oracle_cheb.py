"""Pins of the oracle's Chebyshev polynomial preconditioner (Sec. 4.2,
Eqs. (13)-(17)) and of preconditioned CG (no GPU).

The independent fact used throughout: with u = (2 l - 1 - eps) / (1 - eps)
the affine map of [eps, 1] onto [-1, 1], the polynomial of Eq. (13) obeys

    1 - l P(l) = T_{2n+1}(u) / T_{2n+1}(u(0)),

T_m the Chebyshev polynomial of the first kind (numpy's chebval).  Its roots
in l are the 2n + 1 points where T_{2n+1}(u) equals T_{2n+1}(u(0)): l = 0 and
the complex z_{2n,k} of Eq. (15); its maximum on (eps, 1] is
1 / |T_{2n+1}(u(0))|, which never exceeds the bound of Eq. (16).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import Lattice
from paper_1007_3432_amd import inputs
from tests import dense


def _p_closed(lam, n, eps):
    """P(l) from the Chebyshev closed form (valid for l > 0)."""
    return dense.cheb_closed_form(lam, n, eps)


def _p_product(lam, n, eps):
    """P(l) from the oracle's roots and normalisation (Eqs. (13)-(15))."""
    z = oracle.cheb_roots(n, eps)
    c = oracle.cheb_norm(n, eps)
    return (c * np.prod(np.asarray(lam)[:, None] - z[None, :], axis=1)).real


def _bound(n, eps):
    q = (1.0 - math.sqrt(eps)) / (1.0 + math.sqrt(eps))
    return 2.0 * q ** (2 * n + 1)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8])
@pytest.mark.parametrize("eps", [0.3, 0.05, 0.01, 0.002])
def test_product_form_equals_chebyshev_closed_form(n, eps):
    lam = np.linspace(eps / 4, 1.0, 2001)
    got = _p_product(lam, n, eps)
    want = _p_closed(lam, n, eps)
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-11


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("eps", [0.1, 0.01, 0.001])
def test_relative_error_bound(n, eps):
    """Eq. (16) on (eps, 1], and near equioscillation: the error reaches
    within a factor 2 of the bound whenever the bound is below 1."""
    lam = np.linspace(eps, 1.0, 40001)
    R = lam * _p_product(lam, n, eps) - 1.0
    b = _bound(n, eps)
    assert np.max(np.abs(R)) <= b * (1 + 1e-9) + 1e-13
    if b < 1.0:
        assert np.max(np.abs(R)) >= 0.5 * b


def test_roots_conjugate_pairs_and_positive_polynomial():
    """z_{2n,2n+1-k} is the conjugate of z_{2n,k}, so P is real; no root is
    real, so P keeps the sign it has at l = (1 + eps)/2, where it is
    2 / (1 + eps) by the normalisation."""
    for n, eps in [(1, 0.1), (4, 0.01), (9, 0.003)]:
        z = oracle.cheb_roots(n, eps)
        assert np.allclose(z, np.conj(z[::-1]), rtol=0, atol=1e-15)
        assert np.all(np.abs(z.imag) > 0)
        h = 0.5 * (1 + eps)
        assert _p_product(np.array([h]), n, eps)[0] == pytest.approx(1.0 / h, rel=1e-13)
        lam = np.linspace(0.0, 1.5, 3001)
        assert np.all(_p_product(lam, n, eps) > 0)


@pytest.mark.parametrize("d,nx,nt", [(1, 6, 8), (3, 2, 4)])
def test_cheb_scale_bounds_spectrum(d, nx, nt):
    lat = Lattice(d, nx, nt)
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=3)
    A = oracle.links(lat, sigma)
    Q = dense.dense_from_apply(lambda v: oracle.apply_MtM(lat, A, v), lat.volume)
    lmax = np.linalg.eigvalsh(Q)[-1]
    assert lmax <= oracle.cheb_scale(lat)
    assert lmax >= 0.3 * oracle.cheb_scale(lat)  # not a vacuous bound


@pytest.mark.parametrize("d,nx,nt,n,eps", [(1, 6, 8, 3, 0.01), (1, 4, 6, 8, 0.002),
                                           (3, 2, 4, 2, 0.05)])
def test_cheb_apply_matches_spectral_form(d, nx, nt, n, eps):
    """P(Q/s) r equals V diag(P(l_i / s)) V^T r from a dense eigen-
    decomposition of Q, with P from the Chebyshev closed form."""
    lat = Lattice(d, nx, nt)
    sigma, eta = inputs.sigma_eta(d, nx, nt, seed=1)
    A = oracle.links(lat, sigma)
    s = oracle.cheb_scale(lat)
    Q = dense.dense_from_apply(lambda v: oracle.apply_MtM(lat, A, v), lat.volume)
    w, Vm = np.linalg.eigh(Q)
    want = Vm @ (_p_closed(w / s, n, eps) * (Vm.T @ eta))
    got = oracle.cheb_apply(lat, A, eta, n, eps, s)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-10


def test_cheb_apply_is_linear_and_symmetric():
    lat = Lattice(1, 8, 6)
    sigma, _ = inputs.sigma_eta(1, 8, 6, seed=2)
    A = oracle.links(lat, sigma)
    a = inputs.random_vector(lat.volume, 11)
    b = inputs.random_vector(lat.volume, 12)
    Pa = oracle.cheb_apply(lat, A, a, 4, 0.01)
    Pb = oracle.cheb_apply(lat, A, b, 4, 0.01)
    assert np.dot(a, Pb) == pytest.approx(np.dot(Pa, b), rel=1e-12)
    Pab = oracle.cheb_apply(lat, A, 2.0 * a - 3.0 * b, 4, 0.01)
    assert np.linalg.norm(Pab - (2.0 * Pa - 3.0 * Pb)) <= 1e-12 * np.linalg.norm(Pab)
    assert np.dot(a, Pa) > 0


@pytest.mark.parametrize("d,nx,nt", [(1, 8, 16), (3, 3, 6)])
def test_pcg_matches_dense_solve_in_fewer_iterations(d, nx, nt):
    lat = Lattice(d, nx, nt)
    sigma, eta = inputs.sigma_eta(d, nx, nt, seed=0)
    A = oracle.links(lat, sigma)
    phi = oracle.apply_Mt(lat, A, eta)
    Q = dense.dense_from_apply(lambda v: oracle.apply_MtM(lat, A, v), lat.volume)
    x_ref = np.linalg.solve(Q, phi)
    cond = np.linalg.cond(Q)
    ev = np.linalg.eigvalsh(Q)
    eps = ev[0] / oracle.cheb_scale(lat)
    _, res_cg = oracle.cg(lat, A, phi, tol=1e-10)
    x, res = oracle.pcg(lat, A, phi, 4, eps, tol=1e-10)
    assert res.converged and not res.breakdown
    assert res.true_rel_resid <= 1e-10
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) <= 2 * cond * 1e-10
    assert res.iters < res_cg.iters


def test_pcg_exact_preconditioner_converges_at_once():
    """When the spectrum of Q/s lies in (eps, 1] and the degree is high, P(Q/s)
    is s Q^{-1} to near machine precision and PCG needs one or two steps."""
    lat = Lattice(1, 4, 4)
    sigma, eta = inputs.sigma_eta(1, 4, 4, seed=4)
    A = oracle.links(lat, sigma)
    Q = dense.dense_from_apply(lambda v: oracle.apply_MtM(lat, A, v), lat.volume)
    ev = np.linalg.eigvalsh(Q)
    s = ev[-1]
    eps = 0.9 * ev[0] / s
    n = 1
    while _bound(n, eps) > 1e-13:
        n += 1
    x, res = oracle.pcg(lat, A, eta, n, eps, tol=1e-10, scale=s)
    assert res.converged and res.iters <= 2


def test_pcg_zero_rhs_and_max_iter():
    lat = Lattice(1, 8, 8)
    A = oracle.links(lat, np.zeros(lat.volume))
    x, res = oracle.pcg(lat, A, np.zeros(lat.volume), 2, 0.01)
    assert res.converged and res.iters == 0 and not np.any(x)
    sigma, eta = inputs.sigma_eta(1, 8, 8, seed=0)
    A = oracle.links(lat, sigma)
    x, res = oracle.pcg(lat, A, eta, 1, 0.01, tol=1e-14, max_iter=2)
    assert not res.converged and res.iters == 2
