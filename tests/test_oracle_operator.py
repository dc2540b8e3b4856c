"""Pins of the CPU oracle's operator against what the paper and mathematics
fix (no GPU).  Each test names the passage it follows."""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import Lattice
from paper_1007_3432_amd import inputs
from tests import dense


def _dense_M(lat, A):
    return dense.dense_from_apply(lambda v: oracle.apply_M(lat, A, v), lat.volume)


def _dense_Mt(lat, A):
    return dense.dense_from_apply(lambda v: oracle.apply_Mt(lat, A, v), lat.volume)


# --- Hubbard-Stratonovich coupling (Sec. 2, Eq. (6); compact continuous form)

@pytest.mark.parametrize("dtau", [0.05, 0.1, 0.37])
@pytest.mark.parametrize("U", [0.0, -0.1, -2.0, -4.0, -7.915])
def test_hs_quadrature_identity(dtau, U):
    """(1/2pi) Int dsigma (1 + b sin s n1)(1 + b sin s n2) = exp(-dtau U n1 n2).
    The trapezoid rule on N equispaced points is exact for trigonometric
    polynomials of degree < N, so the integral is evaluated to rounding."""
    b = oracle.hs_coupling(dtau, U)
    s = np.linspace(-math.pi, math.pi, 64, endpoint=False)
    for n1 in (0, 1):
        for n2 in (0, 1):
            integral = np.mean((1 + b * np.sin(s) * n1) * (1 + b * np.sin(s) * n2))
            assert integral == pytest.approx(math.exp(-dtau * U * n1 * n2), rel=1e-14)


def test_hs_repulsive_rejected():
    assert math.isnan(oracle.hs_coupling(0.05, 1.0))


# --- Block form (Eqs. (7)-(9)) versus the stencil form (Eq. (10))

BLOCK_CASES = [
    (1, 5, 4, 1.0, 0.05, -2.0, 0.0),
    (1, 2, 3, 1.0, 0.05, -2.0, 0.3),   # nx = 2: n+e and n-e coincide
    (2, 3, 3, 1.0, 0.1, -4.0, 0.0),
    (3, 3, 3, 1.0, 0.05, -2.0, -0.2),
    (3, 2, 2, 0.7, 0.2, -1.0, 0.0),
    (1, 4, 7, 1.3, 0.08, -7.915, 0.1),
]


@pytest.mark.parametrize("case", BLOCK_CASES)
def test_stencil_equals_premultiplied_block_form(case):
    """diag_tau(exp(dtau K)) M_block has diagonal blocks exp(dtau K) and
    off-diagonal blocks -exp(-dtau V[sigma]) (+ on the wrap).  The stencil
    form replaces exp(dtau K) by 1 + dtau K, so
        M_stencil - diag(exp(dtau K)) M_block = diag(1 + dtau K - exp(dtau K))
    exactly.  Any error in the sign of the wrap, in which slice's field sits on
    a link, or in the hopping term fails this."""
    d, nx, nt, t, dtau, U, mu = case
    lat = Lattice(d, nx, nt, t, dtau, U, mu)
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=7)
    A = oracle.links(lat, sigma)
    Mst = _dense_M(lat, A)
    Mb = dense.block_form_M(d, nx, nt, t, dtau, U, mu, sigma)
    K = dense.kinetic_matrix(d, nx, t)
    Vs = nx ** d
    E = scipy.linalg.block_diag(*[scipy.linalg.expm(dtau * K)] * nt)
    R = scipy.linalg.block_diag(*[np.eye(Vs) + dtau * K - scipy.linalg.expm(dtau * K)] * nt)
    assert np.max(np.abs(Mst - E @ Mb - R)) < 1e-14


def test_trotter_residual_is_second_order():
    """The stencil form agrees with the block form to O(dtau^2) (Sec. 2, the
    order the paper gives for the stencil): |1 + dtau K - exp(dtau K)| shrinks
    4x per halving."""
    K = dense.kinetic_matrix(3, 4, 1.0)
    errs = []
    for dtau in (0.02, 0.01, 0.005):
        R = np.eye(K.shape[0]) + dtau * K - scipy.linalg.expm(dtau * K)
        errs.append(np.linalg.norm(R, 2))
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.05)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.03)


def test_links_sign_and_slice():
    """A_{n,s} = -l(sigma_{n,s-1}) for s >= 1 and +l(sigma_{n,nt-1}) for s = 0,
    checked entry by entry on a lattice where only one sigma is non-zero."""
    lat = Lattice(1, 3, 4, 1.0, 0.05, -2.0, 0.0)
    sigma = np.zeros(lat.volume)
    sigma[1 + 3 * 2] = 0.5 * math.pi        # site n=1, slice 2
    A = oracle.links(lat, sigma)
    b = oracle.hs_coupling(0.05, -2.0)
    expect = -np.ones(lat.volume)
    expect[0:3] = 1.0
    expect[1 + 3 * 3] = -(1.0 + b)          # read by slice 3
    np.testing.assert_array_equal(A, expect)


# --- Plane waves at constant field (translation invariance)

@pytest.mark.parametrize("d,nx,nt,mu", [(1, 6, 8, 0.0), (1, 2, 5, 0.2),
                                        (3, 4, 6, 0.0), (2, 3, 4, -0.3)])
def test_plane_wave_eigenvalues(d, nx, nt, mu):
    """With sigma constant, M psi = (a_k - f e^{-i w}) psi for
    psi_{n,s} = exp(i (k.n + w s)), w antiperiodic."""
    lat = Lattice(d, nx, nt, 1.0, 0.05, -2.0, mu)
    s0 = 0.4
    A = oracle.links(lat, np.full(lat.volume, s0))
    f = math.exp(0.05 * mu) * (1 + oracle.hs_coupling(0.05, -2.0) * math.sin(s0))
    cs = np.array(dense.coords(d, nx))
    for ms, l, lam in dense.plane_wave_lambdas(d, nx, nt, 1.0, 0.05, f)[::3]:
        k = 2 * np.pi * np.array(ms) / nx
        w = np.pi * (2 * l + 1) / nt
        phase_n = cs @ k
        psi = np.concatenate([np.exp(1j * (phase_n + w * s)) for s in range(nt)])
        Mpsi = oracle.apply_M(lat, A, psi.real) + 1j * oracle.apply_M(lat, A, psi.imag)
        assert np.max(np.abs(Mpsi - lam * psi)) < 1e-13


@pytest.mark.parametrize("d,nx,nt", [(1, 8, 6), (3, 3, 4), (1, 2, 3)])
def test_Q_spectrum_closed_form(d, nx, nt):
    """Eigenvalues of Q = M^T M at constant field are |a_k - f e^{-iw}|^2."""
    lat = Lattice(d, nx, nt)
    A = oracle.links(lat, np.full(lat.volume, -1.1))
    f = 1 + oracle.hs_coupling(0.05, -2.0) * math.sin(-1.1)
    Q = dense.dense_from_apply(lambda v: oracle.apply_MtM(lat, A, v), lat.volume)
    ev = np.linalg.eigvalsh(0.5 * (Q + Q.T))
    expect = np.sort([abs(lam) ** 2 for _, _, lam in
                      dense.plane_wave_lambdas(d, nx, nt, 1.0, 0.05, f)])
    np.testing.assert_allclose(ev, expect, rtol=0, atol=1e-13)


# --- Determinant (Sec. 2, Eq. (6)-(7))

def _logdet_closed_form(d, nx, nt, kappa, f):
    tot = 0.0
    for ms in np.ndindex(*([nx] * d)):
        a = 1 - 2 * kappa * sum(math.cos(2 * math.pi * m / nx) for m in ms)
        tot += math.log(a ** nt + f ** nt)
    return tot


@pytest.mark.parametrize("d,nx,nt", [(3, 4, 6), (1, 7, 5), (1, 2, 4), (3, 2, 3)])
def test_logdet_constant_field(d, nx, nt):
    """det M = prod_k (a_k^{nt} + f^{nt}) at constant field: the '+' is the
    antiperiodic wrap of Eq. (7)."""
    lat = Lattice(d, nx, nt)
    s0 = 0.9
    A = oracle.links(lat, np.full(lat.volume, s0))
    f = 1 + oracle.hs_coupling(0.05, -2.0) * math.sin(s0)
    sign, logdet = np.linalg.slogdet(_dense_M(lat, A))
    assert sign == 1.0
    assert logdet == pytest.approx(_logdet_closed_form(d, nx, nt, 0.05, f), abs=1e-11)


@pytest.mark.parametrize("d,nx,nt,mu", [(1, 5, 6, 0.0), (3, 3, 4, 0.0),
                                        (1, 2, 5, 0.1), (3, 2, 3, 0.0),
                                        (2, 3, 5, -0.2)])
def test_logdet_determinant_identity(d, nx, nt, mu):
    """For any field, det M = det(W)^{nt} det(1 + G_{nt-1} ... G_0) with
    W = 1 + dtau K and G_s = W^{-1} exp(dtau mu) diag(1 + b sin sigma_s):
    block Gaussian elimination of the cyclic block-bidiagonal M, written with
    dense numpy matrices and compared with LU (slogdet)."""
    lat = Lattice(d, nx, nt, 1.0, 0.05, -2.0, mu)
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=3)
    A = oracle.links(lat, sigma)
    Vs = nx ** d
    W = np.eye(Vs) + 0.05 * dense.kinetic_matrix(d, nx, 1.0)
    Winv = np.linalg.inv(W)
    b = math.sqrt(2 * (math.exp(0.1) - 1))
    sig = sigma.reshape(nt, Vs)
    P = np.eye(Vs)
    for s in range(nt):
        P = Winv @ np.diag(math.exp(0.05 * mu) * (1 + b * np.sin(sig[s]))) @ P
    s1, l1 = np.linalg.slogdet(W)
    s2, l2 = np.linalg.slogdet(np.eye(Vs) + P)
    sign, logdet = np.linalg.slogdet(_dense_M(lat, A))
    assert sign == s1 ** nt * s2
    assert logdet == pytest.approx(nt * l1 + l2, abs=1e-10)


def test_logdet_no_hopping():
    """Delta tau t = 0: M splits into independent cyclic chains per site and
    det M = prod_n (1 + prod_s l_{n,s})."""
    lat = Lattice(1, 4, 5, 0.0, 0.05, -2.0, 0.0)
    sigma, _ = inputs.sigma_eta(1, 4, 5, seed=11)
    A = oracle.links(lat, sigma)
    ell = np.abs(A).reshape(5, 4)
    expect = np.sum(np.log(1 + np.prod(ell, axis=0)))
    sign, logdet = np.linalg.slogdet(_dense_M(lat, A))
    assert sign == 1.0 and logdet == pytest.approx(expect, abs=1e-13)


@pytest.mark.parametrize("d,nx,mu", [(1, 6, 0.0), (1, 5, 0.3), (2, 3, -0.2)])
def test_trotter_limit_free_fermions(d, nx, mu):
    """U = 0: as dtau -> 0 at fixed beta = nt dtau, det M tends to
    det(1 + exp(-beta (K - mu))), the one-spin factor of the free grand
    partition function Tr exp(-beta (H - mu N)) of Eq. (4); the stencil form
    is first order in dtau, so the error halves when nt doubles.  K is built
    from Eq. (9) independently of the oracle."""
    beta = 2.0
    K = dense.kinetic_matrix(d, nx, 1.0)
    ev = np.linalg.eigvalsh(K)
    exact = float(np.sum(np.log1p(np.exp(-beta * (ev - mu)))))
    logdets = []
    for nt in (8, 16, 32, 64):
        lat = Lattice(d, nx, nt, 1.0, beta / nt, 0.0, mu)
        sigma, _ = inputs.sigma_eta(d, nx, nt, seed=nt)
        A = oracle.links(lat, sigma)
        sign, logdet = np.linalg.slogdet(_dense_M(lat, A))
        assert sign == 1.0
        logdets.append(logdet)
    errs = [l - exact for l in logdets]
    for a, b in zip(errs, errs[1:]):
        assert 0.45 <= b / a <= 0.6, errs   # first order, same sign
    # Richardson extrapolation of the first-order error lands on the limit
    assert abs(2 * logdets[-1] - logdets[-2] - exact) <= 5e-3 * abs(exact)


def test_free_fermions_U0():
    """U = 0: b = 0, every link factor equals exp(dtau mu) whatever sigma."""
    lat = Lattice(3, 3, 4, 1.0, 0.05, 0.0, 0.4)
    sigma, _ = inputs.sigma_eta(3, 3, 4, seed=5)
    A = oracle.links(lat, sigma)
    np.testing.assert_allclose(np.abs(A), math.exp(0.02), rtol=1e-15)


# --- Transpose and Q

@pytest.mark.parametrize("d,nx,nt", [(1, 5, 4), (3, 3, 3), (1, 2, 3), (2, 4, 2)])
def test_Mt_is_dense_transpose(d, nx, nt):
    lat = Lattice(d, nx, nt)
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=2)
    A = oracle.links(lat, sigma)
    np.testing.assert_array_equal(_dense_Mt(lat, A), _dense_M(lat, A).T)


@pytest.mark.parametrize("d,nx,nt", [(1, 64, 32), (3, 8, 8), (3, 5, 7)])
def test_adjoint_identity(d, nx, nt):
    """<y, M x> = <M^T y, x> on random vectors."""
    lat = Lattice(d, nx, nt)
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=4)
    A = oracle.links(lat, sigma)
    x = inputs.random_vector(lat.volume, 1)
    y = inputs.random_vector(lat.volume, 2)
    lhs = np.dot(y, oracle.apply_M(lat, A, x))
    rhs = np.dot(oracle.apply_Mt(lat, A, y), x)
    assert lhs == pytest.approx(rhs, rel=1e-13)


@pytest.mark.parametrize("d,nx,nt", [(1, 6, 6), (3, 3, 4)])
def test_Q_symmetric_positive(d, nx, nt):
    """Q = M^T M is symmetric positive definite (Sec. 4.1) and
    <x, Q x> = |M x|^2."""
    lat = Lattice(d, nx, nt)
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=9)
    A = oracle.links(lat, sigma)
    Q = dense.dense_from_apply(lambda v: oracle.apply_MtM(lat, A, v), lat.volume)
    assert np.max(np.abs(Q - Q.T)) < 1e-15
    assert np.min(np.linalg.eigvalsh(Q)) > 0
    x = inputs.random_vector(lat.volume, 3)
    Mx = oracle.apply_M(lat, A, x)
    assert np.dot(x, oracle.apply_MtM(lat, A, x)) == pytest.approx(np.dot(Mx, Mx), rel=1e-14)
