"""Dense-matrix helpers for the oracle pins (CPU only, tiny lattices).

These build matrices from the paper's definitions directly (the block form
of M, Eq. (7), with the transfer blocks of Eq. (8) and the kinetic matrix of
Eq. (9)), or by applying an operator to unit vectors.  They never call the
GPU library.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg


def coords(d: int, nx: int):
    """Spatial coordinates (c_0 fastest) of every spatial index n."""
    out = []
    for n in range(nx ** d):
        c, m = [], n
        for _ in range(d):
            c.append(m % nx)
            m //= nx
        out.append(tuple(c))
    return out


def kinetic_matrix(d: int, nx: int, t_hop: float) -> np.ndarray:
    """K_{n,n'} = -t sum_j (delta_{n,n'+e_j} + delta_{n,n'-e_j}), periodic."""
    cs = coords(d, nx)
    Vs = len(cs)
    K = np.zeros((Vs, Vs))
    for n, c in enumerate(cs):
        for np_, cp in enumerate(cs):
            for j in range(d):
                plus = list(cp); plus[j] = (plus[j] + 1) % nx
                minus = list(cp); minus[j] = (minus[j] - 1) % nx
                if tuple(plus) == c:
                    K[n, np_] += -t_hop
                if tuple(minus) == c:
                    K[n, np_] += -t_hop
    return K


def dense_from_apply(apply, V: int) -> np.ndarray:
    """Column j of the result is apply(e_j)."""
    out = np.empty((V, V))
    e = np.zeros(V)
    for j in range(V):
        e[j] = 1.0
        out[:, j] = apply(e)
        e[j] = 0.0
    return out


def block_form_M(d, nx, nt, t_hop, dtau, U, mu, sigma) -> np.ndarray:
    """M of Eq. (7): identity blocks on the diagonal, -B_j below it (row j+1,
    1-based) and +B_{N_tau} in the top-right corner, with
    B_j = exp(-dtau K) exp(-dtau V[sigma_j]) (Eq. (8)).  The field factor is
    the compact HS form exp(dtau mu) diag(1 + b sin sigma_j),
    b = sqrt(2 (exp(-dtau U) - 1)).  Slice j (1-based) holds sigma[:, j-1]."""
    Vs = nx ** d
    K = kinetic_matrix(d, nx, t_hop)
    eK = scipy.linalg.expm(-dtau * K)
    b = np.sqrt(2.0 * (np.exp(-dtau * U) - 1.0))
    sig = np.asarray(sigma).reshape(nt, Vs)
    M = np.eye(Vs * nt)

    def B(j):  # 1-based slice index
        return eK @ np.diag(np.exp(dtau * mu) * (1.0 + b * np.sin(sig[j - 1])))

    for row in range(2, nt + 1):      # 1-based block rows 2..nt
        r0 = (row - 1) * Vs
        c0 = (row - 2) * Vs
        M[r0:r0 + Vs, c0:c0 + Vs] = -B(row - 1)
    M[0:Vs, (nt - 1) * Vs:nt * Vs] = B(nt)
    return M


def plane_wave_lambdas(d, nx, nt, t_hop, dtau, f):
    """Closed-form eigenvalues a_k - f exp(-i w) of M at constant field factor
    f, with a_k = 1 - 2 dtau t sum_j cos k_j, k_j = 2 pi m_j / nx and
    w = pi (2l+1) / nt (antiperiodic)."""
    kappa = dtau * t_hop
    out = []
    for ms in itertools.product(range(nx), repeat=d):
        a = 1.0 - 2.0 * kappa * sum(np.cos(2 * np.pi * m / nx) for m in ms)
        for l in range(nt):
            w = np.pi * (2 * l + 1) / nt
            out.append((ms, l, a - f * np.exp(-1j * w)))
    return out


def lanczos_condition(alphas, betas) -> float:
    """cond(Q) estimated from the extreme eigenvalues of the Lanczos
    tridiagonal that CG's coefficients define: T_kk = 1/alpha_k +
    beta_{k-1}/alpha_{k-1}, T_{k,k+1} = sqrt(beta_k)/alpha_k."""
    import scipy.linalg
    a = np.asarray(alphas)
    b = np.asarray(betas)[: a.size - 1]
    diag = 1.0 / a
    diag[1:] += b / a[:-1]
    off = np.sqrt(b) / a[:-1]
    ev = scipy.linalg.eigvalsh_tridiagonal(diag, off)
    return float(ev[-1] / ev[0])


def cheb_closed_form(lam, n: int, eps: float):
    """P(l) of Eq. (13) from the identity 1 - l P(l) = T_{2n+1}(u) / T_{2n+1}(u(0)),
    u = (2 l - 1 - eps) / (1 - eps); valid for l > 0."""
    from numpy.polynomial import chebyshev
    m = 2 * n + 1
    coef = [0.0] * m + [1.0]
    u = (2.0 * np.asarray(lam) - 1.0 - eps) / (1.0 - eps)
    u0 = -(1.0 + eps) / (1.0 - eps)
    return (1.0 - chebyshev.chebval(u, coef) / chebyshev.chebval(u0, coef)) / lam
