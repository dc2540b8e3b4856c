"""CPU oracle for the Hubbard fermion matrix -- TEST INFRASTRUCTURE ONLY.

Plain FP64 reference implementation of the stencil form of the fermion matrix
M (Sec. 2, Eqs. (7), (8) and (10) of Wendt, Drut, Laehde), of M^T, of
Q = M^T M, and of conjugate gradient on Q x = phi (Sec. 4.1).  The arithmetic
lives in ``hub_oracle.c``; this module only marshals numpy arrays.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1007_3432_amd``), and neither imports the other.

Parity status of each function (the pins live under ``tests/``):
  hs_coupling        pinned: HS quadrature identity
  links              pinned: block form of M with exact exponentials
  apply_M            pinned: block form, plane-wave eigenvalues, det closed
                     form, determinant identity vs dense LU
  apply_Mt           pinned: adjoint identity, dense transpose
  apply_MtM          pinned: composition, eigenvalues |lambda|^2
  cg                 pinned: dense solve, finite termination on few
                     distinct eigenvalues, true residual
  cheb_roots/norm    pinned: error bound of Eq. (16) on (eps, 1], near
                     equioscillation
  cheb_apply         pinned: dense eigen-decomposition of Q/scale with the
                     scalar polynomial
  cheb_scale         pinned: bound >= largest eigenvalue of Q (dense)
  pcg                pinned: dense solve, fewer iterations than CG
  force              pinned: central finite differences of S_p(sigma) =
                     phi^T Q^{-1} phi with Q dense (numpy solve)
  md                 pinned: reversibility (pi -> -pi retraces the path),
                     energy error O(eps^2), S_p = eta.eta for phi = M^T eta
  hmc                pinned: Metropolis decision and field restore on reject
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "libhub_oracle.so")
_lib = None


class _Lattice(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("t_hop", ctypes.c_double), ("dtau", ctypes.c_double),
                ("U", ctypes.c_double), ("mu", ctypes.c_double)]


class _CGResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("breakdown", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("true_rel_resid", ctypes.c_double),
                ("iter_rel_resid", ctypes.c_double)]


@dataclass(frozen=True)
class Lattice:
    """d spatial dims of extent nx (periodic) x nt slices (antiperiodic)."""
    d: int
    nx: int
    nt: int
    t_hop: float = 1.0
    dtau: float = 0.05
    U: float = -2.0
    mu: float = 0.0

    @property
    def vs(self) -> int:
        return self.nx ** self.d

    @property
    def volume(self) -> int:
        return self.vs * self.nt

    def _c(self) -> _Lattice:
        return _Lattice(self.d, self.nx, self.nt, 0, self.t_hop, self.dtau,
                        self.U, self.mu)


class _MDResult(ctypes.Structure):
    _fields_ = [("h_start", ctypes.c_double), ("h_end", ctypes.c_double),
                ("solves", ctypes.c_int32), ("cg_iters", ctypes.c_int32),
                ("accepted", ctypes.c_int32), ("failed", ctypes.c_int32)]


@dataclass
class MDResult:
    h_start: float
    h_end: float
    solves: int
    cg_iters: int
    accepted: bool
    failed: bool

    @property
    def delta_h(self) -> float:
        return self.h_end - self.h_start


@dataclass
class CGResult:
    iters: int
    converged: bool
    breakdown: bool
    restarts: int
    true_rel_resid: float
    iter_rel_resid: float


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(_Lattice)
    lib.oracle_hs_coupling.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle_hs_coupling.restype = ctypes.c_double
    lib.oracle_volume.argtypes = [lp]
    lib.oracle_volume.restype = ctypes.c_long
    lib.oracle_links.argtypes = [lp, dp, dp]
    lib.oracle_links.restype = None
    for f in (lib.oracle_apply_M, lib.oracle_apply_Mt):
        f.argtypes = [lp, dp, dp, dp]
        f.restype = None
    lib.oracle_apply_MtM.argtypes = [lp, dp, dp, dp, dp]
    lib.oracle_apply_MtM.restype = None
    lib.oracle_dot.argtypes = [ctypes.c_long, dp, dp]
    lib.oracle_dot.restype = ctypes.c_double
    lib.oracle_cg.argtypes = [lp, dp, dp, dp, ctypes.c_double, ctypes.c_int32,
                              ctypes.POINTER(_CGResult), dp, dp]
    lib.oracle_cg.restype = ctypes.c_int
    lib.oracle_cheb_roots.argtypes = [ctypes.c_int32, ctypes.c_double, dp, dp]
    lib.oracle_cheb_roots.restype = None
    lib.oracle_cheb_norm.argtypes = [ctypes.c_int32, ctypes.c_double]
    lib.oracle_cheb_norm.restype = ctypes.c_double
    lib.oracle_cheb_apply.argtypes = [lp, dp, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                      dp, dp]
    lib.oracle_cheb_apply.restype = ctypes.c_int
    lib.oracle_pcg.argtypes = [lp, dp, dp, dp, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                               ctypes.c_int32, ctypes.c_double, ctypes.POINTER(_CGResult)]
    lib.oracle_pcg.restype = ctypes.c_int
    lib.oracle_force.argtypes = [lp, dp, dp, dp]
    lib.oracle_force.restype = None
    lib.oracle_md.argtypes = [lp, dp, dp, dp, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                              ctypes.c_int32, ctypes.POINTER(_MDResult)]
    lib.oracle_md.restype = ctypes.c_int
    lib.oracle_hmc.argtypes = [lp, dp, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                               ctypes.c_double, ctypes.c_int32, ctypes.POINTER(_MDResult)]
    lib.oracle_hmc.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec(a, n: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (n,):
        raise ValueError(f"expected shape ({n},), got {a.shape}")
    return a


def set_threads(n: int = 0) -> int:
    """Set (n > 0) and return the OpenMP thread count of the stencil loops."""
    return _load().oracle_set_threads(int(n))


def hs_coupling(dtau: float, U: float) -> float:
    """b = sqrt(2 (exp(-dtau U) - 1)) of the compact HS transform."""
    return _load().oracle_hs_coupling(float(dtau), float(U))


def links(lat: Lattice, sigma) -> np.ndarray:
    """Sign-folded time-link coefficients A[n + Vs*s] (Eq. (10))."""
    s = _vec(sigma, lat.volume)
    out = np.empty(lat.volume)
    _load().oracle_links(ctypes.byref(lat._c()), _ptr(s), _ptr(out))
    return out


def apply_M(lat: Lattice, A, x) -> np.ndarray:
    A = _vec(A, lat.volume)
    x = _vec(x, lat.volume)
    y = np.empty(lat.volume)
    _load().oracle_apply_M(ctypes.byref(lat._c()), _ptr(A), _ptr(x), _ptr(y))
    return y


def apply_Mt(lat: Lattice, A, y) -> np.ndarray:
    A = _vec(A, lat.volume)
    y = _vec(y, lat.volume)
    z = np.empty(lat.volume)
    _load().oracle_apply_Mt(ctypes.byref(lat._c()), _ptr(A), _ptr(y), _ptr(z))
    return z


def apply_MtM(lat: Lattice, A, x) -> np.ndarray:
    A = _vec(A, lat.volume)
    x = _vec(x, lat.volume)
    z = np.empty(lat.volume)
    tmp = np.empty(lat.volume)
    _load().oracle_apply_MtM(ctypes.byref(lat._c()), _ptr(A), _ptr(x),
                             _ptr(z), _ptr(tmp))
    return z


def dot(a, b) -> float:
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    if a.shape != b.shape or a.ndim != 1:
        raise ValueError("dot expects two vectors of equal length")
    return _load().oracle_dot(a.size, _ptr(a), _ptr(b))


def cg(lat: Lattice, A, phi, tol: float = 1e-10, max_iter: int = 200000,
       record: bool = False):
    """Solve (M^T M) x = phi by CG from x0 = 0; returns (x, CGResult), and
    with record=True also (alphas, betas) of every iteration."""
    A = _vec(A, lat.volume)
    phi = _vec(phi, lat.volume)
    x = np.empty(lat.volume)
    res = _CGResult()
    al = np.zeros(max_iter) if record else None
    be = np.zeros(max_iter) if record else None
    rc = _load().oracle_cg(ctypes.byref(lat._c()), _ptr(A), _ptr(phi), _ptr(x),
                           float(tol), int(max_iter), ctypes.byref(res),
                           _ptr(al) if record else None, _ptr(be) if record else None)
    if rc < 0:
        raise MemoryError("oracle_cg: allocation failed")
    out = CGResult(res.iters, bool(res.converged), bool(res.breakdown),
                   res.restarts, res.true_rel_resid, res.iter_rel_resid)
    if record:
        return x, out, (al[:res.iters], be[:max(res.iters - 1, 0)])
    return x, out


# --- Chebyshev polynomial preconditioner (Sec. 4.2, Eqs. (13)-(15)) ---

def cheb_roots(n: int, eps: float) -> np.ndarray:
    """z_{2n,k}, k = 1 .. 2n, as complex numbers."""
    re = np.empty(2 * n)
    im = np.empty(2 * n)
    _load().oracle_cheb_roots(int(n), float(eps), _ptr(re), _ptr(im))
    return re + 1j * im


def cheb_norm(n: int, eps: float) -> float:
    """c_{2n}."""
    return _load().oracle_cheb_norm(int(n), float(eps))


def cheb_scale(lat: Lattice) -> float:
    """Bound on the largest eigenvalue of Q: |M| <= 1 + 2 d kappa + max|A|
    (triangle inequality over the stencil's terms), max|A| <= e^{dtau mu}(1+b)."""
    kappa = lat.dtau * lat.t_hop
    amax = np.exp(lat.dtau * lat.mu) * (1.0 + hs_coupling(lat.dtau, lat.U))
    return (1.0 + 2 * lat.d * kappa + amax) ** 2


def cheb_apply(lat: Lattice, A, r, n: int, eps: float, scale: float | None = None) -> np.ndarray:
    """z = P(Q / scale) r."""
    A = _vec(A, lat.volume)
    r = _vec(r, lat.volume)
    z = np.empty(lat.volume)
    s = cheb_scale(lat) if scale is None else float(scale)
    rc = _load().oracle_cheb_apply(ctypes.byref(lat._c()), _ptr(A), s, int(n), float(eps),
                                   _ptr(r), _ptr(z))
    if rc < 0:
        raise MemoryError("oracle_cheb_apply: allocation failed")
    return z


def pcg(lat: Lattice, A, phi, n: int, eps: float, tol: float = 1e-10,
        max_iter: int = 200000, scale: float | None = None):
    """Chebyshev-preconditioned CG; returns (x, CGResult)."""
    A = _vec(A, lat.volume)
    phi = _vec(phi, lat.volume)
    x = np.empty(lat.volume)
    res = _CGResult()
    s = cheb_scale(lat) if scale is None else float(scale)
    rc = _load().oracle_pcg(ctypes.byref(lat._c()), _ptr(A), _ptr(phi), _ptr(x), float(tol),
                            int(max_iter), s, int(n), float(eps), ctypes.byref(res))
    if rc < 0:
        raise MemoryError("oracle_pcg: allocation failed")
    return x, CGResult(res.iters, bool(res.converged), bool(res.breakdown),
                       res.restarts, res.true_rel_resid, res.iter_rel_resid)


# --- Hybrid Monte Carlo, phi-algorithm (Sec. 4.1) ---

def _md_out(r: _MDResult) -> MDResult:
    return MDResult(r.h_start, r.h_end, r.solves, r.cg_iters, bool(r.accepted), bool(r.failed))


def force(lat: Lattice, sigma, x) -> np.ndarray:
    """dS_p/dsigma at every site for x = Q^{-1} phi (S_p = phi^T Q^{-1} phi)."""
    sigma = _vec(sigma, lat.volume)
    x = _vec(x, lat.volume)
    F = np.empty(lat.volume)
    _load().oracle_force(ctypes.byref(lat._c()), _ptr(sigma), _ptr(x), _ptr(F))
    return F


def md(lat: Lattice, sigma, pi, phi, eps: float, n_steps: int, tol: float = 1e-10,
       max_iter: int = 200000):
    """Leapfrog MD trajectory; returns (sigma_end, pi_end, MDResult)."""
    s = _vec(sigma, lat.volume).copy()
    p = _vec(pi, lat.volume).copy()
    phi = _vec(phi, lat.volume)
    r = _MDResult()
    rc = _load().oracle_md(ctypes.byref(lat._c()), _ptr(s), _ptr(p), _ptr(phi), float(eps),
                           int(n_steps), float(tol), int(max_iter), ctypes.byref(r))
    if rc < 0:
        raise MemoryError("oracle_md: allocation failed")
    return s, p, _md_out(r)


def hmc(lat: Lattice, sigma, eta, pi0, u: float, eps: float, n_steps: int,
        tol: float = 1e-10, max_iter: int = 200000):
    """One HMC trajectory (heatbath phi = M^T eta, MD, Metropolis with u);
    returns (sigma_out, MDResult)."""
    s = _vec(sigma, lat.volume).copy()
    eta = _vec(eta, lat.volume)
    pi0 = _vec(pi0, lat.volume)
    r = _MDResult()
    rc = _load().oracle_hmc(ctypes.byref(lat._c()), _ptr(s), _ptr(eta), _ptr(pi0), float(u),
                            float(eps), int(n_steps), float(tol), int(max_iter), ctypes.byref(r))
    if rc < 0:
        raise MemoryError("oracle_hmc: allocation failed")
    return s, _md_out(r)
