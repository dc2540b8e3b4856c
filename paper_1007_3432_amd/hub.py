"""Python binding of libhub (include/hub.h): argument marshalling only.

Every function takes torch tensors already resident on the GPU and passes
their device pointers, plus the current torch stream, to the C ABI.  All
arithmetic runs in the library's HIP kernels; if the library is missing this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libhub.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "hub.h")

HUB_OK, HUB_PENDING = 0, 1
HUB_E_INVALID, HUB_E_NOMEM, HUB_E_NOCONV, HUB_E_DEVICE, HUB_E_NOTFOUND = -1, -2, -3, -4, -5
STATUS_NAMES = {0: "HUB_OK", 1: "HUB_PENDING", -1: "HUB_E_INVALID", -2: "HUB_E_NOMEM",
                -3: "HUB_E_NOCONV", -4: "HUB_E_DEVICE", -5: "HUB_E_NOTFOUND"}
F64, F32, F16 = 0, 1, 2
DTYPE_BYTES = {F64: 8, F32: 4, F16: 2}


class Lattice(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("nx", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("t_hop", ctypes.c_double),
                ("dtau", ctypes.c_double), ("U", ctypes.c_double), ("mu", ctypes.c_double)]

    @property
    def volume(self) -> int:
        return self.nx ** self.d * self.nt


class CGOpts(ctypes.Structure):
    _fields_ = [("bulk", ctypes.c_int), ("link", ctypes.c_int), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("reliable_every", ctypes.c_int32)]


class ChebOpts(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32), ("eps", ctypes.c_double),
                ("scale", ctypes.c_double)]


class CGStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("reliable_updates", ctypes.c_int32),
                ("true_rel_resid", ctypes.c_double), ("ms", ctypes.c_double),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"iters": self.iters, "reliable_updates": self.reliable_updates,
                "true_rel_resid": self.true_rel_resid, "ms": self.ms,
                "status": STATUS_NAMES.get(self.status, str(self.status))}


class MDOpts(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("eps", ctypes.c_double), ("cg", CGOpts)]


class MDStats(ctypes.Structure):
    _fields_ = [("h_start", ctypes.c_double), ("h_end", ctypes.c_double),
                ("solves", ctypes.c_int32), ("cg_iters", ctypes.c_int32),
                ("accepted", ctypes.c_int32), ("status", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"h_start": self.h_start, "h_end": self.h_end,
                "delta_h": self.h_end - self.h_start, "solves": self.solves,
                "cg_iters": self.cg_iters, "accepted": bool(self.accepted),
                "status": STATUS_NAMES.get(self.status, str(self.status))}


class ServeOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_inflight", ctypes.c_int32),
                ("engine", ctypes.c_int32), ("cg", CGOpts)]


class HubError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def lattice(d: int, nx: int, nt: int, t_hop: float = 1.0, dtau: float = 0.05,
            U: float = -2.0, mu: float = 0.0) -> Lattice:
    return Lattice(d, nx, nt, 0, t_hop, dtau, U, mu)


def cg_opts(bulk: int = F64, link: int | None = None, tol: float = 1e-10,
            max_iter: int = 200000, reliable_every: int = 50) -> CGOpts:
    if link is None:
        link = F64 if bulk == F64 else F32
    return CGOpts(bulk, link, tol, max_iter, reliable_every)


def md_opts(n_steps: int, eps: float, cg: CGOpts | None = None) -> MDOpts:
    return MDOpts(int(n_steps), 0, float(eps), cg if cg is not None else cg_opts())


def cheb_opts(n: int, eps: float, scale: float = 0.0) -> ChebOpts:
    """Chebyshev preconditioner of half-degree n on (eps, 1]; scale <= 0 picks
    the library's bound on the largest eigenvalue of Q."""
    return ChebOpts(n, 0, eps, scale)


_lib = None


def load():
    """Load libhub.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    # torch brings its own HIP runtime (same soname, libamdhip64.so.7).  Load
    # it first so that libhub binds to that one copy: two HIP runtimes in one
    # process cannot share the device or each other's memory and streams.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, lp = ctypes.c_void_p, ctypes.POINTER(Lattice)
    lib.hub_links_from_sigma.argtypes = [lp, vp, vp, ctypes.c_int, vp]
    lib.hub_apply_M.argtypes = [lp, vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int, vp]
    lib.hub_apply_MtM.argtypes = [lp, vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    lib.hub_cg_solve.argtypes = [lp, vp, vp, vp, ctypes.POINTER(CGOpts),
                                 ctypes.POINTER(CGStats), vp]
    lib.hub_apply_cheb.argtypes = [lp, vp, vp, vp, ctypes.POINTER(ChebOpts), vp]
    lib.hub_apply_cheb_noalloc.argtypes = [lp, vp, vp, vp, ctypes.POINTER(ChebOpts), vp]
    lib.hub_pcg_solve.argtypes = [lp, vp, vp, vp, ctypes.POINTER(CGOpts),
                                  ctypes.POINTER(ChebOpts), ctypes.POINTER(CGStats), vp]
    lib.hub_hmc_force.argtypes = [lp, vp, vp, vp, vp]
    lib.hub_md_trajectory.argtypes = [lp, vp, vp, vp, ctypes.POINTER(MDOpts),
                                      ctypes.POINTER(MDStats), vp]
    lib.hub_hmc_trajectory.argtypes = [lp, vp, vp, vp, ctypes.c_double, ctypes.POINTER(MDOpts),
                                       ctypes.POINTER(MDStats), vp]
    lib.hub_serve_create.argtypes = [ctypes.POINTER(ServeOpts), ctypes.POINTER(vp)]
    lib.hub_serve_submit.argtypes = [vp, ctypes.c_int32, lp, vp, vp,
                                     ctypes.POINTER(ctypes.c_uint64)]
    lib.hub_serve_poll.argtypes = [vp, ctypes.c_uint64, vp, ctypes.POINTER(CGStats)]
    lib.hub_serve_destroy.argtypes = [vp]
    lib.hub_solver_release.argtypes = []
    for f in (lib.hub_links_from_sigma, lib.hub_apply_M, lib.hub_apply_MtM, lib.hub_cg_solve,
              lib.hub_apply_cheb, lib.hub_apply_cheb_noalloc, lib.hub_pcg_solve,
              lib.hub_hmc_force, lib.hub_md_trajectory, lib.hub_hmc_trajectory,
              lib.hub_serve_create, lib.hub_serve_submit, lib.hub_serve_poll,
              lib.hub_serve_destroy, lib.hub_solver_release):
        f.restype = ctypes.c_int
    lib.hub_last_error.argtypes = []
    lib.hub_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def last_error() -> str:
    return load().hub_last_error().decode()


def _check(status: int, where: str, ok=(HUB_OK,)) -> int:
    if status not in ok:
        raise HubError(status, where, last_error())
    return status


def _torch_dtype(t):
    import torch
    return {F64: torch.float64, F32: torch.float32, F16: torch.float16}[t]


def _dev_ptr(t, dtype: int, n: int, name: str) -> int:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dtype != _torch_dtype(dtype):
        raise ValueError(f"{name}: dtype {t.dtype} does not match hub dtype {dtype}")
    if t.numel() != n:
        raise ValueError(f"{name}: {t.numel()} elements, lattice has {n}")
    return t.data_ptr()


def _stream(stream) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def hub_links_from_sigma(lat: Lattice, sigma, links, link: int = F64, stream=None) -> None:
    V = lat.volume
    _check(load().hub_links_from_sigma(ctypes.byref(lat), _dev_ptr(sigma, F64, V, "sigma"),
                                       _dev_ptr(links, link, V, "links"), link,
                                       _stream(stream)), "hub_links_from_sigma")


def hub_apply_M(lat: Lattice, links, link: int, vec: int, x, y, transpose: int = 0,
                stream=None) -> None:
    V = lat.volume
    _check(load().hub_apply_M(ctypes.byref(lat), _dev_ptr(links, link, V, "links"), link, vec,
                              _dev_ptr(x, vec, V, "x"), _dev_ptr(y, vec, V, "y"),
                              int(transpose), _stream(stream)), "hub_apply_M")


def hub_apply_MtM(lat: Lattice, links, link: int, vec: int, x, z, stream=None) -> None:
    V = lat.volume
    _check(load().hub_apply_MtM(ctypes.byref(lat), _dev_ptr(links, link, V, "links"), link,
                                vec, _dev_ptr(x, vec, V, "x"), _dev_ptr(z, vec, V, "z"),
                                _stream(stream)), "hub_apply_MtM")


def hub_cg_solve(lat: Lattice, sigma, phi, x, opts: CGOpts, stream=None,
                 raise_on_noconv: bool = True) -> dict:
    V = lat.volume
    st = CGStats()
    status = load().hub_cg_solve(ctypes.byref(lat), _dev_ptr(sigma, F64, V, "sigma"),
                                 _dev_ptr(phi, F64, V, "phi"), _dev_ptr(x, F64, V, "x"),
                                 ctypes.byref(opts), ctypes.byref(st), _stream(stream))
    ok = (HUB_OK,) if raise_on_noconv else (HUB_OK, HUB_E_NOCONV)
    _check(status, "hub_cg_solve", ok)
    return st.as_dict()


def hub_solver_release() -> None:
    _check(load().hub_solver_release(), "hub_solver_release")


def hub_apply_cheb(lat: Lattice, links, r, z, cheb: ChebOpts, stream=None) -> None:
    V = lat.volume
    _check(load().hub_apply_cheb(ctypes.byref(lat), _dev_ptr(links, F64, V, "links"),
                                 _dev_ptr(r, F64, V, "r"), _dev_ptr(z, F64, V, "z"),
                                 ctypes.byref(cheb), _stream(stream)), "hub_apply_cheb")


def hub_apply_cheb_noalloc(lat: Lattice, links, r, z, cheb: ChebOpts, stream=None) -> None:
    V = lat.volume
    _check(load().hub_apply_cheb_noalloc(ctypes.byref(lat), _dev_ptr(links, F64, V, "links"),
                                         _dev_ptr(r, F64, V, "r"), _dev_ptr(z, F64, V, "z"),
                                         ctypes.byref(cheb), _stream(stream)),
           "hub_apply_cheb_noalloc")


def hub_pcg_solve(lat: Lattice, sigma, phi, x, opts: CGOpts, cheb: ChebOpts, stream=None,
                  raise_on_noconv: bool = True) -> dict:
    V = lat.volume
    st = CGStats()
    status = load().hub_pcg_solve(ctypes.byref(lat), _dev_ptr(sigma, F64, V, "sigma"),
                                  _dev_ptr(phi, F64, V, "phi"), _dev_ptr(x, F64, V, "x"),
                                  ctypes.byref(opts), ctypes.byref(cheb), ctypes.byref(st),
                                  _stream(stream))
    ok = (HUB_OK,) if raise_on_noconv else (HUB_OK, HUB_E_NOCONV)
    _check(status, "hub_pcg_solve", ok)
    return st.as_dict()


def hub_hmc_force(lat: Lattice, sigma, x, force, stream=None) -> None:
    V = lat.volume
    _check(load().hub_hmc_force(ctypes.byref(lat), _dev_ptr(sigma, F64, V, "sigma"),
                                _dev_ptr(x, F64, V, "x"), _dev_ptr(force, F64, V, "force"),
                                _stream(stream)), "hub_hmc_force")


def hub_md_trajectory(lat: Lattice, sigma, pi, phi, opts: MDOpts, stream=None,
                      raise_on_noconv: bool = True) -> dict:
    V = lat.volume
    st = MDStats()
    status = load().hub_md_trajectory(ctypes.byref(lat), _dev_ptr(sigma, F64, V, "sigma"),
                                      _dev_ptr(pi, F64, V, "pi"), _dev_ptr(phi, F64, V, "phi"),
                                      ctypes.byref(opts), ctypes.byref(st), _stream(stream))
    ok = (HUB_OK,) if raise_on_noconv else (HUB_OK, HUB_E_NOCONV)
    _check(status, "hub_md_trajectory", ok)
    return st.as_dict()


def hub_hmc_trajectory(lat: Lattice, sigma, eta, pi0, u: float, opts: MDOpts, stream=None,
                       raise_on_noconv: bool = True) -> dict:
    V = lat.volume
    st = MDStats()
    status = load().hub_hmc_trajectory(ctypes.byref(lat), _dev_ptr(sigma, F64, V, "sigma"),
                                       _dev_ptr(eta, F64, V, "eta"),
                                       _dev_ptr(pi0, F64, V, "pi0"), float(u),
                                       ctypes.byref(opts), ctypes.byref(st), _stream(stream))
    ok = (HUB_OK,) if raise_on_noconv else (HUB_OK, HUB_E_NOCONV)
    _check(status, "hub_hmc_trajectory", ok)
    return st.as_dict()


class Server:
    """hub_serve_*: continuous batching of CG solves for many HMC chains."""

    ENGINE_BATCHED, ENGINE_PERSISTENT = 0, 1

    def __init__(self, hbm_budget_bytes: int, max_inflight: int, cg: CGOpts, engine: int = 0):
        self._lib = load()
        self._opts = ServeOpts(int(hbm_budget_bytes), int(max_inflight), int(engine), cg)
        h = ctypes.c_void_p()
        _check(self._lib.hub_serve_create(ctypes.byref(self._opts), ctypes.byref(h)),
               "hub_serve_create")
        self._h = h

    def submit(self, chain_id: int, lat: Lattice, sigma_host, phi_host) -> int:
        V = lat.volume
        sig = None
        if sigma_host is not None:
            sig = np.ascontiguousarray(sigma_host, dtype=np.float64)
            if sig.shape != (V,):
                raise ValueError("sigma_host has the wrong size")
        phi = np.ascontiguousarray(phi_host, dtype=np.float64)
        if phi.shape != (V,):
            raise ValueError("phi_host has the wrong size")
        t = ctypes.c_uint64()
        _check(self._lib.hub_serve_submit(self._h, int(chain_id), ctypes.byref(lat),
                                          None if sig is None else sig.ctypes.data,
                                          phi.ctypes.data, ctypes.byref(t)),
               "hub_serve_submit")
        return t.value

    def poll(self, ticket: int, V: int):
        """None while pending, else (x, stats dict); raises on other errors
        except non-convergence, which is reported in the stats."""
        x = np.empty(V, dtype=np.float64)
        st = CGStats()
        s = self._lib.hub_serve_poll(self._h, ctypes.c_uint64(ticket), x.ctypes.data,
                                     ctypes.byref(st))
        if s == HUB_PENDING:
            return None
        _check(s, "hub_serve_poll", (HUB_OK, HUB_E_NOCONV))
        return x, st.as_dict()

    def close(self) -> None:
        if self._h:
            _check(self._lib.hub_serve_destroy(self._h), "hub_serve_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def declared_symbols() -> list[str]:
    """Names of every function include/hub.h declares."""
    import re
    text = open(HEADER).read()
    return re.findall(r"HUB_API\s+[\w\s\*]+?\b(hub_\w+)\s*\(", text)
