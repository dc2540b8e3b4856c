"""Parity of hub_cg_solve (FP64 and mixed precision) with the oracle.

CG iterates depend on rounding order, so the GPU and oracle solutions are not
bitwise equal.  What is unique is the solution of Q x = phi; each solve is
checked by
  * its true relative residual |phi - Q x| / |phi|, recomputed by the oracle
    in FP64 (<= tol, with 10% slack for the rounding of the recompute itself,
    at most ~cond(Q) * 1e-16),
  * its distance to the oracle's own CG solution, which two solutions with
    residual <= tol can differ by at most 2 cond(Q) tol,
and, where the oracle finishes in seconds, by the iteration count.  cond(Q)
comes from the Lanczos tridiagonal of the oracle's CG coefficients.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1007_3432_amd import hub, inputs
from tests import dense, hubtest

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _lib():
    hubtest.ensure_built()
    oracle.set_threads(16)


def _problem(d, nx, nt, seed=0, **kw):
    olat = oracle.Lattice(d, nx, nt, **kw)
    lat = hub.lattice(d, nx, nt, olat.t_hop, olat.dtau, olat.U, olat.mu)
    sigma, eta = inputs.sigma_eta(d, nx, nt, seed=seed)
    A = oracle.links(olat, sigma)
    phi = oracle.apply_Mt(olat, A, eta)
    return olat, lat, sigma, A, phi


def _solve(lat, sigma, phi, opts, raise_on_noconv=True):
    x_d = hubtest.empty(lat.volume, hub.F64)
    st = hub.hub_cg_solve(lat, hubtest.to_dev(sigma), hubtest.to_dev(phi), x_d, opts,
                          raise_on_noconv=raise_on_noconv)
    return x_d.cpu().numpy(), st


def _true_resid(olat, A, phi, x):
    return float(np.linalg.norm(phi - oracle.apply_MtM(olat, A, x)) / np.linalg.norm(phi))


CASES = [
    ("c0_d1_32x64", (1, 32, 64)),
    ("d1_256x128", (1, 256, 128)),
    ("d3_8x80", (3, 8, 80)),
    ("d3_4x7", (3, 4, 7)),
    ("d2_6x10", (2, 6, 10)),
    ("d1_37x9", (1, 37, 9)),
]


@pytest.mark.parametrize("name,shape", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_cg_parity(name, shape, prec):
    olat, lat, sigma, A, phi = _problem(*shape)
    hubtest.log_case(f"cg {name} {prec}")
    x_o, res_o, (al, be) = oracle.cg(olat, A, phi, tol=TOL, record=True)
    assert res_o.converged
    kappa = dense.lanczos_condition(al, be)
    if prec == "f64":
        opts = hub.cg_opts(hub.F64)
    else:
        opts = hub.cg_opts(hub.F32, hub.F32 if prec == "f32" else hub.F16)
    x, st = _solve(lat, sigma, phi, opts)
    assert st["status"] == "HUB_OK"
    assert st["true_rel_resid"] <= TOL
    r = _true_resid(olat, A, phi, x)
    assert r <= 1.1 * TOL, r
    # two solutions with residual <= tol differ by <= 2 cond(Q) tol; the
    # Lanczos estimate of cond(Q) gets a further factor 2 of slack
    assert hubtest.rel_err(x, x_o) <= 4 * kappa * TOL
    if prec == "f64":
        assert abs(st["iters"] - res_o.iters) <= 0.03 * res_o.iters + 3
        assert st["reliable_updates"] >= 1
    else:
        # FP32 bulk converges within a modest factor of FP64's iterations
        assert st["iters"] <= 3 * res_o.iters + 100
        assert st["reliable_updates"] >= st["iters"] // 50


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cg_full_size_c2(prec):
    """d=3 16^3 x 160 (655 360 sites) at full size: the oracle checks the true
    residual of the GPU solution."""
    olat, lat, sigma, A, phi = _problem(3, 16, 160)
    hubtest.log_case(f"cg c2 full {prec}")
    opts = hub.cg_opts(hub.F64) if prec == "f64" else hub.cg_opts(hub.F32, hub.F32)
    x, st = _solve(lat, sigma, phi, opts)
    assert st["status"] == "HUB_OK"
    assert _true_resid(olat, A, phi, x) <= 1.1 * TOL


def test_cg_full_size_c1_fp64():
    olat, lat, sigma, A, phi = _problem(1, 2048, 512)
    hubtest.log_case("cg c1 full f64")
    x, st = _solve(lat, sigma, phi, hub.cg_opts(hub.F64, max_iter=1000000))
    assert st["status"] == "HUB_OK"
    assert _true_resid(olat, A, phi, x) <= 1.1 * TOL


@pytest.mark.parametrize("prec", ["f64", "f16"])
def test_cg_full_size_c3(prec):
    """d=3 32^3 x 256 (8.4M sites): FP64 CG and mixed CG with FP16 links, each
    checked by the oracle's true residual."""
    olat, lat, sigma, A, phi = _problem(3, 32, 256)
    hubtest.log_case(f"cg c3 full {prec}")
    opts = hub.cg_opts(hub.F64) if prec == "f64" else hub.cg_opts(hub.F32, hub.F16)
    x, st = _solve(lat, sigma, phi, opts)
    assert st["status"] == "HUB_OK"
    assert _true_resid(olat, A, phi, x) <= 1.1 * TOL


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cg_d3_nx32(prec):
    """d=3, 32^3 x 5: the FP64 solver's own 32 x 8 x 8 tile and the mixed
    solver's 32 x 8 x 4 tile, two slices per block with a one-slice last
    chunk: oracle true residual and distance to the oracle's solution."""
    olat, lat, sigma, A, phi = _problem(3, 32, 5)
    hubtest.log_case(f"cg d3 nx32 {prec}")
    x_o, res_o, (al, be) = oracle.cg(olat, A, phi, tol=TOL, record=True)
    assert res_o.converged
    kappa = dense.lanczos_condition(al, be)
    opts = hub.cg_opts(hub.F64) if prec == "f64" else hub.cg_opts(hub.F32, hub.F16)
    x, st = _solve(lat, sigma, phi, opts)
    assert st["status"] == "HUB_OK"
    assert _true_resid(olat, A, phi, x) <= 1.1 * TOL
    assert hubtest.rel_err(x, x_o) <= 4 * kappa * TOL
    if prec == "f64":
        assert abs(st["iters"] - res_o.iters) <= 0.03 * res_o.iters + 2


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cg_d3_nx64(prec):
    """d=3, 64^3 x 4 on the default 64 x 4 x 4 tile (FP64 links for the
    residual, bulk links per precision): oracle true residual and distance to
    the oracle's solution."""
    olat, lat, sigma, A, phi = _problem(3, 64, 4)
    hubtest.log_case(f"cg d3 nx64 {prec}")
    x_o, res_o, (al, be) = oracle.cg(olat, A, phi, tol=TOL, record=True)
    assert res_o.converged
    kappa = dense.lanczos_condition(al, be)
    opts = hub.cg_opts(hub.F64) if prec == "f64" else hub.cg_opts(hub.F32, hub.F32)
    x, st = _solve(lat, sigma, phi, opts)
    assert st["status"] == "HUB_OK"
    assert _true_resid(olat, A, phi, x) <= 1.1 * TOL
    assert hubtest.rel_err(x, x_o) <= 4 * kappa * TOL


# --- the workspace and chunk graphs a thread keeps between solves

def test_solves_reuse_workspace_and_graphs_bitwise():
    """Solves on one host thread reuse its workspace and, when lattice,
    options, phi and x are unchanged, its captured chunk graphs.  A sequence
    that grows and shrinks the workspace, switches precision, lattice,
    solver and output buffer, and releases the cache midway, must give
    bitwise the same x and statistics for the same problem each time, and
    every x must pass the oracle's true residual."""
    shapes = {"a": (1, 256, 128), "b": (3, 8, 80), "s": (1, 32, 64)}
    probs = {k: _problem(*shape) for k, shape in shapes.items()}
    dev = {k: (hubtest.to_dev(p[2]), hubtest.to_dev(p[4])) for k, p in probs.items()}
    outs = {k: [hubtest.empty(p[1].volume, hub.F64) for _ in range(2)]
            for k, p in probs.items()}
    solvers = {
        "f64": lambda lat, s, f, x: hub.hub_cg_solve(lat, s, f, x, hub.cg_opts(hub.F64)),
        "f32": lambda lat, s, f, x: hub.hub_cg_solve(lat, s, f, x, hub.cg_opts(hub.F32, hub.F32)),
        "f16": lambda lat, s, f, x: hub.hub_cg_solve(lat, s, f, x, hub.cg_opts(hub.F32, hub.F16)),
        "pcg": lambda lat, s, f, x: hub.hub_pcg_solve(lat, s, f, x, hub.cg_opts(hub.F64),
                                                      hub.cheb_opts(8, 1e-3)),
    }
    seq = [("a", "f64", 0), ("a", "f64", 0), ("a", "f64", 1), ("b", "f32", 0),
           ("a", "f64", 0), ("s", "f64", 0), ("b", "f16", 1), ("a", "pcg", 0), "release",
           ("b", "f32", 0), ("a", "f64", 1), ("a", "pcg", 0), ("b", "f32", 0),
           ("s", "f64", 1), ("b", "f16", 1)]
    first = {}
    for n, item in enumerate(seq):
        if item == "release":
            hub.hub_solver_release()
            continue
        k, how, slot = item
        hubtest.log_case(f"cached solve {n}: {shapes[k]} {how} out{slot}")
        olat, _lat, _sigma, A, phi = probs[k]
        sig_d, phi_d = dev[k]
        x_d = outs[k][slot]
        x_d.fill_(float("nan"))  # the output's old contents must not matter
        st = solvers[how](probs[k][1], sig_d, phi_d, x_d)
        x = x_d.cpu().numpy()
        assert _true_resid(olat, A, phi, x) <= TOL * 1.1
        if (k, how) in first:
            x0, st0 = first[(k, how)]
            assert np.array_equal(x, x0), (n, item)
            assert st["iters"] == st0["iters"], (n, item)
            assert st["true_rel_resid"] == st0["true_rel_resid"], (n, item)
        else:
            first[(k, how)] = (x, st)


# --- failure handling (all forced from the host; every kernel exits normally)

def test_max_iter_reports_noconv_with_stats():
    olat, lat, sigma, A, phi = _problem(1, 32, 64)
    for opts in (hub.cg_opts(hub.F64, max_iter=1), hub.cg_opts(hub.F32, max_iter=7)):
        x, st = _solve(lat, sigma, phi, opts, raise_on_noconv=False)
        assert st["status"] == "HUB_E_NOCONV"
        assert st["iters"] == opts.max_iter
        r = _true_resid(olat, A, phi, x)
        assert r == pytest.approx(st["true_rel_resid"], rel=1e-6)
        assert r > TOL


def test_nan_rhs_reports_noconv():
    olat, lat, sigma, A, phi = _problem(1, 32, 64)
    phi = phi.copy()
    phi[17] = math.nan
    x, st = _solve(lat, sigma, phi, hub.cg_opts(hub.F64), raise_on_noconv=False)
    assert st["status"] == "HUB_E_NOCONV"


def test_zero_rhs_converges_immediately():
    olat, lat, sigma, A, phi = _problem(1, 32, 64)
    x, st = _solve(lat, sigma, np.zeros_like(phi), hub.cg_opts(hub.F64))
    assert st["status"] == "HUB_OK" and st["iters"] == 0 and not np.any(x)


def test_singular_matrix_does_not_converge():
    """t = 0, U = -40 (b = 3.57), nt = 2: on site 0 the field gives link factors
    1 and -1, so prod_s l = -1 and det M = 0; a generic phi has a component
    outside range(Q) and CG must report non-convergence."""
    d, nx, nt = 1, 8, 2
    lat = hub.lattice(d, nx, nt, 0.0, 0.05, -40.0, 0.0)
    olat = oracle.Lattice(d, nx, nt, 0.0, 0.05, -40.0, 0.0)
    b = oracle.hs_coupling(0.05, -40.0)
    sigma = np.zeros(nx * nt)
    sigma[0 + nx * 0] = math.asin(-2.0 / b)   # read by slice 1: l = -1
    A = oracle.links(olat, sigma)
    assert abs(A[0] * A[nx]) == pytest.approx(1.0)
    phi = inputs.random_vector(nx * nt, 3)
    x, st = _solve(lat, sigma, phi, hub.cg_opts(hub.F64, max_iter=500), raise_on_noconv=False)
    assert st["status"] == "HUB_E_NOCONV"
    assert st["true_rel_resid"] > 1e-3


def test_repulsive_coupling_rejected():
    lat = hub.lattice(1, 8, 8, U=1.0)
    x = hubtest.empty(64, hub.F64)
    with pytest.raises(hub.HubError) as e:
        hub.hub_cg_solve(lat, x, x.clone(), hubtest.empty(64, hub.F64), hub.cg_opts())
    assert e.value.status == hub.HUB_E_INVALID
