"""Serving (hub_serve_*): continuous batching of mixed-precision CG solves
from many HMC chains, stepped together by one persistent kernel.

The central check: every request gives the same x alone (hub_cg_solve with
the same options) and inside a mix of concurrent solves.  The serving kernel
runs the same tile and reduction code in the same order as the one-solve
path, so the comparison is bitwise; each result is also checked against the
oracle's FP64 true residual.
"""
import time

import numpy as np
import pytest

import oracle
from paper_1007_3432_amd import hub, inputs
from tests import hubtest

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _lib():
    hubtest.ensure_built()
    oracle.set_threads(16)


def _opts(link=hub.F32):
    return hub.cg_opts(hub.F32, link, tol=TOL, max_iter=200000, reliable_every=50)


def _chain_problem(c, request=0):
    d, nx, nt = inputs.chain_shape(c)
    olat = oracle.Lattice(d, nx, nt)
    sigma = inputs.chain_sigma(c)
    A = oracle.links(olat, sigma)
    phi = oracle.apply_Mt(olat, A, inputs.chain_eta(c, request))
    return hub.lattice(d, nx, nt), olat, sigma, A, phi


def _alone(lat, sigma, phi, opts):
    x_d = hubtest.empty(lat.volume, hub.F64)
    st = hub.hub_cg_solve(lat, hubtest.to_dev(sigma), hubtest.to_dev(phi), x_d, opts)
    return x_d.cpu().numpy(), st


def _wait_all(srv, tickets, sizes, timeout=240.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            r = srv.poll(t, sizes[t])
            if r is not None:
                out[t] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(tickets) - len(out)} solves still pending")
        time.sleep(0.002)
    return out


def _true_resid(olat, A, phi, x):
    return float(np.linalg.norm(phi - oracle.apply_MtM(olat, A, x)) / np.linalg.norm(phi))


@pytest.mark.parametrize("engine", [0, 1], ids=["batched", "persistent"])
@pytest.mark.parametrize("link", [hub.F32, hub.F16], ids=["f32", "f16"])
def test_alone_equals_mix(link, engine):
    chains = list(range(10))
    probs = {c: _chain_problem(c) for c in chains}
    shapes = {inputs.chain_shape(c) for c in chains}
    assert len(shapes) >= 3, shapes
    opts = _opts(link)
    hubtest.log_case(f"serve alone-vs-mix link={link} engine={engine}")
    alone = {c: _alone(p[0], p[2], p[4], opts) for c, p in probs.items()}
    srv = hub.Server(hbm_budget_bytes=64 << 30, max_inflight=64, cg=opts, engine=engine)
    try:
        tickets, sizes, owner = [], {}, {}
        for c, (lat, olat, sigma, A, phi) in probs.items():
            t = srv.submit(c, lat, sigma, phi)
            tickets.append(t)
            sizes[t] = lat.volume
            owner[t] = c
        res = _wait_all(srv, tickets, sizes)
    finally:
        srv.close()
    for t, (x, st) in res.items():
        c = owner[t]
        lat, olat, sigma, A, phi = probs[c]
        xa, sta = alone[c]
        assert st["status"] == "HUB_OK", (c, st)
        assert st["iters"] == sta["iters"], (c, st, sta)
        assert np.array_equal(x, xa), (c, np.max(np.abs(x - xa)))
        assert _true_resid(olat, A, phi, x) <= 1.1 * TOL


def test_small_budget_queues_and_evicts():
    """A budget that holds about two solves: requests wait for memory, idle
    chains are evicted and re-uploaded, and every answer is still right."""
    opts = _opts(hub.F32)
    c_small = [c for c in range(40) if inputs.chain_shape(c) in ((1, 256, 128), (3, 8, 80))][:6]
    probs = {c: _chain_problem(c) for c in c_small}
    biggest = max(p[0].volume for p in probs.values())
    budget = 2 * 80 * biggest  # about 54 B/site per solve plus chain state
    srv = hub.Server(hbm_budget_bytes=budget, max_inflight=64, cg=opts)
    try:
        tickets, sizes, owner = [], {}, {}
        for rnd in range(2):
            for c, (lat, olat, sigma, A, phi) in probs.items():
                t = srv.submit(c, lat, sigma if rnd == 0 else None, phi)
                tickets.append(t)
                sizes[t] = lat.volume
                owner[t] = c
        res = _wait_all(srv, tickets, sizes)
    finally:
        srv.close()
    for t, (x, st) in res.items():
        lat, olat, sigma, A, phi = probs[owner[t]]
        assert st["status"] == "HUB_OK"
        assert _true_resid(olat, A, phi, x) <= 1.1 * TOL


def test_field_reuse_and_new_field():
    """sigma_host = NULL reuses the chain's field; a new field replaces it."""
    opts = _opts(hub.F32)
    c = next(c for c in range(40) if inputs.chain_shape(c) == (1, 256, 128))
    lat, olat, sigma, A, phi = _chain_problem(c, 0)
    _, _, _, _, phi1 = _chain_problem(c, 1)
    sigma2 = -sigma
    A2 = oracle.links(olat, sigma2)
    srv = hub.Server(hbm_budget_bytes=1 << 30, max_inflight=4, cg=opts)
    try:
        t0 = srv.submit(c, lat, sigma, phi)
        t1 = srv.submit(c, lat, None, phi1)
        t2 = srv.submit(c, lat, sigma2, phi)
        res = _wait_all(srv, [t0, t1, t2], {t0: lat.volume, t1: lat.volume, t2: lat.volume})
    finally:
        srv.close()
    assert _true_resid(olat, A, phi, res[t0][0]) <= 1.1 * TOL
    assert _true_resid(olat, A, phi1, res[t1][0]) <= 1.1 * TOL
    assert _true_resid(olat, A2, phi, res[t2][0]) <= 1.1 * TOL


def test_errors():
    opts = _opts(hub.F32)
    lat, olat, sigma, A, phi = _chain_problem(0)
    srv = hub.Server(hbm_budget_bytes=1 << 20, max_inflight=4, cg=opts)
    try:
        with pytest.raises(hub.HubError) as e:
            srv.submit(0, lat, sigma, phi)            # needs more than 1 MiB
        assert e.value.status == hub.HUB_E_NOMEM
        lat2 = hub.lattice(2, 8, 8)
        with pytest.raises(hub.HubError) as e:
            srv.submit(1, lat2, np.zeros(lat2.volume), np.zeros(lat2.volume))
        assert e.value.status == hub.HUB_E_INVALID
        small = hub.lattice(1, 16, 8)
        with pytest.raises(hub.HubError) as e:
            srv.submit(2, small, None, np.zeros(small.volume))  # no field yet
        assert e.value.status == hub.HUB_E_INVALID
        with pytest.raises(hub.HubError) as e:
            srv.poll(12345, 8)
        assert e.value.status == hub.HUB_E_NOTFOUND
        t = srv.submit(3, small, np.zeros(small.volume), np.zeros(small.volume))
        res = _wait_all(srv, [t], {t: small.volume})
        assert res[t][1]["status"] == "HUB_OK" and res[t][1]["iters"] == 0
        with pytest.raises(hub.HubError) as e:
            srv.poll(t, small.volume)                 # retired
        assert e.value.status == hub.HUB_E_NOTFOUND
    finally:
        srv.close()
    with pytest.raises(hub.HubError) as e:
        hub.Server(1 << 30, 4, hub.cg_opts(hub.F64))
    assert e.value.status == hub.HUB_E_INVALID


def test_max_iter_in_mix_reports_noconv():
    opts = hub.cg_opts(hub.F32, hub.F32, tol=TOL, max_iter=30, reliable_every=50)
    lat, olat, sigma, A, phi = _chain_problem(0)
    srv = hub.Server(hbm_budget_bytes=1 << 30, max_inflight=4, cg=opts)
    try:
        t = srv.submit(0, lat, sigma, phi)
        x, st = _wait_all(srv, [t], {t: lat.volume})[t]
    finally:
        srv.close()
    assert st["status"] == "HUB_E_NOCONV" and st["iters"] == 30
    assert _true_resid(olat, A, phi, x) == pytest.approx(st["true_rel_resid"], rel=1e-6)
