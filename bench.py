"""Benchmark of the fermion-matrix hot path on one MI355X.

One step is the d=1 2048 x 512 workload (1 048 576 sites, t=1, dtau=0.05,
U=-2, sigma uniform, phi = M^T eta): links from sigma, phi = M^T eta, 1000
bare hub_apply_MtM calls in FP64 cycling over 24 buffer sets (576 MiB, more
than twice the 256 MiB Infinity Cache, so the sweeps stream from HBM),
captured once into a HIP graph and replayed, and one FP64 CG solve of
M^T M x = phi to a true relative residual of 1e-10.

Printed: one JSON line.  `value` is the effective HBM throughput of the bare
sweeps (24 algorithmic bytes per site: read x and A, write z) over the timed
steps.  `roofline` prices the sweep kernel's average duration (HIP events
around the graph replay, divided by the calls) against the 8 TB/s HBM peak.

`detail` carries, outside the timed steps, every other workload:
  c0   d=1 32 x 64 FP64 CG: solves/s, iterations, true residual and error
       against the oracle's CG solution;
  c1   the timed CG solve's true residual recomputed by the oracle;
  c2   d=3 16^3 x 160, FP64 CG vs mixed CG (FP32 links): ms per solve (min and
       median of 3), iterations, oracle-recomputed true residual and error
       against the oracle's CG solution (solved on a host thread meanwhile);
  c3   d=3 32^3 x 256, FP64 CG vs mixed CG (FP16 sin sigma links), same
       fields except the oracle solution (too slow on the host): the oracle
       recomputes each GPU solution's true residual instead;
  bare sweeps at 8.4M sites (d=3 32^3 x 256 and d=1 8192 x 1024) for the
       asymptotic fraction of the HBM roofline;
  serving: 64 HMC chains, Poisson arrivals at 200/s and at saturation
       (capacity): solves/s, p50/p99 latency, per-shape counts, HBM GB/s;
  Chebyshev-preconditioned CG over a grid of (n, eps).
`cpu_baseline` times the CPU oracle on a bounded sample of the headline sweep
on the host cores, with the single-thread rate, CG solve times and the CPU
model beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SWEEP_BYTES_F64 = 24       # per site: x 8 + A 8 + z 8
CG_ITER_BYTES_F64 = 80     # per site and iteration (phase A 56 + phase B 24)
# Mixed CG per site and iteration: phase A reads r, p_old, x_lo (4 B each)
# and the bulk link (4 B FP32, 2 B FP16 sin sigma) and writes p, q, x_lo;
# phase B reads r, q and writes r.
CG_ITER_BYTES_MIXED = {"f32": 40, "f16_sin_sigma": 38}
# Per site and reliable update: fold (x 8, x_lo 4, p 4 in; x 8, x_lo 4 out)
# plus the FP64 residual sweep (x, A64, phi 8 each, p 4 in; r 4 out).
RELIABLE_BYTES = 60

# HBM bytes one launch of the timed sweep (k_mtm_d1m<OpApply<double>, 512, 8, 8>
# on d=1 2048 x 512) actually moves: rocprofv3 FETCH_SIZE x 2.000 plus
# WRITE_SIZE x 1.000 per dispatch, each factor calibrated on a 256 MiB copy.
# Valid only for that kernel and tile; None once either changes.
SWEEP_TRAFFIC = {"kernel": "k_mtm_d1m<OpApply<double>,512,8,8>", "bytes": 25_678_587}


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--calls", type=int, default=1000, help="bare sweeps per step")
    ap.add_argument("--sets", type=int, default=24, help="rotating buffer sets")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-detail", action="store_true",
                    help="skip every leg beside the headline (same as --legs none)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving workload")
    ap.add_argument("--legs", default="all",
                    help="comma-separated legs beside the headline: sweeps, c0, c2, c3, "
                         "pcg, hmc, serve, cgprof (a few CG iterations per solver, for "
                         "counter runs), mv (the paper's MV experiment: fused vs naive vs "
                         "CPU over lattice sizes, about a minute of host time); 'all' = "
                         "every leg but cgprof and mv, 'none' = headline only")
    ap.add_argument("--cgprof-iters", type=int, default=60,
                    help="iterations per solve of the cgprof leg")
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip the oracle checks of GPU solutions")
    ap.add_argument("--engine", type=int, default=0, help="serving engine: 0 batched, 1 persistent")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--direct", action="store_true",
                    help="launch the bare sweeps one by one instead of replaying a graph "
                         "(for counter collection)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one 256 MiB device copy (counter calibration)")
    return ap.parse_args()


def _build_if_missing():
    from paper_1007_3432_amd import hub
    if not os.path.exists(hub.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()


def _dev(a, dtype=None):
    import numpy as np
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return t if dtype is None else t.to(dtype)


def _progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _rel(a, b) -> float:
    import numpy as np
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


# ---------------------------------------------------------------------------
# Oracle checks (outside every timed region)

class OracleSolve(threading.Thread):
    """The oracle's FP64 CG solve of one workload on a host thread, so that
    the GPU legs run meanwhile (the C oracle releases the GIL)."""

    def __init__(self, shape, threads: int):
        super().__init__(daemon=True)
        self.shape, self.threads = shape, threads
        self.x = self.res = None
        self.seconds = None
        self.error = None

    def run(self):
        try:
            import oracle
            from paper_1007_3432_amd import inputs
            oracle.set_threads(self.threads)
            lat = oracle.Lattice(*self.shape)
            sigma, eta = inputs.sigma_eta(*self.shape, seed=0)
            A = oracle.links(lat, sigma)
            phi = oracle.apply_Mt(lat, A, eta)
            t0 = time.perf_counter()
            self.x, self.res = oracle.cg(lat, A, phi)
            self.seconds = time.perf_counter() - t0
        except Exception as e:  # reported, never hidden
            self.error = repr(e)


def oracle_problem(shape):
    """(oracle lattice, A, phi) of a workload, phi = M^T eta by the oracle."""
    import oracle
    from paper_1007_3432_amd import inputs
    lat = oracle.Lattice(*shape)
    sigma, eta = inputs.sigma_eta(*shape, seed=0)
    A = oracle.links(lat, sigma)
    return lat, A, oracle.apply_Mt(lat, A, eta)


def oracle_true_resid(olat, A, phi, x) -> float:
    import numpy as np
    import oracle
    r = phi - oracle.apply_MtM(olat, A, x)
    return float(np.linalg.norm(r) / np.linalg.norm(phi))


# ---------------------------------------------------------------------------
# GPU legs

def gpu_problem(hub, shape, phi_host=None):
    """Device sigma, FP64 links and phi of a workload.  phi is the oracle's
    when given (parity legs), else M^T eta by the library."""
    import torch
    from paper_1007_3432_amd import inputs
    d, nx, nt = shape
    lat = hub.lattice(d, nx, nt)
    sigma, eta = inputs.sigma_eta(d, nx, nt, seed=0)
    sig_d = _dev(sigma)
    links = torch.empty(lat.volume, dtype=torch.float64, device="cuda:0")
    hub.hub_links_from_sigma(lat, sig_d, links, hub.F64)
    if phi_host is not None:
        phi = _dev(phi_host)
    else:
        eta_d = _dev(eta)
        phi = torch.empty_like(eta_d)
        hub.hub_apply_M(lat, links, hub.F64, hub.F64, eta_d, phi, 1)
    return lat, sig_d, links, phi


def timed_solves(hub, lat, sig_d, phi, opts, reps: int):
    """One warm-up solve, then `reps` timed ones (host wall clock around each
    blocking call, inputs resident on the device)."""
    import torch
    x = torch.empty_like(phi)
    hub.hub_cg_solve(lat, sig_d, phi, x, opts)
    ms, st = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = hub.hub_cg_solve(lat, sig_d, phi, x, opts)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
    return x, st, ms


def solve_record(st, ms, V, iter_bytes):
    med = statistics.median(ms)
    return {"ms_per_solve_min": min(ms), "ms_per_solve_median": med,
            "solves_per_s": 1e3 / med, "reps": len(ms), "iters": st["iters"],
            "reliable_updates": st["reliable_updates"],
            "gpu_true_rel_resid": st["true_rel_resid"], "device_ms": st["ms"],
            "us_per_iter": st["ms"] * 1e3 / max(st["iters"], 1),
            "effective_gbs": iter_bytes * V * st["iters"] / (st["ms"] / 1e3) / 1e9}


def c0_leg(hub, n_solves: int = 40, check: bool = True):
    """d=1 32 x 64 FP64 CG to 1e-10: latency-bound (2048 sites)."""
    import numpy as np
    import torch
    import oracle
    shape = (1, 32, 64)
    olat, A, phi_h = oracle_problem(shape)
    lat, sig_d, _, phi = gpu_problem(hub, shape, phi_h)
    opts = hub.cg_opts(hub.F64)
    x, st, ms = timed_solves(hub, lat, sig_d, phi, opts, n_solves)
    out = solve_record(st, ms, lat.volume, CG_ITER_BYTES_F64)
    if check:
        xh = x.cpu().numpy()
        t0 = time.perf_counter()
        x_o, res_o = oracle.cg(olat, A, phi_h)
        out["oracle_solve_ms"] = (time.perf_counter() - t0) * 1e3
        out["oracle_iters"] = res_o.iters
        out["oracle_true_rel_resid"] = oracle_true_resid(olat, A, phi_h, xh)
        out["rel_err_vs_oracle_solution"] = _rel(xh, x_o)
    return out


def cg_compare(hub, shape, link_mixed: int, reps: int = 3, check: bool = True,
               oracle_x=None):
    """FP64 CG vs mixed CG on one workload: ms per solve (min and median of
    `reps`), iterations, oracle-recomputed true residual, and the error
    against the oracle's CG solution when one is given."""
    import numpy as np
    link_name = {hub.F32: "f32", hub.F16: "f16_sin_sigma"}[link_mixed]
    if check:
        olat, A, phi_h = oracle_problem(shape)
        lat, sig_d, _, phi = gpu_problem(hub, shape, phi_h)
    else:
        lat, sig_d, _, phi = gpu_problem(hub, shape)
    V = lat.volume
    out, xs = {}, {}
    for name, opts, nbytes in (
            ("fp64", hub.cg_opts(hub.F64), CG_ITER_BYTES_F64),
            ("mixed", hub.cg_opts(hub.F32, link_mixed), CG_ITER_BYTES_MIXED[link_name])):
        x, st, ms = timed_solves(hub, lat, sig_d, phi, opts, reps)
        xs[name] = x.cpu().numpy()
        out[name] = solve_record(st, ms, V, nbytes)
        if check:
            out[name]["oracle_true_rel_resid"] = oracle_true_resid(olat, A, phi_h, xs[name])
    out["mixed"]["link"] = link_name
    out["mixed"]["rel_diff_vs_gpu_fp64_solution"] = _rel(xs["mixed"], xs["fp64"])
    out["speedup_mixed_vs_fp64_median"] = (out["fp64"]["ms_per_solve_median"]
                                           / out["mixed"]["ms_per_solve_median"])
    out["speedup_mixed_vs_fp64_min"] = (out["fp64"]["ms_per_solve_min"]
                                        / out["mixed"]["ms_per_solve_min"])
    return out, xs


def pcg_compare(hub, shape, grid):
    """FP64 CG vs Chebyshev-preconditioned FP64 CG on one workload, over a grid
    of (n, eps); the paper gives neither, so every point is reported."""
    import torch
    lat, sig_d, _, phi = gpu_problem(hub, shape)
    x = torch.empty_like(phi)
    opts = hub.cg_opts(hub.F64, max_iter=1000000)
    st = hub.hub_cg_solve(lat, sig_d, phi, x, opts)
    cg = {"ms": st["ms"], "iters": st["iters"], "q_applications": st["iters"]}
    runs = []
    for n, eps in grid:
        st = hub.hub_pcg_solve(lat, sig_d, phi, x, opts, hub.cheb_opts(n, eps))
        runs.append({"n": n, "eps": eps, "ms": st["ms"], "iters": st["iters"],
                     "q_applications": st["iters"] * (2 * n + 1),
                     "true_rel_resid": st["true_rel_resid"]})
    best = min(runs, key=lambda r: r["ms"])
    return {"cg_fp64": cg, "pcg_fp64": runs, "best": best,
            "speedup_best_pcg_vs_cg": cg["ms"] / best["ms"]}


def sweep_rate(hub, shape, sets: int, calls: int, vec=None):
    """Bare FP64 hub_apply_MtM over `sets` rotating (x, A, z) sets, `calls`
    launches captured into one HIP graph; HIP events around a replay."""
    import torch
    from paper_1007_3432_amd import inputs
    d, nx, nt = shape
    lat = hub.lattice(d, nx, nt)
    V = lat.volume
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=0)
    sig_d = _dev(sigma)
    links = [torch.empty(V, dtype=torch.float64, device="cuda:0") for _ in range(sets)]
    xs = [_dev(inputs.random_vector(V, 200 + k)) for k in range(sets)]
    zs = [torch.empty(V, dtype=torch.float64, device="cuda:0") for _ in range(sets)]
    for k in range(sets):
        hub.hub_links_from_sigma(lat, sig_d, links[k], hub.F64)
    del sig_d

    def body():
        for c in range(calls):
            k = c % sets
            hub.hub_apply_MtM(lat, links[k], hub.F64, hub.F64, xs[k], zs[k])
    body()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        body()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / calls

    # torch's z = x + a over the same rotating buffers: the same 24 B/site of
    # streaming traffic without the stencil (practical ceiling at this size).
    def adds():
        for c in range(calls):
            k = c % sets
            torch.add(xs[k], links[k], out=zs[k])
    adds()
    torch.cuda.synchronize()
    ga = torch.cuda.CUDAGraph()
    with torch.cuda.graph(ga):
        adds()
    ga.replay()
    torch.cuda.synchronize()
    e0.record()
    ga.replay()
    e1.record()
    torch.cuda.synchronize()
    add_us = e0.elapsed_time(e1) * 1e3 / calls
    del g, ga
    gbs = SWEEP_BYTES_F64 * V / us / 1e3
    return {"shape": list(shape), "sites": V, "sets": sets,
            "bytes_in_rotation": sets * 3 * 8 * V, "calls": calls,
            "avg_launch_us": us, "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS,
            "stream_add_same_bytes_us": add_us,
            "stream_add_same_bytes_gbs": SWEEP_BYTES_F64 * V / add_us / 1e3,
            "sweep_vs_stream_add": add_us / us}


def row_rates(hub, shape, sets: int, calls: int):
    """The single-operator rows on one lattice, FP64: links from sigma (8 B in,
    8 B out per site), M and M^T (x and A in, y out: 24 B/site algorithmic,
    the neighbours' re-reads served by the caches).  `calls` launches over
    `sets` rotating buffer sets, captured into one HIP graph; HIP events
    around a replay."""
    import torch
    from paper_1007_3432_amd import inputs
    d, nx, nt = shape
    lat = hub.lattice(d, nx, nt)
    V = lat.volume
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=0)
    sig = [_dev(sigma) for _ in range(sets)]
    links = [torch.empty(V, dtype=torch.float64, device="cuda:0") for _ in range(sets)]
    xs = [_dev(inputs.random_vector(V, 300 + k)) for k in range(sets)]
    ys = [torch.empty(V, dtype=torch.float64, device="cuda:0") for _ in range(sets)]
    for k in range(sets):
        hub.hub_links_from_sigma(lat, sig[k], links[k], hub.F64)
    torch.cuda.synchronize()

    def rate(body, bytes_per_site):
        body()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            body()
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / calls
        gbs = bytes_per_site * V / us / 1e3
        return {"avg_launch_us": us, "bytes_per_site": bytes_per_site, "achieved_gbs": gbs,
                "frac": gbs / HBM_PEAK_GBS}

    out = {"shape": list(shape), "sites": V, "sets": sets, "calls": calls}
    out["a1_links_f64"] = rate(lambda: [hub.hub_links_from_sigma(lat, sig[c % sets],
                                                                   links[c % sets], hub.F64)
                                        for c in range(calls)], 16)
    for name, tr in (("a2_apply_M_f64", 0), ("a3_apply_Mt_f64", 1)):
        out[name] = rate(lambda tr=tr: [hub.hub_apply_M(lat, links[c % sets], hub.F64, hub.F64,
                                                        xs[c % sets], ys[c % sets], tr)
                                        for c in range(calls)], 24)
    del sig, links, xs, ys
    return out


def cg_profile_leg(hub, iters: int):
    """A fixed number of CG iterations per solver on c2 and c3 (the solves
    stop at max_iter): a short, representative kernel mix for counter runs."""
    import torch
    out = {}
    for shape, link in (((3, 16, 160), hub.F32), ((3, 32, 256), hub.F16)):
        lat, sig_d, _, phi = gpu_problem(hub, shape)
        x = torch.empty_like(phi)
        for name, opts in (("fp64", hub.cg_opts(hub.F64, max_iter=iters)),
                           ("mixed", hub.cg_opts(hub.F32, link, max_iter=iters))):
            st = hub.hub_cg_solve(lat, sig_d, phi, x, opts, raise_on_noconv=False)
            out["d%d_%dx%d_%s" % (shape + (name,))] = {"iters": st["iters"], "ms": st["ms"]}
    return out


def force_rate(hub, shape, calls: int = 50):
    """hub_hmc_force alone (sigma 8 + x 8 in, F 8 out per site): HIP events
    around a graph replay of `calls` launches."""
    import torch
    from paper_1007_3432_amd import inputs
    d, nx, nt = shape
    lat = hub.lattice(d, nx, nt)
    V = lat.volume
    sigma, _ = inputs.sigma_eta(d, nx, nt, seed=0)
    sig_d, x_d = _dev(sigma), _dev(inputs.random_vector(V, 5))
    F = torch.empty_like(x_d)
    hub.hub_hmc_force(lat, sig_d, x_d, F)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(calls):
            hub.hub_hmc_force(lat, sig_d, x_d, F)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / calls
    return {"shape": list(shape), "avg_launch_us": us, "bytes_per_site": 24,
            "achieved_gbs": 24 * V / us / 1e3, "frac": 24 * V / us / 1e3 / HBM_PEAK_GBS,
            "buffer_sets": 1,
            "note": "one sigma, x, F set replayed: at 24 B/site it fits the 256 MiB "
                    "Infinity Cache up to 11 M sites, so the rate is partly cache-resident"}


def hmc_leg(hub, check: bool = True, n_traj: int = 20):
    """HMC trajectories (Sec. 4.1): a chain of n_traj trajectories on the
    d=1 32 x 64 lattice (10 leapfrog steps of 0.05, FP64 CG to 1e-10 per
    force), the first one also run by the oracle on the same random numbers;
    one trajectory on d=3 16^3 x 160 with mixed-precision solves; and the
    force kernel's rate at 1M and 8.4M sites."""
    import math
    import numpy as np
    import torch
    from paper_1007_3432_amd import inputs
    out = {}
    shape = (1, 32, 64)
    lat = hub.lattice(*shape)
    V = lat.volume
    sigma0, _ = inputs.sigma_eta(*shape, seed=0)
    sig_d = _dev(sigma0)
    rng = np.random.default_rng(2024)
    opts = hub.md_opts(10, 0.05, hub.cg_opts(hub.F64))
    recs, first = [], None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_traj):
        eta = rng.standard_normal(V) / math.sqrt(2.0)
        pi0 = rng.standard_normal(V)
        u = float(rng.uniform())
        if k == 0:
            first = (sig_d.cpu().numpy(), eta, pi0, u)
        st = hub.hub_hmc_trajectory(lat, sig_d, _dev(eta), _dev(pi0), u, opts)
        recs.append(st)
        if k == 0:
            first = first + (sig_d.cpu().numpy(), st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["c0_d1_32x64"] = {
        "trajectories": n_traj, "n_steps": 10, "eps": 0.05, "solver": "fp64",
        "trajectories_per_s": n_traj / dt, "ms_per_trajectory": dt / n_traj * 1e3,
        "acceptance": float(np.mean([r["accepted"] for r in recs])),
        "mean_abs_delta_h": float(np.mean([abs(r["delta_h"]) for r in recs])),
        "solves_per_trajectory": recs[0]["solves"],
        "mean_cg_iters_per_solve": float(np.mean([r["cg_iters"] / r["solves"] for r in recs]))}
    if check:
        import oracle
        s_in, eta, pi0, u, s_out, st = first
        olat = oracle.Lattice(*shape)
        s_ref, r_ref = oracle.hmc(olat, s_in, eta, pi0, u, 0.05, 10)
        out["c0_d1_32x64"]["oracle_check_first_trajectory"] = {
            "delta_h_gpu": st["delta_h"], "delta_h_oracle": r_ref.delta_h,
            "accepted_gpu": st["accepted"], "accepted_oracle": r_ref.accepted,
            "max_abs_sigma_diff": float(np.max(np.abs(s_out - s_ref)))}
    shape = (3, 16, 160)
    lat = hub.lattice(*shape)
    V = lat.volume
    sigma, _ = inputs.sigma_eta(*shape, seed=0)
    rng = np.random.default_rng(2025)
    eta = rng.standard_normal(V) / math.sqrt(2.0)
    pi0 = rng.standard_normal(V)
    sig_d = _dev(sigma)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = hub.hub_hmc_trajectory(lat, sig_d, _dev(eta), _dev(pi0), 0.5,
                                hub.md_opts(4, 0.01, hub.cg_opts(hub.F32, hub.F32)))
    torch.cuda.synchronize()
    out["c2_d3_16x160"] = dict(st, n_steps=4, eps=0.01, solver="mixed f32",
                               ms=(time.perf_counter() - t0) * 1e3)
    out["force_c1_d1_2048x512"] = force_rate(hub, (1, 2048, 512))
    out["force_c3_d3_32x256"] = force_rate(hub, (3, 32, 256), 20)
    return out


def mv_table(hub, cpu: bool = True):
    """The paper's matrix-vector experiment (Sec. 4.3, Fig. 3) on this GPU:
    Q x = M^T M x on d=3 lattices Nx in {8, 16, 32, 64} x Nt in {32, 64,
    128, 256} (and d=1 for the 30-350x context), FP64.  Per lattice: the
    fused sweep (hub_apply_MtM), the naive one-lane-per-site M then M^T
    (two hub_apply_M calls, the design the paper starts from), and the
    oracle's M^T M on one host thread (the paper's CPU methodology) and on
    all host cores.  GPU calls: repeated on one buffer set, captured in a
    HIP graph, HIP events around a replay."""
    import numpy as np
    import torch
    from paper_1007_3432_amd import inputs
    if cpu:
        import oracle
    rows = []
    grid = [(3, nx, nt) for nx in (8, 16, 32, 64) for nt in (32, 64, 128, 256)]
    grid += [(1, nx, nt) for nx in (256, 1024, 4096) for nt in (64, 256, 1024)]
    for d, nx, nt in grid:
        lat = hub.lattice(d, nx, nt)
        V = lat.volume
        rng = np.random.default_rng(7)
        sigma = rng.uniform(-np.pi, np.pi, V)
        x_h = rng.standard_normal(V)
        sig_d, x_d = _dev(sigma), _dev(x_h)
        A_d = torch.empty_like(x_d)
        hub.hub_links_from_sigma(lat, sig_d, A_d, hub.F64)
        del sig_d
        y_d, z_d = torch.empty_like(x_d), torch.empty_like(x_d)
        calls = int(min(2000, max(10, 2e9 / (24 * V))))

        def timed(body):
            body()
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                for _ in range(calls):
                    body()
            g.replay()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            g.replay()
            e1.record()
            torch.cuda.synchronize()
            del g
            return e0.elapsed_time(e1) * 1e3 / calls

        fused = timed(lambda: hub.hub_apply_MtM(lat, A_d, hub.F64, hub.F64, x_d, z_d))
        naive = timed(lambda: (hub.hub_apply_M(lat, A_d, hub.F64, hub.F64, x_d, y_d, 0),
                               hub.hub_apply_M(lat, A_d, hub.F64, hub.F64, y_d, z_d, 1)))
        row = {"d": d, "nx": nx, "nt": nt, "sites": V, "gpu_calls": calls,
               "fused_us": fused, "fused_gbs": 24 * V / fused / 1e3,
               "naive_two_pass_us": naive, "naive_gbs_at_24B": 24 * V / naive / 1e3,
               "fused_vs_naive": naive / fused}
        del x_d, y_d, z_d, A_d
        if cpu:
            olat = oracle.Lattice(d, nx, nt)
            A = oracle.links(olat, sigma)
            for label, threads in (("cpu_1thread_ms", 1), ("cpu_all_cores_ms",
                                                          os.cpu_count() or 1)):
                oracle.set_threads(threads)
                n, t0 = 0, time.perf_counter()
                while n == 0 or (time.perf_counter() - t0 < 0.3 and n < 50):
                    oracle.apply_MtM(olat, A, x_h)
                    n += 1
                row[label] = (time.perf_counter() - t0) / n * 1e3
            row["speedup_fused_vs_cpu_1thread"] = row["cpu_1thread_ms"] * 1e3 / fused
            row["speedup_naive_vs_cpu_1thread"] = row["cpu_1thread_ms"] * 1e3 / naive
            row["speedup_fused_vs_cpu_all_cores"] = row["cpu_all_cores_ms"] * 1e3 / fused
        rows.append(row)
        _progress("mv d=%d %dx%d: fused %.1f us, naive %.1f us" % (d, nx, nt, fused, naive))
        torch.cuda.empty_cache()
    return {"rows": rows, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "note": "oracle parallel loops switch on at >= 65536 sites; smaller lattices "
                    "run on one thread in both CPU columns"}


def launch_floor_us(reps: int = 1000) -> float:
    """Back-to-back graph-replayed launches of a one-element kernel."""
    import torch
    t = torch.zeros(1, device="cuda:0")
    g = torch.cuda.CUDAGraph()
    t.add_(1.0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        for _ in range(reps):
            t.add_(1.0)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def serve_bench(hub, engine: int, seconds: float, think_mean_s: float | None,
                n_chains: int = 64, check: bool = True):
    """Serving workload: n_chains HMC chains on the four lattice shapes, each
    issuing one mixed-precision solve at a time.  With think_mean_s, a chain
    waits an exponential think time after each completion (aggregate Poisson
    arrivals at n_chains / think_mean_s per second while the system keeps
    up); with None every chain resubmits at once (capacity).  Latency is
    submit -> result visible to poll."""
    import numpy as np
    import torch
    from paper_1007_3432_amd import inputs
    opts = hub.cg_opts(hub.F32, hub.F32, tol=1e-10, max_iter=200000, reliable_every=50)
    srv = hub.Server(hbm_budget_bytes=64 << 30, max_inflight=n_chains, cg=opts, engine=engine)
    rng = np.random.default_rng(7)
    chains = []
    for c in range(n_chains):
        d, nx, nt = inputs.chain_shape(c)
        lat = hub.lattice(d, nx, nt)
        sigma = inputs.chain_sigma(c)
        sig_d = torch.from_numpy(sigma).cuda()
        links = torch.empty(lat.volume, dtype=torch.float64, device="cuda")
        hub.hub_links_from_sigma(lat, sig_d, links, hub.F64)
        phis = []
        for k in range(2):
            eta = torch.from_numpy(inputs.chain_eta(c, k)).cuda()
            phi = torch.empty_like(eta)
            hub.hub_apply_M(lat, links, hub.F64, hub.F64, eta, phi, 1)
            phis.append(phi.cpu().numpy())
        chains.append({"lat": lat, "sigma": sigma, "phis": phis, "sent_sigma": False,
                       "ticket": None, "t_submit": 0.0, "next_at": 0.0, "k": 0, "phi_k": 0})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ch in chains:
        ch["next_at"] = t0 + (rng.exponential(think_mean_s) if think_mean_s else 0.0)
    done = []      # (t_done, latency_ms, iters, volume, shape key)
    samples = {}   # first served result per shape, for the oracle check
    while True:
        now = time.perf_counter()
        if now - t0 > seconds:
            break
        for c, ch in enumerate(chains):
            if ch["ticket"] is None and now >= ch["next_at"]:
                sig = None if ch["sent_sigma"] else ch["sigma"]
                ch["phi_k"] = ch["k"] % 2
                ch["ticket"] = srv.submit(c, ch["lat"], sig, ch["phis"][ch["phi_k"]])
                ch["sent_sigma"] = True
                ch["t_submit"] = time.perf_counter()
                ch["k"] += 1
            elif ch["ticket"] is not None:
                r = srv.poll(ch["ticket"], ch["lat"].volume)
                if r is not None:
                    t = time.perf_counter()
                    lat = ch["lat"]
                    key = "d%d_%dx%d" % (lat.d, lat.nx, lat.nt)
                    assert r[1]["status"] == "HUB_OK", r[1]
                    done.append((t - t0, (t - ch["t_submit"]) * 1e3, r[1]["iters"],
                                 lat.volume, key))
                    if check and key not in samples:
                        samples[key] = (c, ch["phi_k"], r[0], r[1])
                    ch["ticket"] = None
                    ch["next_at"] = t + (rng.exponential(think_mean_s) if think_mean_s else 0.0)
        time.sleep(0.0005)
    # drain
    for ch in chains:
        while ch["ticket"] is not None:
            if srv.poll(ch["ticket"], ch["lat"].volume) is not None:
                ch["ticket"] = None
            else:
                time.sleep(0.001)
    srv.close()
    # steady state: skip the first 20% of the run
    warm = 0.2 * seconds
    keep = [r for r in done if r[0] >= warm]
    span = seconds - warm
    if not keep:
        keep, span = done, seconds
    lat_ms = np.array([r[1] for r in keep])
    by_shape = {}
    for r in keep:
        s = by_shape.setdefault(r[4], {"solves": 0, "iters": []})
        s["solves"] += 1
        s["iters"].append(r[2])
    for s in by_shape.values():
        s["mean_iters"] = float(np.mean(s.pop("iters")))
    per_iter = CG_ITER_BYTES_MIXED["f32"] + RELIABLE_BYTES / opts.reliable_every
    hbm = sum(per_iter * r[2] * r[3] for r in keep) / span / 1e9
    out = {"engine": "persistent" if engine == 1 else "batched", "chains": n_chains,
           "offered_per_s": (n_chains / think_mean_s) if think_mean_s else None,
           "solves_per_s": len(keep) / span, "completed": len(done),
           "p50_latency_ms": float(np.percentile(lat_ms, 50)) if lat_ms.size else None,
           "p99_latency_ms": float(np.percentile(lat_ms, 99)) if lat_ms.size else None,
           "mean_iters": float(np.mean([r[2] for r in keep])) if keep else None,
           "by_shape": by_shape, "algorithmic_hbm_gbs": hbm,
           "hbm_frac": hbm / HBM_PEAK_GBS, "seconds": seconds,
           "steady_state_window_s": span}
    if check and samples:
        import oracle
        chk = {}
        for key, (c, k, x, st) in samples.items():
            d, nx, nt = inputs.chain_shape(c)
            olat = oracle.Lattice(d, nx, nt)
            A = oracle.links(olat, inputs.chain_sigma(c))
            phi = chains[c]["phis"][k]
            chk[key] = {"chain": c, "iters": st["iters"],
                        "oracle_true_rel_resid": oracle_true_resid(olat, A, phi, x)}
        out["oracle_check"] = chk
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(seconds: float, c2_job: OracleSolve | None):
    """The CPU oracle (FP64 C, gcc -O2 -fopenmp -ffp-contract=off, no
    -march=native) on the host cores: its M^T M sweep on the same d=1
    2048 x 512 workload for about `seconds` on all cores (the reported value)
    and for a few seconds on one core (the paper's methodology), plus the
    c0 CG solve time."""
    import numpy as np
    import oracle
    from paper_1007_3432_amd import inputs
    cores = oracle.set_threads(os.cpu_count() or 1)
    lat = oracle.Lattice(1, 2048, 512)
    sigma, eta = inputs.sigma_eta(1, 2048, 512, seed=0)
    A = oracle.links(lat, sigma)
    x = np.ascontiguousarray(eta)
    oracle.apply_MtM(lat, A, x)
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        oracle.apply_MtM(lat, A, x)
        n += 1
    dt = time.perf_counter() - t0
    gbs = SWEEP_BYTES_F64 * lat.volume * n / dt / 1e9
    oracle.set_threads(1)
    n1, t1 = 0, time.perf_counter()
    while time.perf_counter() - t1 < max(2.0, seconds / 4):
        oracle.apply_MtM(lat, A, x)
        n1 += 1
    dt1 = time.perf_counter() - t1
    olat0, A0, phi0 = oracle_problem((1, 32, 64))
    t2 = time.perf_counter()
    _, r0 = oracle.cg(olat0, A0, phi0)
    c0_1t = (time.perf_counter() - t2) * 1e3
    oracle.set_threads(cores)
    t2 = time.perf_counter()
    oracle.cg(olat0, A0, phi0)
    c0_all = (time.perf_counter() - t2) * 1e3
    out = {"value": gbs, "unit": "GB/s", "cores": cores, "kind": "oracle",
           "sample": f"{n} oracle apply_MtM calls (FP64) on d=1 2048x512 in {dt:.1f} s on "
                     f"{cores} threads, same 24 B/site accounting",
           "ms_per_call": dt / n * 1e3,
           "one_thread": {"gbs": SWEEP_BYTES_F64 * lat.volume * n1 / dt1 / 1e9,
                          "ms_per_call": dt1 / n1 * 1e3, "calls": n1},
           "cg_c0_solve_ms": {"one_thread": c0_1t, "all_cores": c0_all, "iters": r0.iters},
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "build": "gcc -std=c11 -O2 -fopenmp -ffp-contract=off -fno-fast-math "
                    "(no -march=native); stencil loops OpenMP, dot products serial"}
    if c2_job is not None and c2_job.seconds is not None:
        out["cg_c2_solve_s"] = {"threads": c2_job.threads, "seconds": c2_job.seconds,
                                "iters": c2_job.res.iters}
    return out


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                          f"--gpus {a.gpus} is not supported (single-GPU build)"}))
        sys.exit(2)
    _build_if_missing()
    import numpy as np
    import torch
    from paper_1007_3432_amd import hub, inputs
    hub.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    check = not a.no_oracle
    all_legs = {"sweeps", "c0", "c2", "c3", "pcg", "hmc", "serve"}
    if a.no_detail or a.legs == "none":
        legs = set()
    elif a.legs == "all":
        legs = set(all_legs)
    else:
        legs = set(a.legs.split(","))
        unknown = legs - all_legs - {"cgprof", "mv"}
        if unknown:
            raise SystemExit(f"unknown legs: {sorted(unknown)}")
    if a.no_serve:
        legs.discard("serve")

    # The oracle's c2 solve takes tens of seconds on the host: start it now,
    # on half the host cores, and collect it after the GPU legs.
    c2_job = None
    if "c2" in legs and check:
        c2_job = OracleSolve((3, 16, 160), threads=max(1, (os.cpu_count() or 2) // 2))
        c2_job.start()

    d, nx, nt = 1, 2048, 512
    lat = hub.lattice(d, nx, nt)
    V = lat.volume
    sigma, eta = inputs.sigma_eta(d, nx, nt, seed=0)
    sig_d, eta_d = _dev(sigma), _dev(eta)
    nsets = a.sets
    links = [torch.empty(V, dtype=torch.float64, device="cuda:0") for _ in range(nsets)]
    xs = [_dev(inputs.random_vector(V, 100 + k)) for k in range(nsets)]
    zs = [torch.empty(V, dtype=torch.float64, device="cuda:0") for _ in range(nsets)]
    phi = torch.empty_like(eta_d)
    x_cg = torch.empty_like(eta_d)
    opts = hub.cg_opts(hub.F64, max_iter=1000000)

    if a.copy_calib:
        src = torch.empty(32 * 2 ** 20, dtype=torch.float64, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    # The 1000 bare sweeps are captured once into a HIP graph and replayed
    # each step (the host would otherwise spend longer issuing 1000 launches
    # through ctypes than the GPU spends running them).
    for k in range(nsets):
        hub.hub_links_from_sigma(lat, sig_d, links[k], hub.F64)
    for k in range(nsets):
        hub.hub_apply_MtM(lat, links[k], hub.F64, hub.F64, xs[k], zs[k])
    torch.cuda.synchronize()

    def sweeps():
        for c in range(a.calls):
            k = c % nsets
            hub.hub_apply_MtM(lat, links[k], hub.F64, hub.F64, xs[k], zs[k])

    graph = None
    if not a.direct:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            sweeps()
    torch.cuda.synchronize()

    def step():
        for k in range(nsets):
            hub.hub_links_from_sigma(lat, sig_d, links[k], hub.F64)
        hub.hub_apply_M(lat, links[0], hub.F64, hub.F64, eta_d, phi, 1)
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record()
        if graph is not None:
            graph.replay()
        else:
            sweeps()
        s1.record()
        # The solve sets up its graphs on the host (and the runtime moves
        # their launch data to the device) while the sweeps still run; wait
        # for them so that only the sweeps are inside the timed region.
        s1.synchronize()
        st = hub.hub_cg_solve(lat, sig_d, phi, x_cg, opts)
        return s0, s1, st

    _progress("c1 warm-up")
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    _progress(f"c1 timed: {a.steps} steps")
    t0 = time.perf_counter()
    recs = [step() for _ in range(a.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    sweep_ms = sum(s0.elapsed_time(s1) for s0, s1, _ in recs)
    avg_kern_s = sweep_ms / 1e3 / (a.calls * a.steps)
    value = SWEEP_BYTES_F64 * V * a.calls * a.steps / (sweep_ms / 1e3) / 1e9
    achieved = SWEEP_BYTES_F64 * V / avg_kern_s / 1e9
    del graph

    # Context: the same sweeps launched one by one from Python.
    torch.cuda.synchronize()
    d0 = torch.cuda.Event(enable_timing=True)
    d1 = torch.cuda.Event(enable_timing=True)
    d0.record()
    for c in range(200):
        k = c % nsets
        hub.hub_apply_MtM(lat, links[k], hub.F64, hub.F64, xs[k], zs[k])
    d1.record()
    torch.cuda.synchronize()
    direct_us = d0.elapsed_time(d1) * 1e3 / 200
    traffic = (SWEEP_TRAFFIC["bytes"] if SWEEP_TRAFFIC and not os.environ.get("HUB_D1P_TILE")
               and not os.environ.get("HUB_SWEEP") else None)
    cg_stats = [r[2] for r in recs]
    cg_ms = [s["ms"] for s in cg_stats]
    cg_iters = cg_stats[-1]["iters"]
    c1_cg = {"iters": cg_iters, "device_ms_per_solve": statistics.mean(cg_ms),
             "device_ms_min": min(cg_ms), "device_ms_median": statistics.median(cg_ms),
             "solves_per_s": 1e3 / statistics.mean(cg_ms),
             "us_per_iter": statistics.mean(cg_ms) * 1e3 / cg_iters,
             "gpu_true_rel_resid": cg_stats[-1]["true_rel_resid"],
             "effective_gbs": CG_ITER_BYTES_F64 * V * cg_iters
             / (statistics.mean(cg_ms) / 1e3) / 1e9}
    if check:
        import oracle
        olat = oracle.Lattice(d, nx, nt)
        A_h = oracle.links(olat, sigma)
        c1_cg["oracle_true_rel_resid"] = oracle_true_resid(olat, A_h, phi.cpu().numpy(),
                                                           x_cg.cpu().numpy())
    del links, xs, zs
    torch.cuda.empty_cache()
    detail = {"sweep_direct_launch_us": direct_us,
              "sweep_direct_launch_gbs": SWEEP_BYTES_F64 * V / direct_us / 1e3,
              "cg_fp64_c1": c1_cg}
    line = {
        "metric": "MtM apply GB/s; CG solves/s FP64 vs mixed at 1e-10 resid; "
                  "p50/p99 solve latency",
        "value": value, "unit": "GB/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": wall / a.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "d=1 Nx=2048 x Nt=512 (1,048,576 sites): "
                               f"{a.calls} FP64 hub_apply_MtM over {nsets} rotating "
                               "buffer sets + 1 FP64 CG solve to 1e-10",
                   "d": d, "nx": nx, "nt": nt, "t_hop": 1.0, "dtau": 0.05, "U": -2.0,
                   "mu": 0.0, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "copy-calibrated)",
                     "kernel": "k_mtm_d1m<OpApply<double>,512,8,8> (fused M^T M sweep, two sites "
                               "per lane, 8 slices per wavefront)",
                     "avg_launch_us": avg_kern_s * 1e6,
                     "bytes_per_launch": SWEEP_BYTES_F64 * V,
                     "timing": ("HIP events around the sweeps launched one by one, / calls"
                                if a.direct else
                                "HIP events around a graph replay of the sweeps, / calls")},
        "detail": detail,
    }
    if "sweeps" in legs:
        _progress("sweep rates: c1 context, d=3 16^3x160 and 32^3x256, d=1 8192x1024")
        detail["launch_floor_us"] = launch_floor_us()
        detail["sweep_c1_d1_2048x512"] = sweep_rate(hub, (1, 2048, 512), 24, 500)
        # The same sweeps on one buffer set (25 MB, inside the 256 MB Infinity
        # Cache): the cache-resident rate, labelled as such, beside the HBM one.
        detail["sweep_c1_d1_2048x512_cache_resident_1set"] = sweep_rate(
            hub, (1, 2048, 512), 1, 500)
        detail["sweep_c2_d3_16x160"] = sweep_rate(hub, (3, 16, 160), 24, 500)
        detail["sweep_c3_d3_32x256"] = sweep_rate(hub, (3, 32, 256), 3, 60)
        detail["sweep_d1_8192x1024"] = sweep_rate(hub, (1, 8192, 1024), 3, 60)
        torch.cuda.empty_cache()
        # The single-operator rows (links, M, M^T) on c1 and c3, streamed
        # from HBM (rotating sets larger than the Infinity Cache).
        detail["rows_c1_d1_2048x512"] = row_rates(hub, (1, 2048, 512), 24, 240)
        detail["rows_c3_d3_32x256"] = row_rates(hub, (3, 32, 256), 3, 30)
        torch.cuda.empty_cache()
    if "cgprof" in legs:
        _progress(f"cgprof: {a.cgprof_iters} iterations per solver on c2 and c3")
        detail["cgprof"] = cg_profile_leg(hub, a.cgprof_iters)
    if "c0" in legs:
        _progress("c0 FP64 CG")
        detail["cg_c0_d1_32x64"] = c0_leg(hub, check=check)
    if "c2" in legs:
        _progress("c2 FP64 vs mixed CG")
        c2, c2_x = cg_compare(hub, (3, 16, 160), hub.F32, check=check)
        detail["cg_c2_d3_16x160"] = c2
    if "c3" in legs:
        _progress("c3 FP64 vs mixed CG")
        detail["cg_c3_d3_32x256"], _ = cg_compare(hub, (3, 32, 256), hub.F16, check=check)
        torch.cuda.empty_cache()
    if "pcg" in legs:
        _progress("Chebyshev PCG grids")
        grid = [(n, e) for n in (4, 8, 16, 32) for e in (1e-4, 4e-4, 1.6e-3)]
        detail["pcg_c1_d1_2048x512"] = pcg_compare(hub, (1, 2048, 512), grid)
        detail["pcg_c2_d3_16x160"] = pcg_compare(hub, (3, 16, 160), grid)
    if "hmc" in legs:
        _progress("HMC trajectories")
        detail["hmc"] = hmc_leg(hub, check=check)
    if "mv" in legs:
        _progress("MV experiment table")
        detail["mv_table"] = mv_table(hub, cpu=not a.no_cpu)
    if "serve" in legs:
        _progress("serving: Poisson 200/s")
        detail["serve_poisson_200_per_s"] = serve_bench(hub, a.engine, a.serve_seconds,
                                                       64 / 200, check=check)
        _progress("serving: capacity")
        detail["serve_capacity"] = serve_bench(hub, a.engine, a.serve_seconds, None,
                                               check=check)
    if c2_job is not None:
        _progress("waiting for the oracle's c2 solve")
        c2_job.join()
        c2 = detail["cg_c2_d3_16x160"]
        if c2_job.error:
            c2["oracle_solution_error"] = c2_job.error
        else:
            c2["oracle_iters"] = c2_job.res.iters
            c2["oracle_solve_s"] = c2_job.seconds
            for name in ("fp64", "mixed"):
                c2[name]["rel_err_vs_oracle_solution"] = _rel(c2_x[name], c2_job.x)
    if not a.no_cpu:
        _progress("CPU baseline")
        line["cpu_baseline"] = cpu_baseline(a.cpu_seconds, c2_job)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
