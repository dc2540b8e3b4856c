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
around the graph replay, divided by the calls) against the 8 TB/s HBM peak.  `detail` holds
the CG solve rates (FP64 vs mixed precision on the d=3 workloads) and, with
--serve, the served solves/s and latency percentiles.  `cpu_baseline` times
the CPU oracle on a bounded sample of the same sweep on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SWEEP_BYTES_F64 = 24       # per site: x 8 + A 8 + z 8
CG_ITER_BYTES_F64 = 80     # per site and iteration (phase A 56 + phase B 24)

# HBM bytes one launch of the timed sweep (k_mtm_d1p<OpApply<double>, 512, 2>
# on d=1 2048 x 512) actually moves: rocprofv3 FETCH_SIZE x 2.000 plus
# WRITE_SIZE x 1.000 per dispatch, each factor calibrated on a 256 MiB copy.
# Valid only for that kernel and tile; None once either changes.
SWEEP_TRAFFIC = {"kernel": "k_mtm_d1p<OpApply<double>,512,2>", "bytes": 25_612_871}


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--calls", type=int, default=1000, help="bare sweeps per step")
    ap.add_argument("--sets", type=int, default=24, help="rotating buffer sets")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-detail", action="store_true", help="skip the d=3 CG comparisons")
    ap.add_argument("--serve", action="store_true", help="also run the serving workload")
    ap.add_argument("--engine", type=int, default=0, help="serving engine: 0 batched, 1 persistent")
    ap.add_argument("--serve-seconds", type=float, default=15.0)
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


def cg_compare(hub, inputs, shape, link_mixed, reps=1):
    """FP64 CG vs mixed CG on one workload; solves/s and speedup."""
    import torch
    d, nx, nt = shape
    lat = hub.lattice(d, nx, nt)
    V = lat.volume
    sigma, eta = inputs.sigma_eta(d, nx, nt, seed=0)
    sig_d, eta_d = _dev(sigma), _dev(eta)
    links = torch.empty(V, dtype=torch.float64, device="cuda:0")
    hub.hub_links_from_sigma(lat, sig_d, links, hub.F64)
    phi = torch.empty_like(eta_d)
    hub.hub_apply_M(lat, links, hub.F64, hub.F64, eta_d, phi, 1)
    out = {}
    xs = {}
    for name, opts in (("fp64", hub.cg_opts(hub.F64)),
                       ("mixed", hub.cg_opts(hub.F32, link_mixed))):
        x = torch.empty_like(phi)
        hub.hub_cg_solve(lat, sig_d, phi, x, opts)           # warm-up
        ms = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = hub.hub_cg_solve(lat, sig_d, phi, x, opts)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
        xs[name] = x
        out[name] = {"ms_per_solve": min(ms), "solves_per_s": 1e3 / min(ms),
                     "iters": st["iters"], "reliable_updates": st["reliable_updates"],
                     "true_rel_resid": st["true_rel_resid"],
                     "device_ms": st["ms"]}
    out["mixed"]["link"] = {hub.F32: "f32", hub.F16: "f16_sin_sigma"}[link_mixed]
    diff = (xs["mixed"] - xs["fp64"]).norm() / xs["fp64"].norm()
    out["mixed"]["rel_diff_vs_fp64_solution"] = float(diff)
    out["speedup_mixed_vs_fp64"] = out["fp64"]["ms_per_solve"] / out["mixed"]["ms_per_solve"]
    return out


def pcg_compare(hub, inputs, shape, grid):
    """FP64 CG vs Chebyshev-preconditioned FP64 CG on one workload, over a grid
    of (n, eps); the paper gives neither, so every point is reported."""
    import torch
    d, nx, nt = shape
    lat = hub.lattice(d, nx, nt)
    sigma, eta = inputs.sigma_eta(d, nx, nt, seed=0)
    sig_d, eta_d = _dev(sigma), _dev(eta)
    links = torch.empty(lat.volume, dtype=torch.float64, device="cuda:0")
    hub.hub_links_from_sigma(lat, sig_d, links, hub.F64)
    phi = torch.empty_like(eta_d)
    hub.hub_apply_M(lat, links, hub.F64, hub.F64, eta_d, phi, 1)
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


def serve_bench(hub, inputs, engine: int, seconds: float, think_mean_s: float | None,
                n_chains: int = 64):
    """Serving workload: n_chains HMC chains on the four lattice shapes, each
    issuing one mixed-precision solve at a time.  With think_mean_s, a chain
    waits an exponential think time after each completion (aggregate Poisson
    arrivals at n_chains / think_mean_s per second while the system keeps
    up); with None every chain resubmits at once (capacity).  Latency is
    submit -> result visible to poll."""
    import numpy as np
    import torch
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
                       "ticket": None, "t_submit": 0.0, "next_at": 0.0, "k": 0})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ch in chains:
        ch["next_at"] = t0 + (rng.exponential(think_mean_s) if think_mean_s else 0.0)
    lat_ms, iters, done_t = [], [], []
    shapes = {}
    while True:
        now = time.perf_counter()
        if now - t0 > seconds:
            break
        for c, ch in enumerate(chains):
            if ch["ticket"] is None and now >= ch["next_at"]:
                sig = None if ch["sent_sigma"] else ch["sigma"]
                ch["ticket"] = srv.submit(c, ch["lat"], sig, ch["phis"][ch["k"] % 2])
                ch["sent_sigma"] = True
                ch["t_submit"] = time.perf_counter()
                ch["k"] += 1
            elif ch["ticket"] is not None:
                r = srv.poll(ch["ticket"], ch["lat"].volume)
                if r is not None:
                    t = time.perf_counter()
                    lat_ms.append((t - ch["t_submit"]) * 1e3)
                    iters.append(r[1]["iters"])
                    done_t.append(t - t0)
                    key = "d%d_%dx%d" % (ch["lat"].d, ch["lat"].nx, ch["lat"].nt)
                    shapes[key] = shapes.get(key, 0) + 1
                    assert r[1]["status"] == "HUB_OK", r[1]
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
    keep = [i for i, t in enumerate(done_t) if t >= warm]
    lat_keep = np.array([lat_ms[i] for i in keep]) if keep else np.array(lat_ms)
    rate = len(keep) / (seconds - warm) if keep else len(done_t) / seconds
    return {"engine": "persistent" if engine == 1 else "batched",
            "chains": n_chains, "offered_per_s": (n_chains / think_mean_s) if think_mean_s else None,
            "solves_per_s": rate, "completed": len(done_t),
            "p50_latency_ms": float(np.percentile(lat_keep, 50)) if lat_keep.size else None,
            "p99_latency_ms": float(np.percentile(lat_keep, 99)) if lat_keep.size else None,
            "mean_iters": float(np.mean(iters)) if iters else None, "by_shape": shapes,
            "seconds": seconds}


def cpu_baseline(inputs, seconds: float):
    """The CPU oracle's M^T M sweep on the host cores, same d=1 2048 x 512
    workload, as many calls as fit in about `seconds`."""
    import numpy as np
    import oracle
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
    return {"value": gbs, "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} oracle apply_MtM calls (FP64) on d=1 2048x512 "
                      f"in {dt:.1f} s, same 24 B/site accounting",
            "ms_per_call": dt / n * 1e3}


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
        st = hub.hub_cg_solve(lat, sig_d, phi, x_cg, opts)
        return s0, s1, st

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [step() for _ in range(a.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    sweep_ms = sum(s0.elapsed_time(s1) for s0, s1, _ in recs)
    avg_kern_s = sweep_ms / 1e3 / (a.calls * a.steps)
    value = SWEEP_BYTES_F64 * V * a.calls * a.steps / (sweep_ms / 1e3) / 1e9
    achieved = SWEEP_BYTES_F64 * V / avg_kern_s / 1e9

    # Context: a plain streaming kernel (torch's z = x + a) over the same
    # rotating buffers moves the same 24 B/site; its rate is the practical
    # HBM ceiling at this transfer size.
    def adds():
        for c in range(a.calls):
            k = c % nsets
            torch.add(xs[k], links[k], out=zs[k])
    adds()
    torch.cuda.synchronize()
    add_graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(add_graph):
        adds()
    add_graph.replay()
    torch.cuda.synchronize()
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record()
    add_graph.replay()
    c1.record()
    torch.cuda.synchronize()
    add_us = c0.elapsed_time(c1) * 1e3 / a.calls
    del add_graph

    # For reference: the same sweeps launched one by one from Python.
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
                     "kernel": "k_mtm_d1p<OpApply<double>,512,2> (fused M^T M sweep, two sites per lane)",
                     "avg_launch_us": avg_kern_s * 1e6,
                     "bytes_per_launch": SWEEP_BYTES_F64 * V,
                     "timing": ("HIP events around the sweeps launched one by one, / calls"
                                if a.direct else
                                "HIP events around a graph replay of the sweeps, / calls")},
        "detail": {
            "stream_add_same_bytes_us": add_us,
            "stream_add_same_bytes_gbs": SWEEP_BYTES_F64 * V / add_us / 1e3,
            "sweep_vs_stream_add": add_us / avg_kern_s / 1e6,
            "sweep_direct_launch_us": direct_us,
            "sweep_direct_launch_gbs": SWEEP_BYTES_F64 * V / direct_us / 1e3,
            "cg_fp64_c1": {"iters": cg_iters, "device_ms_per_solve": statistics.mean(cg_ms),
                           "solves_per_s": 1e3 / statistics.mean(cg_ms),
                           "true_rel_resid": cg_stats[-1]["true_rel_resid"],
                           "effective_gbs": CG_ITER_BYTES_F64 * V * cg_iters
                           / (statistics.mean(cg_ms) / 1e3) / 1e9},
        },
    }
    if not a.no_detail:
        line["detail"]["cg_c2_d3_16x160"] = cg_compare(hub, inputs, (3, 16, 160), hub.F32)
        line["detail"]["cg_c3_d3_32x256"] = cg_compare(hub, inputs, (3, 32, 256), hub.F16)
        grid = [(n, e) for n in (4, 8, 16, 32) for e in (1e-4, 4e-4, 1.6e-3)]
        line["detail"]["pcg_c1_d1_2048x512"] = pcg_compare(hub, inputs, (1, 2048, 512), grid)
        line["detail"]["pcg_c2_d3_16x160"] = pcg_compare(hub, inputs, (3, 16, 160), grid)
    if a.serve:
        line["detail"]["serve_poisson_200_per_s"] = serve_bench(hub, inputs, a.engine,
                                                               a.serve_seconds, 64 / 200)
        line["detail"]["serve_capacity"] = serve_bench(hub, inputs, a.engine,
                                                       a.serve_seconds, None)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(inputs, a.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
