// Conjugate gradient on Q = M^T M (Sec. 4.1): FP64 Hestenes-Stiefel CG and
// mixed-precision CG with FP64 reliable updates, all state device-resident.
//
// One iteration is three kernels around two grid-wide reductions:
//   A  p_new = gamma r + beta p_old, q = Q p_new, x += alpha_prev p_old, and
//      one p.q deposit per tile (the fused sweep with OpPhaseA);
//   B  every block adds all p.q deposits itself (in one fixed order, so all
//      blocks get the same bits), sets alpha = rho / p.q, then r -= alpha q
//      and one r.r deposit per tile; its loads of r and q are issued before
//      that sum, so the sum costs about nothing;
//   F  one block adds the r.r deposits and sets rho, beta, the iteration
//      count and the convergence decision.
// (Taking F into the next A as well was measured slower: A's loads depend
// on beta, so the sum would sit in front of the whole sweep.)  The state
// sits in two slots: A reads slot 0, B reads slot 0 and block 0 writes the
// updated state to slot 1, F writes slot 0 from slot 1, so no block reads
// what its own launch writes.  Every kernel returns at once when the solve
// has finished (still handing the state on), so the host enqueues whole
// chunks of iterations and looks at the state only between chunks (one
// chunk ahead).  A chunk ends with a fold (x += pending alpha p [+ x_lo])
// and an FP64 true-residual sweep: always in the mixed solver (the reliable
// update), only after an iterated convergence in the FP64 solver.  The
// preconditioned solver keeps the one-block finalize after phase A as well
// (its preconditioner's 2n sweeps dwarf it).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>

#include "cgtiles.h"
#include "cheb.h"
#include "sweep.h"

namespace hub {

Link16 make_link16(const Geom& g, const void* links);

// Zero `count` consecutive scalar slots.
__global__ void k_zero_scalars(CGScalars* sc, int count) {
    uint32_t* w = reinterpret_cast<uint32_t*>(sc);
    for (int k = threadIdx.x; k < count * (int)(sizeof(CGScalars) / 4); k += blockDim.x)
        w[k] = 0;
}

// r = phi, p = 0, x = 0 (x_lo = 0), |phi|^2 (deposits; k_init_finish).
template <class RVec>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ phi,
                                              RVec* __restrict__ r, RVec* __restrict__ p0,
                                              double* __restrict__ x, float* __restrict__ xlo,
                                              int V, double* partials) {
    double part[1] = {0.0};
    tile_init<RVec>(phi, r, p0, x, xlo, V, blockIdx.x, part);
    deposit<256, 1>(part, partials, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_init_finish(CGScalars* sc, const double* partials,
                                                     int n, double tol2, double delta2,
                                                     int max_iter) {
    double tot[1];
    reduce_deposits<256, 1>(partials, n, tot);
    if (threadIdx.x == 0) finish_init(sc, tot[0], tol2, delta2, max_iter);
}

// r -= alpha q, r.r (deposits; k_phaseB_finish).
template <class Vec>
__global__ __launch_bounds__(256) void k_phaseB(const CGScalars* sc, Vec* __restrict__ r,
                                                const Vec* __restrict__ q, int V,
                                                double* partials) {
    if (sc->done != kRunning) return;
    double part[1] = {0.0};
    tile_phaseB<Vec>(r, q, (Vec)sc->alpha, V, blockIdx.x, part);
    deposit<256, 1>(part, partials, blockIdx.x);
}

// Phase B with the phase-A reduction taken in: every block adds the n_pq
// p.q deposits (the order of reduce_deposits<256, 1>), sets alpha = rho/p.q,
// then r -= alpha q and r.r deposits.  Block 0 writes the state to sc_out.
template <class Vec>
__global__ __launch_bounds__(256) void k_phaseB_fused(const CGScalars* __restrict__ sc_in,
                                                      CGScalars* __restrict__ sc_out,
                                                      const double* __restrict__ dep_pq,
                                                      int n_pq, Vec* __restrict__ r,
                                                      const Vec* __restrict__ q, int V,
                                                      double* dep_rr) {
    if (sc_in->done != kRunning) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *sc_out = *sc_in;
        return;
    }
    // The loads of r and q do not depend on alpha: issue them before the
    // reduction (a barrier does not wait for outstanding global loads).
    const int base = lane_base(blockIdx.x), cnt = lane_count(base, V);
    Vec rv[8], qv[8];
    if (cnt == 8) {
        ld8(r + base, rv);
        ld8(q + base, qv);
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            rv[k] = k < cnt ? r[base + eoff(k)] : (Vec)0;
            qv[k] = k < cnt ? q[base + eoff(k)] : (Vec)0;
        }
    }
    const double pq = reduce_deposits_canon(dep_pq, n_pq);
    CGScalars s = *sc_in;
    s.pq = pq;
    s.gamma = 1.0;
    if (!(pq > 0.0) || !isfinite(pq)) {
        s.done = kDoneBreakdown;
        s.alpha = 0.0;  // alpha_prev was applied by phase A
    } else {
        s.alpha = s.rho / pq;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *sc_out = s;
    if (s.done != kRunning) return;
    const Vec alpha = (Vec)s.alpha;
    double part[1] = {0.0};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        rv[k] = rv[k] - alpha * qv[k];
        part[0] += (double)rv[k] * (double)rv[k];
    }
    if (cnt == 8) {
        st8(r + base, rv);
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k < cnt) r[base + eoff(k)] = rv[k];
    }
    deposit<256, 1>(part, dep_rr, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_phaseB_finish(CGScalars* sc, const double* partials,
                                                       int n) {
    if (sc->done != kRunning) return;
    double tot[1];
    reduce_deposits<256, 1>(partials, n, tot);
    if (threadIdx.x == 0) finish_phaseB(sc, tot[0]);
}

// As k_phaseB_finish, reading the state from sc_in and writing it to sc_out.
// The sum does not depend on the state, so its loads go out first, beside
// the load of the state; a finished solve's state is only copied.
__global__ __launch_bounds__(256) void k_phaseB_finish_to(const CGScalars* __restrict__ sc_in,
                                                          CGScalars* __restrict__ sc_out,
                                                          const double* partials, int n) {
    double tot[1];
    reduce_deposits<256, 1>(partials, n, tot);
    if (threadIdx.x == 0) {
        CGScalars s = *sc_in;
        if (s.done == kRunning) finish_phaseB(&s, tot[0]);
        *sc_out = s;
    }
}

__global__ __launch_bounds__(256) void k_pcg_phaseB_finish(CGScalars* sc,
                                                           const double* partials, int n) {
    if (sc->done != kRunning) return;
    double tot[1];
    reduce_deposits<256, 1>(partials, n, tot);
    if (threadIdx.x == 0) finish_pcg_phaseB(sc, tot[0]);
}

// x += alpha p (+ x_lo, then x_lo = 0): the pending update, in FP64.
template <class PVec>
__global__ __launch_bounds__(256) void k_fold(CGScalars* sc, int mode, double* __restrict__ x,
                                              float* __restrict__ xlo,
                                              const PVec* __restrict__ p0,
                                              const PVec* __restrict__ p1, int V) {
    if (!mode_runs(mode, sc->done)) return;
    tile_fold<PVec>(x, xlo, (sc->iter & 1) ? p1 : p0, sc->alpha, V, blockIdx.x);
}

namespace {

// Mixed solver: besides the fixed period, recompute the true residual once
// the iterated one has dropped by this factor since the last recompute, so
// that the FP32 recurrence never runs far ahead of the FP64 residual.
constexpr double kReliableDelta = 0.1;

// Everything a captured chunk graph depends on besides device memory
// contents: geometry, options, preconditioner, the caller's phi and x, the
// workspace address.  Two solves with equal keys replay the same graphs.
using SolveKey = std::array<uint64_t, 20>;

inline uint64_t bits_of(double v) {
    uint64_t u;
    std::memcpy(&u, &v, sizeof u);
    return u;
}

// Per host thread: pinned snapshot buffers, events and the stream of the
// chunk pipeline, and the last solve's workspace and chunk graphs, kept for
// the next solve.  Freeing the workspace after every call would return its
// pages to the driver, and the page-table update that follows slows the
// caller's next kernels (measured on MI355X: the d=1 2048x512 sweep after a
// solve 6.71 us instead of 6.53 us); capturing two graphs per call costs host
// time the device waits for.
struct HostCtx {
    int device = -1;
    CGScalars* snap = nullptr;  // [2], pinned
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t t0 = nullptr, t1 = nullptr, in_ev = nullptr;
    hipStream_t stream = nullptr;  // the solve runs (and is captured) here
    char* ws = nullptr;            // solver workspace (hipMalloc), ws_bytes long
    size_t ws_bytes = 0;
    hipGraphExec_t gex[2] = {nullptr, nullptr};  // chunk graphs, valid for gkey
    bool gvalid = false;
    SolveKey gkey{};
    ~HostCtx() {
        if (device < 0) return;
        (void)hipSetDevice(device);
        release();
        if (snap) (void)hipHostFree(snap);
        for (auto e : {ev[0], ev[1], t0, t1, in_ev})
            if (e) (void)hipEventDestroy(e);
        if (stream) (void)hipStreamDestroy(stream);
    }
    void drop_graphs() {
        for (auto& e : gex) {
            if (e) (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
        gvalid = false;
    }
    // Frees the cached workspace and graphs (no solve may be running on
    // this thread: every solve has returned, so none is).
    void release() {
        drop_graphs();
        if (ws) (void)hipFree(ws);
        ws = nullptr;
        ws_bytes = 0;
    }
    // A workspace of at least `bytes`, reusing the cached one when it is
    // large enough.  Growing it drops the graphs, which point into it.
    hub_status workspace(size_t bytes, char** out) {
        if (bytes > ws_bytes) {
            release();
            if (hipMalloc((void**)&ws, bytes) != hipSuccess) {
                (void)hipGetLastError();
                ws = nullptr;
                return set_error(HUB_E_NOMEM,
                                 "hub_cg_solve: cannot allocate %zu bytes of workspace", bytes);
            }
            ws_bytes = bytes;
        }
        *out = ws;
        return HUB_OK;
    }
    hub_status ensure() {
        int dev = 0;
        HUB_HIP(hipGetDevice(&dev));
        if (dev == device) return HUB_OK;
        if (device >= 0) return set_error(HUB_E_INVALID, "hub_cg_solve: one device per thread");
        HUB_HIP(hipHostMalloc((void**)&snap, 2 * sizeof(CGScalars), hipHostMallocDefault));
        HUB_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
        HUB_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
        HUB_HIP(hipEventCreate(&t0));
        HUB_HIP(hipEventCreate(&t1));
        HUB_HIP(hipEventCreateWithFlags(&in_ev, hipEventDisableTiming));
        HUB_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        device = dev;
        return HUB_OK;
    }
};

thread_local HostCtx g_ctx;

#define HUB_TRY(expr)                       \
    do {                                    \
        hub_status s_ = (expr);             \
        if (s_ != HUB_OK) return s_;        \
    } while (0)

template <class Vec, class Lnk>
struct Solver {
    const Geom& g;
    const hub_cg_opts& o;
    hipStream_t st;
    SweepPlan P;
    // device buffers
    CGScalars* sc;     // slot 0 (slot 1 follows it)
    double* partials;  // phase A / residual / preconditioner deposits
    double* dep_rr;    // phase B deposits (fused iterations)
    const double* phi;
    double* x;
    const double* A64;
    Lnk lk;
    Vec *r, *p0, *p1, *q;
    float* xlo;        // mixed only
    double* yscratch;  // generic sweeps only (holds V doubles)
    // Chebyshev-preconditioned CG (FP64 only): z = P r before each direction
    // update; empty cheb means plain CG.
    std::vector<ChebFactor> cheb;
    double* z = nullptr;
    double* w = nullptr;
    SolveKey key{};  // what the chunk graphs depend on

    hub_status fold_and_residual(int mode) {
        k_fold<Vec><<<elem_tiles(g.V), 256, 0, st>>>(sc, mode, x, xlo, p0, p1, g.V);
        OpResidual<Vec> op{sc, x, phi, r, p0, p1, Link64{A64}, mode};
        return launch_q(g, P, op, yscratch, partials, st);
    }

    // One chunk of `iters` iterations and its closing fold / true residual,
    // then the scalars into `snap` (pinned).  Captured once into a graph.
    hub_status chunk(int iters, CGScalars* snap, bool mixed) {
        OpPhaseA<Vec, Vec, typename std::conditional<sizeof(Vec) == 8, double, float>::type, Lnk>
            opA{};
        opA.sc = sc;
        opA.r = r;
        opA.pbuf0 = p0;
        opA.pbuf1 = p1;
        opA.q = q;
        if constexpr (sizeof(Vec) == 8) opA.x = x; else opA.x = xlo;
        opA.lk = lk;
        const bool pcg = !cheb.empty();
        if constexpr (sizeof(Vec) == 8) {
            if (pcg) opA.r = z;  // p_new = z + beta p_old
        }
        if (!pcg) {
            // A reads slot 0; B reads slot 0 and writes slot 1; F writes slot 0.
            const int ne = elem_tiles(g.V);
            for (int k = 0; k < iters; ++k) {
                HUB_TRY(launch_q(g, P, opA, (Vec*)yscratch, partials, st, false));
                k_phaseB_fused<Vec><<<ne, 256, 0, st>>>(sc, sc + 1, partials, P.ntiles, r, q,
                                                        g.V, dep_rr);
                k_phaseB_finish_to<<<1, 256, 0, st>>>(sc + 1, sc, dep_rr, ne);
            }
            HUB_TRY(fold_and_residual(mixed ? kModeReliable : kModeCheck));
            HUB_HIP(hipMemcpyAsync(snap, sc, sizeof(CGScalars), hipMemcpyDeviceToHost, st));
            return HUB_OK;
        }
        for (int k = 0; k < iters; ++k) {
            if constexpr (sizeof(Vec) == 8) {
                if (pcg)
                    HUB_TRY(launch_cheb(g, P, A64, sc, r, z, w, yscratch, partials, cheb.data(),
                                        (int)cheb.size(), true, st));
            }
            HUB_TRY(launch_q(g, P, opA, (Vec*)yscratch, partials, st));
            k_phaseB<Vec><<<elem_tiles(g.V), 256, 0, st>>>(sc, r, q, g.V, partials);
            if (pcg)
                k_pcg_phaseB_finish<<<1, 256, 0, st>>>(sc, partials, elem_tiles(g.V));
            else
                k_phaseB_finish<<<1, 256, 0, st>>>(sc, partials, elem_tiles(g.V));
        }
        HUB_TRY(fold_and_residual(mixed ? kModeReliable : kModeCheck));
        HUB_HIP(hipMemcpyAsync(snap, sc, sizeof(CGScalars), hipMemcpyDeviceToHost, st));
        return HUB_OK;
    }
};

// Chunks are captured into two HIP graphs (one per snapshot buffer) and
// replayed: the host then pays one graph launch per chunk instead of four
// kernel launches per iteration.  HUB_CG_GRAPH=0 launches kernels directly.
inline bool use_graphs() {
    static bool v = [] {
        const char* e = std::getenv("HUB_CG_GRAPH");
        return !(e && e[0] == '0');
    }();
    return v;
}

template <class Vec, class Lnk>
hub_status capture_chunk(Solver<Vec, Lnk>& S, int iters, CGScalars* snap, bool mixed,
                         hipGraphExec_t* out) {
    HUB_HIP(hipStreamBeginCapture(S.st, hipStreamCaptureModeThreadLocal));
    const hub_status body = S.chunk(iters, snap, mixed);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(S.st, &gr);
    if (body != HUB_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return body;
    }
    if (e != hipSuccess)
        return set_error(HUB_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(out, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e2 != hipSuccess)
        return set_error(HUB_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e2));
    return HUB_OK;
}

template <class Vec, class Lnk>
hub_status run_solver(Solver<Vec, Lnk>& S, bool mixed, hub_cg_stats* out) {
    const Geom& g = S.g;
    const hub_cg_opts& o = S.o;
    HostCtx& H = g_ctx;
    // Work the caller queued on its stream (sigma, phi) comes first.
    HUB_HIP(hipEventRecord(H.in_ev, S.st));
    HUB_HIP(hipStreamWaitEvent(H.stream, H.in_ev, 0));
    S.st = H.stream;
    hipStream_t st = S.st;
    HUB_HIP(hipEventRecord(H.t0, st));
    k_zero_scalars<<<1, 64, 0, st>>>(S.sc, 2);
    k_init<Vec><<<elem_tiles(g.V), 256, 0, st>>>(S.phi, S.r, S.p0, S.x, S.xlo, g.V, S.partials);
    k_init_finish<<<1, 256, 0, st>>>(S.sc, S.partials, elem_tiles(g.V), o.tol * o.tol,
                                     mixed ? kReliableDelta * kReliableDelta : 0.0, o.max_iter);
    HUB_HIP(hipGetLastError());
    // Iterations per chunk: about 150 sweeps for plain CG (50 its), the
    // reliable-update period for mixed CG, and about 200 sweeps (each
    // iteration 2n + 1) with the preconditioner.
    const int C = mixed ? o.reliable_every
                        : (S.cheb.empty() ? 50
                                          : std::max(2, 200 / (2 * (int)S.cheb.size() + 1)));
    // The chunk graphs of the previous solve on this thread are replayed
    // when nothing they depend on has changed; otherwise they are captured
    // again.
    const bool graphs = use_graphs();
    if (graphs && !(H.gvalid && H.gkey == S.key)) {
        H.drop_graphs();
        HUB_TRY(capture_chunk(S, C, &H.snap[0], mixed, &H.gex[0]));
        HUB_TRY(capture_chunk(S, C, &H.snap[1], mixed, &H.gex[1]));
        H.gkey = S.key;
        H.gvalid = true;
    }
    auto enqueue = [&](int slot) -> hub_status {
        if (graphs) {
            HUB_HIP(hipGraphLaunch(H.gex[slot], st));
        } else {
            HUB_TRY(S.chunk(C, &H.snap[slot], mixed));
        }
        HUB_HIP(hipEventRecord(H.ev[slot], st));
        return HUB_OK;
    };
    // Every chunk either runs at least one iteration or ends the solve, so
    // this bound is never reached by a healthy solve.
    const long long max_chunks = 2LL * (o.max_iter / C + 2) + 8;
    HUB_TRY(enqueue(0));
    HUB_TRY(enqueue(1));
    long long enq = 2;
    int cur = 0;
    CGScalars s{};
    for (;;) {
        HUB_HIP(hipEventSynchronize(H.ev[cur]));
        s = H.snap[cur];
        if (s.done >= kDoneConverged) break;
        if (enq >= max_chunks) {
            (void)hipStreamSynchronize(st);
            return set_error(HUB_E_NOCONV, "hub_cg_solve: chunk limit reached");
        }
        HUB_TRY(enqueue(cur));
        ++enq;
        cur ^= 1;
    }
    if (s.done != kDoneConverged) HUB_TRY(S.fold_and_residual(kModeFinal));
    HUB_HIP(hipMemcpyAsync(&H.snap[cur], S.sc, sizeof(CGScalars), hipMemcpyDeviceToHost, st));
    HUB_HIP(hipEventRecord(H.t1, st));
    HUB_HIP(hipStreamSynchronize(st));
    s = H.snap[cur];
    float ms = 0.0f;
    HUB_HIP(hipEventElapsedTime(&ms, H.t0, H.t1));
    hub_cg_stats stats{};
    stats.iters = s.iter;
    stats.reliable_updates = s.reliable_updates;
    stats.true_rel_resid = s.phi2 > 0 ? std::sqrt(s.rho_true / s.phi2) : 0.0;
    stats.ms = ms;
    stats.status = s.done == kDoneConverged ? HUB_OK : HUB_E_NOCONV;
    if (out) *out = stats;
    if (stats.status != HUB_OK)
        return set_error(HUB_E_NOCONV,
                         "CG did not converge: %d iterations, true relative residual %.3e%s",
                         s.iter, stats.true_rel_resid,
                         s.done == kDoneBreakdown ? " (breakdown)" : "");
    return HUB_OK;
}

}  // namespace

namespace {

hub_status solve(const Geom& g, const double* sigma, const double* phi, double* x,
                 const hub_cg_opts& o, const hub_cheb_opts* cheb, hub_cg_stats* out,
                 hipStream_t st) {
    const bool mixed = o.bulk == HUB_F32;
    // A lattice that fits one workgroup is solved inside it: the iteration is
    // then bound by barriers, not by three kernel launches.
    if (!mixed && !cheb && cg_small_fits(g)) return cg_solve_small(g, sigma, phi, x, o, out, st);
    HUB_TRY(g_ctx.ensure());
    const size_t V = (size_t)g.V;
    const size_t vb = mixed ? 4 : 8;
    const SweepPlan P = plan_sweep(g, !mixed, true);
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    size_t off = 0;
    const size_t o_sc = off; off += al(2 * sizeof(CGScalars));
    const size_t o_part = off; off += al(sizeof(double) * max_partials(g));
    const size_t o_rr = off; off += al(sizeof(double) * elem_tiles(g.V));
    const size_t o_A64 = off; off += al(8 * V);
    const size_t o_lnk = off; off += mixed ? al(dtype_size(o.link) * V) : 0;
    const size_t o_r = off; off += al(vb * V);
    const size_t o_p0 = off; off += al(vb * V);
    const size_t o_p1 = off; off += al(vb * V);
    const size_t o_q = off; off += al(vb * V);
    const size_t o_xlo = off; off += mixed ? al(4 * V) : 0;
    const size_t o_y = off; off += P.fused ? 0 : al(8 * V);
    const size_t o_z = off; off += cheb ? al(8 * V) : 0;
    const size_t o_w = off; off += cheb ? al(8 * V) : 0;
    char* ws = nullptr;
    HUB_TRY(g_ctx.workspace(off, &ws));
    const double cheb_scale =
        cheb ? (cheb->scale > 0 ? cheb->scale : cheb_default_scale(g)) : 0.0;
    const SolveKey key = {(uint64_t)g.d, (uint64_t)g.nx, (uint64_t)g.nt, bits_of(g.kappa),
                          bits_of(g.lscale), bits_of(g.b), (uint64_t)o.bulk,
                          (uint64_t)o.link, bits_of(o.tol), (uint64_t)(uint32_t)o.max_iter,
                          (uint64_t)(uint32_t)o.reliable_every,
                          cheb ? (uint64_t)(uint32_t)cheb->n : 0,
                          cheb ? bits_of(cheb->eps) : 0, bits_of(cheb_scale),
                          (uint64_t)(uintptr_t)phi, (uint64_t)(uintptr_t)x,
                          (uint64_t)(uintptr_t)ws, (uint64_t)off, 0, 0};
    hub_status result = HUB_OK;
    const double* A64 = (const double*)(ws + o_A64);
    result = launch_links(g, sigma, ws + o_A64, HUB_F64, st);
    if (result == HUB_OK && mixed) result = launch_links(g, sigma, ws + o_lnk, o.link, st);
    if (result == HUB_OK) {
        if (!mixed) {
            Solver<double, Link64> S{g, o, st, P};
            S.sc = (CGScalars*)(ws + o_sc);
            S.partials = (double*)(ws + o_part);
            S.dep_rr = (double*)(ws + o_rr);
            S.phi = phi;
            S.x = x;
            S.A64 = A64;
            S.lk = Link64{A64};
            S.r = (double*)(ws + o_r);
            S.p0 = (double*)(ws + o_p0);
            S.p1 = (double*)(ws + o_p1);
            S.q = (double*)(ws + o_q);
            S.xlo = nullptr;
            S.yscratch = P.fused ? nullptr : (double*)(ws + o_y);
            S.key = key;
            if (cheb) {
                S.cheb = cheb_factors(cheb->n, cheb->eps, cheb_scale);
                S.z = (double*)(ws + o_z);
                S.w = (double*)(ws + o_w);
            }
            result = run_solver(S, false, out);
        } else if (o.link == HUB_F32) {
            Solver<float, Link32> S{g, o, st, P};
            S.sc = (CGScalars*)(ws + o_sc);
            S.partials = (double*)(ws + o_part);
            S.dep_rr = (double*)(ws + o_rr);
            S.phi = phi;
            S.x = x;
            S.A64 = A64;
            S.lk = Link32{(const float*)(ws + o_lnk)};
            S.r = (float*)(ws + o_r);
            S.p0 = (float*)(ws + o_p0);
            S.p1 = (float*)(ws + o_p1);
            S.q = (float*)(ws + o_q);
            S.xlo = (float*)(ws + o_xlo);
            S.yscratch = P.fused ? nullptr : (double*)(ws + o_y);
            S.key = key;
            result = run_solver(S, true, out);
        } else {
            Solver<float, Link16> S{g, o, st, P};
            S.sc = (CGScalars*)(ws + o_sc);
            S.partials = (double*)(ws + o_part);
            S.dep_rr = (double*)(ws + o_rr);
            S.phi = phi;
            S.x = x;
            S.A64 = A64;
            S.lk = make_link16(g, ws + o_lnk);
            S.r = (float*)(ws + o_r);
            S.p0 = (float*)(ws + o_p0);
            S.p1 = (float*)(ws + o_p1);
            S.q = (float*)(ws + o_q);
            S.xlo = (float*)(ws + o_xlo);
            S.yscratch = P.fused ? nullptr : (double*)(ws + o_y);
            S.key = key;
            result = run_solver(S, true, out);
        }
    }
    // The solve ran on the context stream: let it drain (also on an error
    // path) before the workspace can be used again, and let the caller's
    // stream drain too (the links were computed there).
    const hipError_t e = hipStreamSynchronize(g_ctx.stream);
    const hipError_t e2 = hipStreamSynchronize(st);
    if (result == HUB_OK && (e != hipSuccess || e2 != hipSuccess))
        return set_error(HUB_E_DEVICE, "hub_cg_solve: %s",
                         hipGetErrorString(e != hipSuccess ? e : e2));
    return result;
}

}  // namespace

hub_status solver_workspace(size_t bytes, char** out) {
    HUB_TRY(g_ctx.ensure());
    return g_ctx.workspace(bytes, out);
}

// Nothing of this thread's runs on the context stream: every solve waits
// for its work before returning.
void solver_release() { g_ctx.release(); }

hub_status cg_solve(const Geom& g, const double* sigma, const double* phi, double* x,
                    const hub_cg_opts& o, hub_cg_stats* out, hipStream_t st) {
    return solve(g, sigma, phi, x, o, nullptr, out, st);
}

hub_status pcg_solve(const Geom& g, const double* sigma, const double* phi, double* x,
                     const hub_cg_opts& o, const hub_cheb_opts& c, hub_cg_stats* out,
                     hipStream_t st) {
    return solve(g, sigma, phi, x, o, &c, out, st);
}

// ---------------------------------------------------------------------------
// Set-up and wrap-up of one solve of the serving kernel: the same kernels the
// one-solve path runs before its first and after its last chunk.

double reliable_delta() { return kReliableDelta; }

hub_status serve_slot_init(const Geom& g, CGScalars* sc, const double* phi, float* r, float* p0,
                           double* x, float* xlo, double tol2, double delta2, int max_iter,
                           double* partials, hipStream_t st) {
    k_zero_scalars<<<1, 64, 0, st>>>(sc, 1);
    k_init<float><<<elem_tiles(g.V), 256, 0, st>>>(phi, r, p0, x, xlo, g.V, partials);
    k_init_finish<<<1, 256, 0, st>>>(sc, partials, elem_tiles(g.V), tol2, delta2, max_iter);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status serve_slot_final(const Geom& g, const SweepPlan& P, CGScalars* sc, const double* phi,
                            double* x, float* xlo, float* r, float* p0, float* p1,
                            const double* A64, double* partials, hipStream_t st) {
    k_fold<float><<<elem_tiles(g.V), 256, 0, st>>>(sc, kModeFinal, x, xlo, p0, p1, g.V);
    OpResidual<float> op{sc, x, phi, r, p0, p1, Link64{A64}, kModeFinal};
    return launch_q(g, P, op, nullptr, partials, st);
}

}  // namespace hub
