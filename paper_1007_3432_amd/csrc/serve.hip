// Serving: continuous batching of mixed-precision CG solves from many HMC
// chains (each chain issues one solve of Q x = phi per molecular-dynamics
// force evaluation, Sec. 4.1).
//
// Host side: one worker thread per server owns a HIP stream, the resident
// per-chain state (field sigma, FP64 links, bulk links) and a slot table of
// in-flight solves (Krylov vectors, scalars, deposits).  Requests are admitted
// in arrival order while their footprint fits the HBM budget and a slot is
// free; idle chains are evicted least-recently-used when memory is needed.
//
// Device side: one cooperative persistent kernel per epoch steps every
// in-flight solve through reliable_every CG iterations and the reliable
// update that closes them.  Each phase pools the tiles of all solves; grid
// barriers separate the phases.  Every tile and every reduction runs the same
// device functions, in the same order, as the one-solve path (hub_cg_solve),
// so a solve gives the same bits alone and in the mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "cgtiles.h"
#include "sweep.h"

namespace hub {

Link16 make_link16(const Geom& g, const void* links);

// Launch geometry of the solves the serving kernel can step (the default
// fused plans; see plan_sweep).
static bool serve_supported(const SweepPlan& P) {
    if (P.kind == kSweepD1)
        return P.variant == kD1_256x4 || P.variant == kD1_128x4 || P.variant == kD1_64x4;
    if (P.kind == kSweepD3)
        return P.variant == kD3_8x8x8 || P.variant == kD3_16x4x4 || P.variant == kD3_32x8x4;
    return false;
}

// One in-flight solve as the epoch kernel sees it.
struct SlotDesc {
    Geom g;
    int kind, variant, tiles_x, tiles_y, tiles_z, tc;
    int sweep_tiles, elem_tiles;
    int off_sweep, off_elem;  // first work item of this solve in each phase
    CGScalars* sc;
    double* partials;
    const double* phi;
    double* x;
    const double* A64;
    const void* lnk;
    float *r, *p0, *p1, *q, *xlo;
};

struct EpochCtl {
    uint32_t count;
    uint32_t gen;
    int32_t abort;
    int32_t pad;
};

// LDS elements a serving tile needs (d = 1 tiles use none).
static int serve_lds_elems(int kind, int variant) {
    if (kind != kSweepD3) return 0;
    switch (variant) {
        case kD3_8x8x8: return d3_lds_elems<8, 8, 8>();
        case kD3_16x4x4: return d3_lds_elems<16, 4, 4>();
        default: return d3_lds_elems<32, 8, 4>();
    }
}

// LDS of the largest tile the serving kernel runs (FP64 residual sweeps):
// what the persistent engine reserves, as its one launch runs every phase.
constexpr int kServeLdsBytes = [] {
    int m = d1_lds_elems<256, 4>();
    m = std::max(m, d3_lds_elems<8, 8, 8>());
    m = std::max(m, d3_lds_elems<16, 4, 4>());
    m = std::max(m, d3_lds_elems<32, 8, 4>());
    return m * 8;
}();

// Grid barrier for a cooperative launch.  Bounded: after spin_limit polls a
// block gives up, raises abort and every block leaves at its next barrier,
// so the kernel always terminates.
__device__ bool grid_barrier(EpochCtl* ctl, long spin_limit) {
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        ok = 1;
        const uint32_t g0 = __hip_atomic_load(&ctl->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t arrived =
            __hip_atomic_fetch_add(&ctl->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1;
        if (arrived == gridDim.x) {
            __hip_atomic_store(&ctl->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&ctl->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long spins = 0;
            while (__hip_atomic_load(&ctl->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
                if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                    ++spins > spin_limit) {
                    __hip_atomic_store(&ctl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
    }
    __syncthreads();
    return ok != 0;
}

// Solve owning work item w of a phase (offsets ascend with the slot index).
__device__ inline int find_slot(const SlotDesc* S, int n, int w, bool sweep) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int off = sweep ? S[mid].off_sweep : S[mid].off_elem;
        if (off <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <class Lnk>
__device__ Lnk slot_link(const SlotDesc& S);
template <>
__device__ Link32 slot_link<Link32>(const SlotDesc& S) { return Link32{(const float*)S.lnk}; }
template <>
__device__ Link16 slot_link<Link16>(const SlotDesc& S) {
    Link16 l;
    l.sn = (const _Float16*)S.lnk;
    l.ls = (float)S.g.lscale;
    l.lb = (float)(S.g.lscale * S.g.b);
    return l;
}

template <class Lnk>
__device__ OpPhaseA<float, float, float, Lnk> slot_phaseA(const SlotDesc& S) {
    OpPhaseA<float, float, float, Lnk> op{};
    op.sc = S.sc;
    op.r = S.r;
    op.pbuf0 = S.p0;
    op.pbuf1 = S.p1;
    op.q = S.q;
    op.x = S.xlo;
    op.lk = slot_link<Lnk>(S);
    (void)op.begin();
    return op;
}

__device__ OpResidual<float> slot_residual(const SlotDesc& S) {
    OpResidual<float> op{S.sc, S.x, S.phi, S.r, S.p0, S.p1, Link64{S.A64}, kModeReliable};
    (void)op.begin();
    return op;
}

// Dynamic LDS of the epoch kernel, shared by every tile function it calls.
extern __shared__ __align__(16) char serve_smem[];

struct Sums2 {
    double a, b;
};

// One sweep tile of solve *S.  Returns the block sums (thread 0).  The
// batched engine launches one kernel per tile shape, with these bodies
// inlined; the persistent engine runs every shape in one kernel and calls
// them as functions (serve_tile_A / serve_tile_R), each (op, tile shape)
// pair register-allocated on its own.
template <class Lnk, int KIND, int A, int B, int C>
__device__ __forceinline__ Sums2 serve_tile_A_body(const SlotDesc* S, int tile) {
    const auto op = slot_phaseA<Lnk>(*S);
    double part[1] = {0.0};
    float* lds = reinterpret_cast<float*>(serve_smem);
    if constexpr (KIND == kSweepD1)
        tile_mtm_d1<decltype(op), A, B>(S->g, op, S->tiles_x, tile, lds, part);
    else
        tile_mtm_d3<decltype(op), A, B, C, 256>(S->g, op, S->tiles_y, S->tiles_z, S->tc, tile,
                                                lds, part);
    Sums2 r{block_sum<256>(part[0]), 0.0};
    return r;
}

template <int KIND, int A, int B, int C>
__device__ __forceinline__ Sums2 serve_tile_R_body(const SlotDesc* S, int tile) {
    const auto op = slot_residual(*S);
    double part[2] = {0.0, 0.0};
    double* lds = reinterpret_cast<double*>(serve_smem);
    if constexpr (KIND == kSweepD1)
        tile_mtm_d1<decltype(op), A, B>(S->g, op, S->tiles_x, tile, lds, part);
    else
        tile_mtm_d3<decltype(op), A, B, C, 256>(S->g, op, S->tiles_y, S->tiles_z, S->tc, tile,
                                                lds, part);
    Sums2 r;
    r.a = block_sum<256>(part[0]);
    r.b = block_sum<256>(part[1]);
    return r;
}

template <class Lnk, int KIND, int A, int B, int C>
__device__ __noinline__ Sums2 serve_tile_A(const SlotDesc* S, int tile) {
    return serve_tile_A_body<Lnk, KIND, A, B, C>(S, tile);
}

template <int KIND, int A, int B, int C>
__device__ __noinline__ Sums2 serve_tile_R(const SlotDesc* S, int tile) {
    return serve_tile_R_body<KIND, A, B, C>(S, tile);
}

template <class Lnk>
__device__ Sums2 serve_sweep_A(const SlotDesc* S, int tile) {
    if (S->kind == kSweepD1) {
        switch (S->variant) {
            case kD1_256x4: return serve_tile_A<Lnk, kSweepD1, 256, 4, 0>(S, tile);
            case kD1_128x4: return serve_tile_A<Lnk, kSweepD1, 128, 4, 0>(S, tile);
            default: return serve_tile_A<Lnk, kSweepD1, 64, 4, 0>(S, tile);
        }
    }
    switch (S->variant) {
        case kD3_8x8x8: return serve_tile_A<Lnk, kSweepD3, 8, 8, 8>(S, tile);
        case kD3_16x4x4: return serve_tile_A<Lnk, kSweepD3, 16, 4, 4>(S, tile);
        default: return serve_tile_A<Lnk, kSweepD3, 32, 8, 4>(S, tile);
    }
}

__device__ Sums2 serve_sweep_R(const SlotDesc* S, int tile) {
    if (S->kind == kSweepD1) {
        switch (S->variant) {
            case kD1_256x4: return serve_tile_R<kSweepD1, 256, 4, 0>(S, tile);
            case kD1_128x4: return serve_tile_R<kSweepD1, 128, 4, 0>(S, tile);
            default: return serve_tile_R<kSweepD1, 64, 4, 0>(S, tile);
        }
    }
    switch (S->variant) {
        case kD3_8x8x8: return serve_tile_R<kSweepD3, 8, 8, 8>(S, tile);
        case kD3_16x4x4: return serve_tile_R<kSweepD3, 16, 4, 4>(S, tile);
        default: return serve_tile_R<kSweepD3, 32, 8, 4>(S, tile);
    }
}

// Thread 0 stores the block sums of a tile into its deposit slot.
template <int NP>
__device__ inline void store_deposit(const Sums2& s, double* partials, int slot) {
    if (threadIdx.x == 0) {
        __hip_atomic_store(&partials[NP * slot], s.a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (NP > 1)
            __hip_atomic_store(&partials[NP * slot + 1], s.b, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One epoch: `iters` CG iterations of every solve, then its reliable update.
template <class Lnk>
__global__ __launch_bounds__(256) void k_serve_epoch(const SlotDesc* __restrict__ slots, int n,
                                                     int iters, int total_sweep, int total_elem,
                                                     EpochCtl* ctl, long spin_limit) {
    for (int it = 0; it < iters; ++it) {
        // A: p = gamma r + beta p, q = Q p, x_lo += alpha p_old, p.q
        for (int w = blockIdx.x; w < total_sweep; w += gridDim.x) {
            const SlotDesc& S = slots[find_slot(slots, n, w, true)];
            if (S.sc->done != kRunning) continue;
            const int tile = w - S.off_sweep;
            store_deposit<1>(serve_sweep_A<Lnk>(&S, tile), S.partials, tile);
            __syncthreads();
        }
        if (!grid_barrier(ctl, spin_limit)) return;
        for (int j = blockIdx.x; j < n; j += gridDim.x) {
            const SlotDesc& S = slots[j];
            if (S.sc->done != kRunning) continue;
            double tot[1];
            reduce_deposits<256, 1>(S.partials, S.sweep_tiles, tot);
            if (threadIdx.x == 0) slot_phaseA<Lnk>(S).finish(tot);
            __syncthreads();
        }
        if (!grid_barrier(ctl, spin_limit)) return;
        // B: r -= alpha q, r.r
        for (int w = blockIdx.x; w < total_elem; w += gridDim.x) {
            const SlotDesc& S = slots[find_slot(slots, n, w, false)];
            if (S.sc->done != kRunning) continue;
            double part[1] = {0.0};
            const int tile = w - S.off_elem;
            tile_phaseB<float>(S.r, S.q, (float)S.sc->alpha, S.g.V, tile, part);
            deposit<256, 1>(part, S.partials, tile);
            __syncthreads();
        }
        if (!grid_barrier(ctl, spin_limit)) return;
        for (int j = blockIdx.x; j < n; j += gridDim.x) {
            const SlotDesc& S = slots[j];
            if (S.sc->done != kRunning) continue;
            double tot[1];
            reduce_deposits<256, 1>(S.partials, S.elem_tiles, tot);
            if (threadIdx.x == 0) finish_phaseB(S.sc, tot[0]);
            __syncthreads();
        }
        if (!grid_barrier(ctl, spin_limit)) return;
    }
    // Reliable update: x += x_lo + alpha p (FP64), r = phi - Q x (FP64).
    for (int w = blockIdx.x; w < total_elem; w += gridDim.x) {
        const SlotDesc& S = slots[find_slot(slots, n, w, false)];
        if (!mode_runs(kModeReliable, S.sc->done)) continue;
        tile_fold<float>(S.x, S.xlo, (S.sc->iter & 1) ? S.p1 : S.p0, S.sc->alpha, S.g.V,
                         w - S.off_elem);
    }
    if (!grid_barrier(ctl, spin_limit)) return;
    for (int w = blockIdx.x; w < total_sweep; w += gridDim.x) {
        const SlotDesc& S = slots[find_slot(slots, n, w, true)];
        if (!mode_runs(kModeReliable, S.sc->done)) continue;
        const int tile = w - S.off_sweep;
        store_deposit<2>(serve_sweep_R(&S, tile), S.partials, tile);
        __syncthreads();
    }
    if (!grid_barrier(ctl, spin_limit)) return;
    for (int j = blockIdx.x; j < n; j += gridDim.x) {
        const SlotDesc& S = slots[j];
        if (!mode_runs(kModeReliable, S.sc->done)) continue;
        double tot[2];
        reduce_deposits<256, 2>(S.partials, S.sweep_tiles, tot);
        if (threadIdx.x == 0) slot_residual(S).finish(tot);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Batched engine: the same phases as k_serve_epoch, one launch per phase for
// all in-flight solves, with one-block-per-solve finalize launches in place
// of grid barriers (kernel boundaries are the cheaper device-wide sync).

// Sweep kernels of one tile shape over the in-flight solves of that shape
// (slots[0 .. n), whose off_sweep count within the group).
template <class Lnk, int KIND, int A, int B, int C>
__global__ __launch_bounds__(256) void k_serve_A(const SlotDesc* __restrict__ slots, int n) {
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    const SlotDesc& S = slots[find_slot(slots, n, w, true)];
    if (S.sc->done != kRunning) return;
    const int tile = w - S.off_sweep;
    store_deposit<1>(serve_tile_A_body<Lnk, KIND, A, B, C>(&S, tile), S.partials, tile);
}

template <class Lnk>
__global__ __launch_bounds__(256) void k_serve_finA(const SlotDesc* __restrict__ slots) {
    const SlotDesc& S = slots[blockIdx.x];
    if (S.sc->done != kRunning) return;
    double tot[1];
    reduce_deposits<256, 1>(S.partials, S.sweep_tiles, tot);
    if (threadIdx.x == 0) slot_phaseA<Lnk>(S).finish(tot);
}

__global__ __launch_bounds__(256) void k_serve_B(const SlotDesc* __restrict__ slots, int n) {
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    const SlotDesc& S = slots[find_slot(slots, n, w, false)];
    if (S.sc->done != kRunning) return;
    double part[1] = {0.0};
    const int tile = w - S.off_elem;
    tile_phaseB<float>(S.r, S.q, (float)S.sc->alpha, S.g.V, tile, part);
    deposit<256, 1>(part, S.partials, tile);
}

__global__ __launch_bounds__(256) void k_serve_finB(const SlotDesc* __restrict__ slots) {
    const SlotDesc& S = slots[blockIdx.x];
    if (S.sc->done != kRunning) return;
    double tot[1];
    reduce_deposits<256, 1>(S.partials, S.elem_tiles, tot);
    if (threadIdx.x == 0) finish_phaseB(S.sc, tot[0]);
}

__global__ __launch_bounds__(256) void k_serve_fold(const SlotDesc* __restrict__ slots, int n) {
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    const SlotDesc& S = slots[find_slot(slots, n, w, false)];
    if (!mode_runs(kModeReliable, S.sc->done)) return;
    tile_fold<float>(S.x, S.xlo, (S.sc->iter & 1) ? S.p1 : S.p0, S.sc->alpha, S.g.V,
                     w - S.off_elem);
}

template <int KIND, int A, int B, int C>
__global__ __launch_bounds__(256) void k_serve_R(const SlotDesc* __restrict__ slots, int n) {
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    const SlotDesc& S = slots[find_slot(slots, n, w, true)];
    if (!mode_runs(kModeReliable, S.sc->done)) return;
    const int tile = w - S.off_sweep;
    store_deposit<2>(serve_tile_R_body<KIND, A, B, C>(&S, tile), S.partials, tile);
}

// Launch the phase-A (R = false) or residual (R = true) sweep of one group of
// solves that share a tile shape.
template <class Lnk>
static hipError_t launch_serve_sweep(bool R, int kind, int variant, const SlotDesc* slots, int n,
                                     int tiles, size_t lds, hipStream_t st) {
#define HUB_SERVE_CASE(KIND, A, B, C)                                                    \
    do {                                                                                 \
        if (R)                                                                           \
            k_serve_R<KIND, A, B, C><<<tiles, 256, lds, st>>>(slots, n);                  \
        else                                                                             \
            k_serve_A<Lnk, KIND, A, B, C><<<tiles, 256, lds, st>>>(slots, n);             \
    } while (0)
    if (kind == kSweepD1) {
        switch (variant) {
            case kD1_256x4: HUB_SERVE_CASE(kSweepD1, 256, 4, 0); break;
            case kD1_128x4: HUB_SERVE_CASE(kSweepD1, 128, 4, 0); break;
            default: HUB_SERVE_CASE(kSweepD1, 64, 4, 0); break;
        }
    } else {
        switch (variant) {
            case kD3_8x8x8: HUB_SERVE_CASE(kSweepD3, 8, 8, 8); break;
            case kD3_16x4x4: HUB_SERVE_CASE(kSweepD3, 16, 4, 4); break;
            default: HUB_SERVE_CASE(kSweepD3, 32, 8, 4); break;
        }
    }
#undef HUB_SERVE_CASE
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_serve_finR(const SlotDesc* __restrict__ slots) {
    const SlotDesc& S = slots[blockIdx.x];
    if (!mode_runs(kModeReliable, S.sc->done)) return;
    double tot[2];
    reduce_deposits<256, 2>(S.partials, S.sweep_tiles, tot);
    if (threadIdx.x == 0) slot_residual(S).finish(tot);
}

__global__ void k_zero_ctl(EpochCtl* c) {
    if (threadIdx.x == 0) {
        c->count = 0;
        c->gen = 0;
        c->abort = 0;
        c->pad = 0;
    }
}

// One-solve kernels reused for a slot's set-up and wrap-up (cg.hip).
hub_status serve_slot_init(const Geom& g, CGScalars* sc, const double* phi, float* r, float* p0,
                           double* x, float* xlo, double tol2, double delta2, int max_iter,
                           double* partials, hipStream_t st);
hub_status serve_slot_final(const Geom& g, const SweepPlan& P, CGScalars* sc, const double* phi,
                            double* x, float* xlo, float* r, float* p0, float* p1,
                            const double* A64, double* partials, hipStream_t st);
double reliable_delta();

}  // namespace hub

using namespace hub;

namespace {

using Clock = std::chrono::steady_clock;

struct Chain {
    int id = 0;
    hub_lattice lat{};
    Geom g{};
    std::vector<double> sigma_host;  // kept for re-upload after eviction
    bool announced = false;          // a field has been submitted
    hub_lattice lat_announced{};     // lattice of the latest submitted field
    double* sigma_d = nullptr;
    double* A64 = nullptr;
    void* lnk = nullptr;
    size_t bytes = 0;
    bool resident = false;
    bool busy = false;       // a request of this chain is queued or running
    uint64_t last_use = 0;
};

struct Request {
    uint64_t ticket;
    int chain;
    hub_lattice lat;
    Geom g;
    bool new_sigma;
    std::vector<double> sigma;
    std::vector<double> phi;
    Clock::time_point t_submit;
};

struct Slot {
    bool used = false;
    Request req;
    Chain* chain = nullptr;
    SweepPlan P{};
    char* mem = nullptr;  // one allocation holding everything below
    size_t bytes = 0;
    double *phi = nullptr, *x = nullptr, *partials = nullptr;
    float *r = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr, *xlo = nullptr;
    Clock::time_point t_admit;
};

struct Result {
    std::vector<double> x;
    hub_cg_stats stats{};
    hub_status status = HUB_OK;
};

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

size_t chain_bytes(const Geom& g, hub_dtype link) {
    const size_t V = (size_t)g.V;
    return al256(8 * V) * 2 + al256(dtype_size(link) * V);
}

size_t slot_bytes(const Geom& g) {
    const size_t V = (size_t)g.V;
    const SweepPlan P = plan_sweep(g, false);
    const int e = elem_tiles(g.V);
    const size_t parts = sizeof(double) * kMaxNP * (size_t)std::max(P.ntiles, e);
    return al256(8 * V) * 2 + al256(4 * V) * 5 + al256(parts);
}

}  // namespace

struct hub_server {
    hub_serve_opts opts{};
    int device = 0;
    hipStream_t stream = nullptr;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::deque<Request> queue;
    std::unordered_set<uint64_t> pending;
    std::unordered_map<uint64_t, Result> results;
    std::map<int, Chain> chains;
    uint64_t next_ticket = 1;
    uint64_t use_clock = 0;
    size_t resident = 0;  // device bytes of resident chains and slots
    hub_status fatal = HUB_OK;
    char fatal_msg[512] = {0};
    // device tables
    std::vector<Slot> slots;
    SlotDesc* desc_d = nullptr;
    SlotDesc* desc_h = nullptr;  // pinned
    CGScalars* sc_d = nullptr;   // one per slot
    CGScalars* sc_h = nullptr;   // pinned mirror
    EpochCtl* ctl_d = nullptr;
    EpochCtl* ctl_h = nullptr;   // pinned
    int coop_grid = 0;
};

namespace {

#define SRV_TRY(expr)                \
    do {                             \
        hub_status s_ = (expr);      \
        if (s_ != HUB_OK) return s_; \
    } while (0)

hub_status free_chain(hub_server* S, Chain& c) {
    if (!c.resident) return HUB_OK;
    HUB_HIP(hipFreeAsync(c.sigma_d, S->stream));
    HUB_HIP(hipFreeAsync(c.A64, S->stream));
    HUB_HIP(hipFreeAsync(c.lnk, S->stream));
    c.sigma_d = c.A64 = nullptr;
    c.lnk = nullptr;
    c.resident = false;
    S->resident -= c.bytes;
    return HUB_OK;
}

// Make room for `need` bytes by evicting idle chains other than `keep`,
// least recently used first.  Returns whether it fits.
bool make_room(hub_server* S, size_t need, int keep) {
    while (S->resident + need > S->opts.hbm_budget_bytes) {
        Chain* victim = nullptr;
        for (auto& kv : S->chains) {
            Chain& c = kv.second;
            if (!c.resident || c.busy || c.id == keep) continue;
            if (!victim || c.last_use < victim->last_use) victim = &c;
        }
        if (!victim) return false;
        if (free_chain(S, *victim) != HUB_OK) return false;
    }
    return true;
}

hub_status upload_chain(hub_server* S, Chain& c, const Request& R) {
    const hub_dtype link = S->opts.cg.link;
    if (c.resident && (c.g.V != R.g.V || std::memcmp(&c.lat, &R.lat, sizeof(hub_lattice)) != 0))
        SRV_TRY(free_chain(S, c));
    c.lat = R.lat;
    c.g = R.g;
    if (R.new_sigma) c.sigma_host = R.sigma;
    const size_t V = (size_t)c.g.V;
    if (!c.resident) {
        c.bytes = chain_bytes(c.g, link);
        HUB_HIP(hipMallocAsync((void**)&c.sigma_d, 8 * V, S->stream));
        HUB_HIP(hipMallocAsync((void**)&c.A64, 8 * V, S->stream));
        HUB_HIP(hipMallocAsync(&c.lnk, dtype_size(link) * V, S->stream));
        c.resident = true;
        S->resident += c.bytes;
    } else if (!R.new_sigma) {
        return HUB_OK;  // field and links already on the device
    }
    HUB_HIP(hipMemcpyAsync(c.sigma_d, c.sigma_host.data(), 8 * V, hipMemcpyHostToDevice,
                           S->stream));
    SRV_TRY(launch_links(c.g, c.sigma_d, c.A64, HUB_F64, S->stream));
    SRV_TRY(launch_links(c.g, c.sigma_d, c.lnk, link, S->stream));
    return HUB_OK;
}

hub_status start_slot(hub_server* S, int k, Request&& R) {
    Slot& sl = S->slots[k];
    sl = Slot{};
    sl.used = true;
    sl.req = std::move(R);
    sl.t_admit = Clock::now();
    Chain& c = S->chains[sl.req.chain];
    c.id = sl.req.chain;
    sl.chain = &c;
    SRV_TRY(upload_chain(S, c, sl.req));
    const Geom& g = sl.req.g;
    const size_t V = (size_t)g.V;
    sl.P = plan_sweep(g, false);
    sl.bytes = slot_bytes(g);
    HUB_HIP(hipMallocAsync((void**)&sl.mem, sl.bytes, S->stream));
    S->resident += sl.bytes;
    size_t off = 0;
    auto take = [&](size_t b) { char* p = sl.mem + off; off += al256(b); return p; };
    sl.phi = (double*)take(8 * V);
    sl.x = (double*)take(8 * V);
    sl.r = (float*)take(4 * V);
    sl.p0 = (float*)take(4 * V);
    sl.p1 = (float*)take(4 * V);
    sl.q = (float*)take(4 * V);
    sl.xlo = (float*)take(4 * V);
    sl.partials = (double*)take(sizeof(double) * kMaxNP *
                                (size_t)std::max(sl.P.ntiles, elem_tiles(g.V)));
    HUB_HIP(hipMemcpyAsync(sl.phi, sl.req.phi.data(), 8 * V, hipMemcpyHostToDevice, S->stream));
    const hub_cg_opts& o = S->opts.cg;
    SRV_TRY(serve_slot_init(g, &S->sc_d[k], sl.phi, sl.r, sl.p0, sl.x, sl.xlo, o.tol * o.tol,
                            reliable_delta() * reliable_delta(), o.max_iter, sl.partials,
                            S->stream));
    return HUB_OK;
}

void record_fatal(hub_server* S, hub_status st) {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fatal == HUB_OK) {
        S->fatal = st;
        std::snprintf(S->fatal_msg, sizeof(S->fatal_msg), "%s", hub_last_error());
    }
}

// Admit queued requests that fit (arrival order; a chain's next request
// waits for its running one).  Runs on the worker with the lock held, so
// that chain bookkeeping never races hub_serve_submit.
hub_status admit(hub_server* S) {
    std::lock_guard<std::mutex> lk(S->mu);
    std::unordered_set<int> running;
    for (auto& sl : S->slots)
        if (sl.used) running.insert(sl.req.chain);
    for (auto it = S->queue.begin(); it != S->queue.end();) {
        if (running.count(it->chain)) { ++it; continue; }
        int free_k = -1;
        for (int k = 0; k < (int)S->slots.size(); ++k)
            if (!S->slots[k].used) { free_k = k; break; }
        if (free_k < 0) break;
        Chain& c = S->chains[it->chain];
        const bool same = c.resident && c.g.V == it->g.V &&
                          std::memcmp(&c.lat, &it->lat, sizeof(hub_lattice)) == 0;
        // A resident chain on another lattice is released on re-upload.
        const size_t freed = (c.resident && !same) ? c.bytes : 0;
        const size_t need = slot_bytes(it->g) + (same ? 0 : chain_bytes(it->g, S->opts.cg.link));
        if (S->resident - freed + need > S->opts.hbm_budget_bytes &&
            !make_room(S, need > freed ? need - freed : 0, c.id))
            break;
        c.last_use = ++S->use_clock;
        running.insert(it->chain);
        Request R = std::move(*it);
        it = S->queue.erase(it);
        SRV_TRY(start_slot(S, free_k, std::move(R)));
    }
    return HUB_OK;
}

hub_status finish_slot(hub_server* S, int k) {
    Slot& sl = S->slots[k];
    const Geom& g = sl.req.g;
    if (S->sc_h[k].done != kDoneConverged) {
        SRV_TRY(serve_slot_final(g, sl.P, &S->sc_d[k], sl.phi, sl.x, sl.xlo, sl.r, sl.p0, sl.p1,
                                 sl.chain->A64, sl.partials, S->stream));
        HUB_HIP(hipMemcpyAsync(&S->sc_h[k], &S->sc_d[k], sizeof(CGScalars),
                               hipMemcpyDeviceToHost, S->stream));
    }
    Result res;
    res.x.resize((size_t)g.V);
    HUB_HIP(hipMemcpyAsync(res.x.data(), sl.x, 8 * (size_t)g.V, hipMemcpyDeviceToHost,
                           S->stream));
    HUB_HIP(hipStreamSynchronize(S->stream));
    const CGScalars& s = S->sc_h[k];
    res.stats.iters = s.iter;
    res.stats.reliable_updates = s.reliable_updates;
    res.stats.true_rel_resid = s.phi2 > 0 ? std::sqrt(s.rho_true / s.phi2) : 0.0;
    res.stats.ms = std::chrono::duration<double, std::milli>(Clock::now() - sl.t_admit).count();
    res.status = s.done == kDoneConverged ? HUB_OK : HUB_E_NOCONV;
    res.stats.status = res.status;
    HUB_HIP(hipFreeAsync(sl.mem, S->stream));
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->resident -= sl.bytes;
        sl.chain->busy = false;
        for (auto& q : S->queue)
            if (q.chain == sl.req.chain) sl.chain->busy = true;
        S->pending.erase(sl.req.ticket);
        S->results.emplace(sl.req.ticket, std::move(res));
        sl.used = false;
    }
    return HUB_OK;
}

hub_status run_epoch(hub_server* S) {
    // In-flight solves, grouped by tile shape so that each sweep launch runs
    // one shape: off_sweep counts within the group, off_elem over all.
    std::vector<int> ks;
    for (int k = 0; k < (int)S->slots.size(); ++k)
        if (S->slots[k].used) ks.push_back(k);
    const int n = (int)ks.size();
    if (n == 0) return HUB_OK;
    auto shape_key = [&](int k) { return S->slots[k].P.kind * 64 + S->slots[k].P.variant; };
    std::stable_sort(ks.begin(), ks.end(),
                     [&](int a, int b) { return shape_key(a) < shape_key(b); });
    struct Group { int first, count, tiles, kind, variant; };
    std::vector<Group> groups;
    int tot_sweep = 0, tot_elem = 0;
    for (int j = 0; j < n; ++j) {
        Slot& sl = S->slots[ks[j]];
        if (groups.empty() || shape_key(ks[groups.back().first]) != shape_key(ks[j]))
            groups.push_back({j, 0, 0, sl.P.kind, sl.P.variant});
        Group& gr = groups.back();
        SlotDesc& d = S->desc_h[j];
        d = SlotDesc{};
        d.g = sl.req.g;
        d.kind = sl.P.kind;
        d.variant = sl.P.variant;
        d.tiles_x = sl.P.tiles_x;
        d.tiles_y = sl.P.tiles_y;
        d.tiles_z = sl.P.tiles_z;
        d.tc = sl.P.tc;
        d.sweep_tiles = sl.P.ntiles;
        d.elem_tiles = elem_tiles(d.g.V);
        d.off_sweep = gr.tiles;
        d.off_elem = tot_elem;
        d.sc = &S->sc_d[ks[j]];
        d.partials = sl.partials;
        d.phi = sl.phi;
        d.x = sl.x;
        d.A64 = sl.chain->A64;
        d.lnk = sl.chain->lnk;
        d.r = sl.r;
        d.p0 = sl.p0;
        d.p1 = sl.p1;
        d.q = sl.q;
        d.xlo = sl.xlo;
        gr.count += 1;
        gr.tiles += d.sweep_tiles;
        tot_elem += d.elem_tiles;
    }
    HUB_HIP(hipMemcpyAsync(S->desc_d, S->desc_h, sizeof(SlotDesc) * n, hipMemcpyHostToDevice,
                           S->stream));
    int iters = S->opts.cg.reliable_every;
    const SlotDesc* descp = S->desc_d;
    const bool f16 = S->opts.cg.link == HUB_F16;
    if (S->opts.engine == 1) {
        // The persistent kernel runs every phase over all solves: offsets of
        // the sweep phases over all groups.
        for (int j = 0; j < n; ++j) {
            S->desc_h[j].off_sweep = tot_sweep;
            tot_sweep += S->desc_h[j].sweep_tiles;
        }
        HUB_HIP(hipMemcpyAsync(S->desc_d, S->desc_h, sizeof(SlotDesc) * n,
                               hipMemcpyHostToDevice, S->stream));
        k_zero_ctl<<<1, 64, 0, S->stream>>>(S->ctl_d);
        EpochCtl* ctl = S->ctl_d;
        // ~1 s of polling per barrier before giving up (a healthy barrier
        // takes tens of microseconds).
        long spin_limit = 1L << 22;
        int nn = n;
        void* args[] = {(void*)&descp, (void*)&nn, (void*)&iters, (void*)&tot_sweep,
                        (void*)&tot_elem, (void*)&ctl, (void*)&spin_limit};
        const void* fn = f16 ? (const void*)k_serve_epoch<Link16>
                             : (const void*)k_serve_epoch<Link32>;
        HUB_HIP(hipLaunchCooperativeKernel(fn, dim3(S->coop_grid), dim3(256), args,
                                           kServeLdsBytes, S->stream));
    } else {
        const hipStream_t st = S->stream;
        auto sweeps = [&](bool R) -> hipError_t {
            for (const Group& gr : groups) {
                const size_t lds = (R ? 8 : 4) * (size_t)serve_lds_elems(gr.kind, gr.variant);
                const hipError_t e =
                    f16 ? launch_serve_sweep<Link16>(R, gr.kind, gr.variant, descp + gr.first,
                                                     gr.count, gr.tiles, lds, st)
                        : launch_serve_sweep<Link32>(R, gr.kind, gr.variant, descp + gr.first,
                                                     gr.count, gr.tiles, lds, st);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        };
        for (int it = 0; it < iters; ++it) {
            HUB_HIP(sweeps(false));
            if (f16)
                k_serve_finA<Link16><<<n, 256, 0, st>>>(descp);
            else
                k_serve_finA<Link32><<<n, 256, 0, st>>>(descp);
            k_serve_B<<<tot_elem, 256, 0, st>>>(descp, n);
            k_serve_finB<<<n, 256, 0, st>>>(descp);
        }
        k_serve_fold<<<tot_elem, 256, 0, st>>>(descp, n);
        HUB_HIP(sweeps(true));
        k_serve_finR<<<n, 256, 0, st>>>(descp);
        HUB_HIP(hipGetLastError());
    }
    HUB_HIP(hipMemcpyAsync(S->sc_h, S->sc_d, sizeof(CGScalars) * S->slots.size(),
                           hipMemcpyDeviceToHost, S->stream));
    HUB_HIP(hipMemcpyAsync(S->ctl_h, S->ctl_d, sizeof(EpochCtl), hipMemcpyDeviceToHost,
                           S->stream));
    HUB_HIP(hipStreamSynchronize(S->stream));
    if (S->opts.engine == 1 && S->ctl_h->abort)
        return set_error(HUB_E_DEVICE, "serving kernel: a grid barrier timed out");
    for (int k : ks)
        if (S->sc_h[k].done >= kDoneConverged) SRV_TRY(finish_slot(S, k));
    return HUB_OK;
}

void worker_main(hub_server* S) {
    if (hipSetDevice(S->device) != hipSuccess) {
        set_error(HUB_E_DEVICE, "serve worker: hipSetDevice failed");
        record_fatal(S, HUB_E_DEVICE);
        return;
    }
    for (;;) {
        hub_status st = admit(S);
        if (st != HUB_OK) { record_fatal(S, st); break; }
        bool any = false;
        for (auto& sl : S->slots) any = any || sl.used;
        if (!any) {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop) break;
            if (S->queue.empty())
                S->cv.wait_for(lk, std::chrono::milliseconds(20));
            continue;
        }
        st = run_epoch(S);
        if (st != HUB_OK) { record_fatal(S, st); break; }
    }
    // Fail whatever is left.
    std::lock_guard<std::mutex> lk(S->mu);
    for (auto& sl : S->slots)
        if (sl.used) {
            Result r;
            r.status = S->fatal != HUB_OK ? S->fatal : HUB_E_DEVICE;
            r.stats.status = r.status;
            S->pending.erase(sl.req.ticket);
            S->results.emplace(sl.req.ticket, std::move(r));
            sl.used = false;
        }
}

hub_status serve_validate_opts(const hub_serve_opts* o) {
    if (!o) return set_error(HUB_E_INVALID, "serve opts is NULL");
    if (o->max_inflight < 1 || o->max_inflight > 4096)
        return set_error(HUB_E_INVALID, "max_inflight = %d, expected 1..4096", o->max_inflight);
    if (o->engine != 0 && o->engine != 1)
        return set_error(HUB_E_INVALID, "engine = %d, expected 0 (batched) or 1 (persistent)",
                         o->engine);
    if (o->cg.bulk != HUB_F32)
        return set_error(HUB_E_INVALID, "serving runs the mixed-precision solver: cg.bulk must be F32");
    if (o->cg.link != HUB_F32 && o->cg.link != HUB_F16)
        return set_error(HUB_E_INVALID, "cg.link must be F32 or F16");
    if (!(o->cg.tol > 0) || !(o->cg.tol < 1))
        return set_error(HUB_E_INVALID, "tol = %g, expected 0 < tol < 1", o->cg.tol);
    if (o->cg.max_iter < 1) return set_error(HUB_E_INVALID, "max_iter must be >= 1");
    if (o->cg.reliable_every < 1) return set_error(HUB_E_INVALID, "reliable_every must be >= 1");
    if (o->hbm_budget_bytes == 0) return set_error(HUB_E_INVALID, "hbm_budget_bytes is 0");
    return HUB_OK;
}

hub_status server_create(const hub_serve_opts* o, hub_server** out) {
    SRV_TRY(serve_validate_opts(o));
    hub_server* S = new hub_server();
    S->opts = *o;
    auto fail = [&](hub_status st) {
        if (S->stream) (void)hipStreamDestroy(S->stream);
        if (S->desc_d) (void)hipFree(S->desc_d);
        if (S->sc_d) (void)hipFree(S->sc_d);
        if (S->ctl_d) (void)hipFree(S->ctl_d);
        if (S->desc_h) (void)hipHostFree(S->desc_h);
        if (S->sc_h) (void)hipHostFree(S->sc_h);
        if (S->ctl_h) (void)hipHostFree(S->ctl_h);
        delete S;
        return st;
    };
#define SRV_HIP(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(set_error(HUB_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_))); \
    } while (0)
    SRV_HIP(hipGetDevice(&S->device));
    if (o->engine == 1) {
        int coop = 0, ncu = 0;
        SRV_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, S->device));
        if (!coop)
            return fail(set_error(HUB_E_DEVICE, "device does not support cooperative launch"));
        SRV_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, S->device));
        int per_cu = 0;
        const void* fn = o->cg.link == HUB_F16 ? (const void*)k_serve_epoch<Link16>
                                               : (const void*)k_serve_epoch<Link32>;
        SRV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, kServeLdsBytes));
        if (per_cu < 1) return fail(set_error(HUB_E_DEVICE, "serving kernel does not fit a CU"));
        S->coop_grid = per_cu * ncu;
    }
    SRV_HIP(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
    const int m = o->max_inflight;
    S->slots.resize(m);
    SRV_HIP(hipMalloc((void**)&S->desc_d, sizeof(SlotDesc) * m));
    SRV_HIP(hipMalloc((void**)&S->sc_d, sizeof(CGScalars) * m));
    SRV_HIP(hipMalloc((void**)&S->ctl_d, sizeof(EpochCtl)));
    SRV_HIP(hipHostMalloc((void**)&S->desc_h, sizeof(SlotDesc) * m, hipHostMallocDefault));
    SRV_HIP(hipHostMalloc((void**)&S->sc_h, sizeof(CGScalars) * m, hipHostMallocDefault));
    SRV_HIP(hipHostMalloc((void**)&S->ctl_h, sizeof(EpochCtl), hipHostMallocDefault));
#undef SRV_HIP
    S->worker = std::thread(worker_main, S);
    *out = S;
    return HUB_OK;
}

}  // namespace

extern "C" {

hub_status hub_serve_create(const hub_serve_opts* opts, hub_server** out) {
    try {
        clear_error();
        if (!out) return set_error(HUB_E_INVALID, "out is NULL");
        *out = nullptr;
        return server_create(opts, out);
    } catch (const std::bad_alloc&) {
        return set_error(HUB_E_NOMEM, "host allocation failed");
    } catch (...) {
        return set_error(HUB_E_INVALID, "internal error (unexpected exception)");
    }
}

hub_status hub_serve_submit(hub_server* srv, int32_t chain_id, const hub_lattice* lat,
                            const double* sigma_host, const double* phi_host, uint64_t* ticket) {
    try {
        clear_error();
        if (!srv) return set_error(HUB_E_INVALID, "server is NULL");
        if (!ticket) return set_error(HUB_E_INVALID, "ticket is NULL");
        if (!phi_host) return set_error(HUB_E_INVALID, "phi_host is NULL");
        Geom g;
        SRV_TRY(make_geom(lat, &g));
        const SweepPlan P = plan_sweep(g, false);
        if (!serve_supported(P))
            return set_error(HUB_E_INVALID,
                             "serving steps d=1 lattices and d=3 lattices with nx in {8, 16, "
                             "32}; use hub_cg_solve for this one");
        const size_t need = slot_bytes(g) + chain_bytes(g, srv->opts.cg.link);
        if (need > srv->opts.hbm_budget_bytes)
            return set_error(HUB_E_NOMEM, "request needs %zu bytes, budget is %zu", need,
                             srv->opts.hbm_budget_bytes);
        Request R;
        R.chain = chain_id;
        R.lat = *lat;
        R.g = g;
        R.new_sigma = sigma_host != nullptr;
        R.t_submit = Clock::now();
        const size_t V = (size_t)g.V;
        R.phi.assign(phi_host, phi_host + V);
        if (sigma_host) R.sigma.assign(sigma_host, sigma_host + V);
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->fatal != HUB_OK)
            return set_error(srv->fatal, "server stopped: %s", srv->fatal_msg);
        if (srv->stop) return set_error(HUB_E_INVALID, "server is shutting down");
        Chain& c = srv->chains[chain_id];
        c.id = chain_id;
        if (!sigma_host) {
            if (!c.announced)
                return set_error(HUB_E_INVALID, "chain %d has no field yet: pass sigma_host",
                                 chain_id);
            if (std::memcmp(&c.lat_announced, lat, sizeof(hub_lattice)) != 0)
                return set_error(HUB_E_INVALID,
                                 "chain %d changes lattice: pass its new sigma_host", chain_id);
        } else {
            c.announced = true;
            c.lat_announced = *lat;
        }
        R.ticket = srv->next_ticket++;
        *ticket = R.ticket;
        c.busy = true;
        srv->pending.insert(R.ticket);
        srv->queue.push_back(std::move(R));
        srv->cv.notify_one();
        return HUB_OK;
    } catch (const std::bad_alloc&) {
        return set_error(HUB_E_NOMEM, "host allocation failed");
    } catch (...) {
        return set_error(HUB_E_INVALID, "internal error (unexpected exception)");
    }
}

hub_status hub_serve_poll(hub_server* srv, uint64_t ticket, double* x_host, hub_cg_stats* out) {
    try {
        clear_error();
        if (!srv) return set_error(HUB_E_INVALID, "server is NULL");
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->results.find(ticket);
        if (it == srv->results.end()) {
            if (srv->pending.count(ticket)) return HUB_PENDING;
            return set_error(HUB_E_NOTFOUND, "ticket %llu is unknown or already retired",
                             (unsigned long long)ticket);
        }
        Result r = std::move(it->second);
        srv->results.erase(it);
        if (x_host && !r.x.empty()) std::memcpy(x_host, r.x.data(), 8 * r.x.size());
        if (out) *out = r.stats;
        if (r.status == HUB_E_NOCONV) set_error(HUB_E_NOCONV, "solve did not converge");
        else if (r.status != HUB_OK) set_error(r.status, "solve failed: %s", srv->fatal_msg);
        return r.status;
    } catch (...) {
        return set_error(HUB_E_INVALID, "internal error (unexpected exception)");
    }
}

hub_status hub_serve_destroy(hub_server* srv) {
    if (!srv) return HUB_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        // requests not yet admitted are dropped
        for (auto& q : srv->queue) srv->pending.erase(q.ticket);
        srv->queue.clear();
    }
    srv->cv.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    (void)hipSetDevice(srv->device);
    for (auto& kv : srv->chains) (void)free_chain(srv, kv.second);
    (void)hipStreamSynchronize(srv->stream);
    (void)hipStreamDestroy(srv->stream);
    (void)hipFree(srv->desc_d);
    (void)hipFree(srv->sc_d);
    (void)hipFree(srv->ctl_d);
    (void)hipHostFree(srv->desc_h);
    (void)hipHostFree(srv->sc_h);
    (void)hipHostFree(srv->ctl_h);
    delete srv;
    return HUB_OK;
}

}  // extern "C"
