// Shared device/host definitions of libhub (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "hub.h"

namespace hub {

// n / d for 0 <= n < 2^31 and 1 <= d < 2^31 by one multiply and a shift
// (rounded-up multiplier, after Granlund and Montgomery 1994): with
// s = ceil(log2 d) and m = ceil(2^(32+s) / d), m d = 2^(32+s) + e with
// 0 <= e < d, so n m / 2^(32+s) exceeds n / d by less than n / 2^(32+s) <
// 1 / (2d), which never reaches the next integer.  The one-lane-per-site
// kernels need two to four divisions per site for its coordinates; as
// integer divisions those cost more than the kernels' memory traffic.
struct FastDiv {
    uint64_t m;  // <= 2^33
    int sh;      // 32 + s
};

inline FastDiv make_fastdiv(uint32_t d) {
    int s = 0;
    while ((1ull << s) < d) ++s;
    return {((1ull << (32 + s)) + d - 1) / d, 32 + s};
}

__host__ __device__ __forceinline__ int fdiv(int n, const FastDiv& f) {
    return (int)(((uint64_t)(uint32_t)n * f.m) >> f.sh);
}

// Lattice geometry and operator constants, passed to kernels by value.
struct Geom {
    int d;          // spatial dimensions
    int nx;         // spatial extent
    int nt;         // time slices
    int vs;         // nx^d
    int V;          // vs * nt
    double kappa;   // dtau * t_hop
    double lscale;  // exp(dtau * mu)
    double b;       // Hubbard-Stratonovich coupling sqrt(2 (exp(-dtau U) - 1))
    FastDiv fnx;    // division by nx
    FastDiv fvs;    // division by vs
};

// Device-resident solver state of one CG solve.  Every field is written by
// exactly one thread: thread 0 of a one-block finalize kernel, or an
// initialisation kernel.
struct CGScalars {
    double rho;        // current iterated r.r (FP64 accumulation)
    double rho_prev;   // r.r of the previous iteration
    double alpha;      // step length still to be added to x (0 once folded)
    double beta;       // p_new = gamma r + beta p_old
    double gamma;      // 1 except right after a reliable update
    double phi2;       // |phi|^2
    double tol2phi2;   // tol^2 |phi|^2
    double rho_true;   // |phi - Q x|^2 of the last true-residual recompute
    double rho_ru;     // r.r right after the last reliable update
    double delta2;     // reliable update once rho < delta2 * rho_ru (0: never)
    double pq;         // last p.Qp
    double rr;         // preconditioned CG: iterated r.r (rho holds r.z)
    int32_t iter;      // iterations completed
    int32_t max_iter;
    int32_t done;      // see kDone* below
    int32_t reliable_updates;
    int32_t restart;   // preconditioned CG: next beta is 0 (fresh residual)
    int32_t pad[3];
};

enum : int32_t {
    kRunning = 0,
    kDoneIterConverged = 1,  // iterated residual met tol, or dropped by
                             // delta since the last reliable update: recompute
    kDoneConverged = 2,      // true residual met tol
    kDoneBreakdown = 3,      // p.Qp <= 0 or a non-finite scalar
    kDoneMaxIter = 4,
};

// When the fold / true-residual kernels run.
enum : int32_t {
    kModeReliable = 0,  // periodic reliable update: run while done <= 1
    kModeCheck = 1,     // verify an iterated convergence: run iff done == 1
    kModeFinal = 2,     // end of solve: always run
};

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)
// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X, each
// with its own L2.  Map hardware block ids so that every XCD receives a
// contiguous range of logical tiles: neighbouring tiles (which share halo
// sites) then hit in the same L2.
__device__ inline int xcd_remap(int bid, int nblocks) {
    constexpr int kXcd = 8;
    const int q = nblocks / kXcd, r = nblocks % kXcd;
    const int x = bid % kXcd, k = bid / kXcd;
    return x * q + (x < r ? x : r) + k;
}

// Wrap an index that is at most one period out of [0, n).
__device__ inline int wrap1(int v, int n) {
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

// Sum over a 64-wide wavefront, result valid in every lane.
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum (fixed tree); result valid in thread 0.
template <int BLOCK>
__device__ inline double block_sum(double v) {
    static_assert(BLOCK % 64 == 0 && BLOCK <= 1024, "block must be whole waves");
    __shared__ double red[BLOCK / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();  // red[] may still be read by a previous call
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) s += red[w];
    }
    return s;
}

// Sum of n deposits of NP values (deposit b at partials[NP*b + k]) in a
// fixed order: thread t adds deposits t, t+BLOCK, ... (four at a time, the
// loads issued together), then the block tree.  Every caller that sums the
// same deposits gets the same bits.  Result in thread 0.  Callers read the
// deposits after a kernel boundary or a grid barrier, so plain loads see
// them.
template <int BLOCK, int NP>
__device__ inline void reduce_deposits(const double* partials, int n, double (&total)[NP]) {
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        double s = 0.0;
        int b = threadIdx.x;
        for (; b + 3 * BLOCK < n; b += 4 * BLOCK) {
            const double v0 = partials[NP * b + k];
            const double v1 = partials[NP * (b + BLOCK) + k];
            const double v2 = partials[NP * (b + 2 * BLOCK) + k];
            const double v3 = partials[NP * (b + 3 * BLOCK) + k];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; b < n; b += BLOCK) s += partials[NP * b + k];
        total[k] = block_sum<BLOCK>(s);
    }
}

// The sum of n single-value deposits in exactly the order of
// reduce_deposits<256, 1> (so with the same bits), computed by a block of
// any multiple of 64 lanes: its waves take the four 64-lane groups of a
// 256-lane block in turn.  Result in every thread.  Lets a kernel of any
// block size reduce the previous kernel's deposits itself and get what a
// one-block finalize would.
__device__ inline double reduce_deposits_canon(const double* partials, int n) {
    constexpr int B = 256;
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (int)(blockDim.x >> 6);
    __syncthreads();  // red[] may still be read by a previous call
    for (int vw = wid; vw < 4; vw += nw) {
        double s = 0.0;
        int b = vw * 64 + lane;
        for (; b + 3 * B < n; b += 4 * B) {
            const double v0 = partials[b];
            const double v1 = partials[b + B];
            const double v2 = partials[b + 2 * B];
            const double v3 = partials[b + 3 * B];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; b < n; b += B) s += partials[b];
        s = wave_sum(s);
        if (lane == 0) red[vw] = s;
    }
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) tot += red[w];
    return tot;
}

// Largest number of sums any reduction deposits per tile.
constexpr int kMaxNP = 2;

// Block sums of one tile into deposit slot `slot`.  Grid reductions are two
// kernels: every tile deposits its sums, then a one-block kernel adds the
// deposits in tile order (reduce_deposits) and updates the solver scalars.
// The kernel boundary in between is the device-wide synchronisation; on
// MI355X it costs about a launch, far less than per-block release fences
// and same-address atomics inside one kernel.
template <int BLOCK, int NP>
__device__ inline void deposit(const double (&part)[NP], double* partials, int slot) {
    double bs[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) bs[k] = block_sum<BLOCK>(part[k]);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NP; ++k)
            __hip_atomic_store(&partials[NP * slot + k], bs[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

#endif

}  // namespace hub
