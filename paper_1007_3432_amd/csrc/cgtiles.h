// Element-wise tiles of the conjugate-gradient iteration (Sec. 4.1) and the
// scalar updates that follow each grid reduction.  Shared by the one-solve
// kernels (cg.hip) and the persistent multi-solve serving kernel (serve.hip),
// so that a solve takes the same steps, with the same rounding, in both.
#pragma once

#include "common.h"

namespace hub {

// Sites per element-wise tile: 256 lanes x 8 sites.  Lane t handles the
// site pairs tile*kETile + 512 j + 2t, +1 (j = 0..3): each access of a
// wavefront is one contiguous run (1 KiB for FP64, 512 B for FP32).
constexpr int kETile = 2048;

// Offset of a lane's element k (0..7) from its first site; increasing in k,
// so the elements inside [0, V) are always a prefix.
__host__ __device__ constexpr int eoff(int k) { return 512 * (k >> 1) + (k & 1); }

__host__ __device__ inline int elem_tiles(int V) { return (V + kETile - 1) / kETile; }

// A lane's eight elements from its first site p (pairs aligned to 8 bytes
// per element).
template <class T>
__device__ __forceinline__ void ld8(const T* __restrict__ p, T (&v)[8]) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double2 w = *reinterpret_cast<const double2*>(p + eoff(2 * j));
            v[2 * j] = w.x;
            v[2 * j + 1] = w.y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float2 w = *reinterpret_cast<const float2*>(p + eoff(2 * j));
            v[2 * j] = w.x;
            v[2 * j + 1] = w.y;
        }
    }
}

template <class T>
__device__ __forceinline__ void st8(T* __restrict__ p, const T (&v)[8]) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            *reinterpret_cast<double2*>(p + eoff(2 * j)) = make_double2(v[2 * j], v[2 * j + 1]);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            *reinterpret_cast<float2*>(p + eoff(2 * j)) = make_float2(v[2 * j], v[2 * j + 1]);
    }
}

// Lane's first site and how many of its 8 sites are inside [0, V).
__device__ __forceinline__ int lane_base(int tile) { return tile * kETile + 2 * threadIdx.x; }
// How many of the lane's elements lie inside [0, V) (a prefix).
__device__ __forceinline__ int lane_count(int base, int V) {
    int c = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) c += base + eoff(k) < V ? 1 : 0;
    return c;
}

// r = phi, p0 = 0, x = 0 (x_lo = 0); part[0] += phi.phi.
template <class RVec>
__device__ __forceinline__ void tile_init(const double* __restrict__ phi, RVec* __restrict__ r,
                                          RVec* __restrict__ p0, double* __restrict__ x,
                                          float* __restrict__ xlo, int V, int tile,
                                          double (&part)[1]) {
    const int base = lane_base(tile), cnt = lane_count(base, V);
    double f[8];
    if (cnt == 8) {
        ld8(phi + base, f);
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) f[k] = k < cnt ? phi[base + eoff(k)] : 0.0;
    }
    RVec rv[8], zr[8];
    double zd[8];
    float zf[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        rv[k] = (RVec)f[k];
        zr[k] = (RVec)0;
        zd[k] = 0.0;
        zf[k] = 0.0f;
        part[0] += f[k] * f[k];
    }
    if (cnt == 8) {
        st8(r + base, rv);
        st8(p0 + base, zr);
        st8(x + base, zd);
        if (xlo) st8(xlo + base, zf);
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k < cnt) {
                r[base + eoff(k)] = rv[k];
                p0[base + eoff(k)] = (RVec)0;
                x[base + eoff(k)] = 0.0;
                if (xlo) xlo[base + eoff(k)] = 0.0f;
            }
    }
}

__device__ __forceinline__ void finish_init(CGScalars* sc, double total, double tol2,
                                            double delta2, int max_iter) {
    sc->phi2 = total;
    sc->rho = total;
    sc->rho_prev = total;
    sc->rho_true = total;
    sc->rho_ru = total;
    sc->delta2 = delta2;
    sc->alpha = 0.0;
    sc->beta = 0.0;
    sc->gamma = 1.0;
    sc->tol2phi2 = tol2 * total;
    sc->iter = 0;
    sc->max_iter = max_iter;
    sc->reliable_updates = 0;
    sc->rr = total;
    sc->restart = 1;
    sc->done = !isfinite(total) ? kDoneBreakdown : (total == 0.0 ? kDoneConverged : kRunning);
}

// r -= alpha q; part[0] += r.r (FP64 accumulation of the stored r).
template <class Vec>
__device__ __forceinline__ void tile_phaseB(Vec* __restrict__ r, const Vec* __restrict__ q,
                                            Vec alpha, int V, int tile, double (&part)[1]) {
    const int base = lane_base(tile), cnt = lane_count(base, V);
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
}

// After r.r: rho, beta, iteration count; ask for a true-residual recompute
// when rho meets tol or has dropped by delta^2 since the last one.
__device__ __forceinline__ void finish_phaseB(CGScalars* sc, double total) {
    if (!isfinite(total)) {
        sc->done = kDoneBreakdown;
        return;
    }
    sc->rho_prev = sc->rho;
    sc->rho = total;
    sc->beta = total / sc->rho_prev;
    sc->iter += 1;
    if (total <= sc->tol2phi2 || total < sc->delta2 * sc->rho_ru)
        sc->done = kDoneIterConverged;
    else if (sc->iter >= sc->max_iter)
        sc->done = kDoneMaxIter;
}

// Preconditioned CG after r.r: iteration count and convergence on |r|^2
// (rho, beta belong to r.z and are set after the preconditioner).
__device__ __forceinline__ void finish_pcg_phaseB(CGScalars* sc, double total) {
    if (!isfinite(total)) {
        sc->done = kDoneBreakdown;
        return;
    }
    sc->rr = total;
    sc->iter += 1;
    if (total <= sc->tol2phi2)
        sc->done = kDoneIterConverged;
    else if (sc->iter >= sc->max_iter)
        sc->done = kDoneMaxIter;
}

// x += alpha p (+ x_lo, then x_lo = 0): the pending update, in FP64.
template <class PVec>
__device__ __forceinline__ void tile_fold(double* __restrict__ x, float* __restrict__ xlo,
                                          const PVec* __restrict__ p, double alpha, int V,
                                          int tile) {
    const int base = lane_base(tile), cnt = lane_count(base, V);
    double xv[8];
    PVec pv[8];
    float lv[8];
    if (cnt == 8) {
        ld8(x + base, xv);
        ld8(p + base, pv);
        if (xlo) ld8(xlo + base, lv);
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            xv[k] = k < cnt ? x[base + eoff(k)] : 0.0;
            pv[k] = k < cnt ? p[base + eoff(k)] : (PVec)0;
            lv[k] = (xlo && k < cnt) ? xlo[base + eoff(k)] : 0.0f;
        }
    }
    if (!xlo) {
#pragma unroll
        for (int k = 0; k < 8; ++k) lv[k] = 0.0f;
    }
    float zf[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        xv[k] = xv[k] + alpha * (double)pv[k] + (double)lv[k];
        zf[k] = 0.0f;
    }
    if (cnt == 8) {
        st8(x + base, xv);
        if (xlo) st8(xlo + base, zf);
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k < cnt) {
                x[base + eoff(k)] = xv[k];
                if (xlo) xlo[base + eoff(k)] = 0.0f;
            }
    }
}

}  // namespace hub
