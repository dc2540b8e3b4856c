// Element-wise tiles of the conjugate-gradient iteration (Sec. 4.1) and the
// scalar updates that follow each grid reduction.  Shared by the one-solve
// kernels (cg.hip) and the persistent multi-solve serving kernel (serve.hip),
// so that a solve takes the same steps, with the same rounding, in both.
#pragma once

#include "common.h"

namespace hub {

// Sites per element-wise tile: 256 lanes x 8 sites, lane t handling sites
// tile*kETile + t + 256 k.
constexpr int kETile = 2048;

__host__ __device__ inline int elem_tiles(int V) { return (V + kETile - 1) / kETile; }

// r = phi, p0 = 0, x = 0 (x_lo = 0); part[0] += phi.phi.
template <class RVec>
__device__ __forceinline__ void tile_init(const double* __restrict__ phi, RVec* __restrict__ r,
                                          RVec* __restrict__ p0, double* __restrict__ x,
                                          float* __restrict__ xlo, int V, int tile,
                                          double (&part)[1]) {
    const int base = tile * kETile + threadIdx.x;
    double f[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) f[k] = phi[min(base + 256 * k, V - 1)];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int i = base + 256 * k;
        if (i < V) {
            r[i] = (RVec)f[k];
            p0[i] = (RVec)0;
            x[i] = 0.0;
            if (xlo) xlo[i] = 0.0f;
            part[0] += f[k] * f[k];
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
    sc->done = !isfinite(total) ? kDoneBreakdown : (total == 0.0 ? kDoneConverged : kRunning);
}

// r -= alpha q; part[0] += r.r (FP64 accumulation of the stored r).
template <class Vec>
__device__ __forceinline__ void tile_phaseB(Vec* __restrict__ r, const Vec* __restrict__ q,
                                            Vec alpha, int V, int tile, double (&part)[1]) {
    const int base = tile * kETile + threadIdx.x;
    Vec rv[8], qv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int i = min(base + 256 * k, V - 1);
        rv[k] = r[i];
        qv[k] = q[i];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int i = base + 256 * k;
        if (i < V) {
            const Vec v = rv[k] - alpha * qv[k];
            r[i] = v;
            part[0] += (double)v * (double)v;
        }
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

// x += alpha p (+ x_lo, then x_lo = 0): the pending update, in FP64.
template <class PVec>
__device__ __forceinline__ void tile_fold(double* __restrict__ x, float* __restrict__ xlo,
                                          const PVec* __restrict__ p, double alpha, int V,
                                          int tile) {
    const int base = tile * kETile + threadIdx.x;
    double xv[8], pv[8], lv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int i = min(base + 256 * k, V - 1);
        xv[k] = x[i];
        pv[k] = (double)p[i];
        lv[k] = xlo ? (double)xlo[i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int i = base + 256 * k;
        if (i < V) {
            x[i] = xv[k] + alpha * pv[k] + lv[k];
            if (xlo) xlo[i] = 0.0f;
        }
    }
}

}  // namespace hub
