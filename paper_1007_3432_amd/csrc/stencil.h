// Stencil kernels of the fermion matrix M (Sec. 2, Eq. (10)) and of
// Q = M^T M (Sec. 4.2-4.3), templated over how the input vector is formed and
// what happens to the result ("ops"), so that one tiled sweep serves the bare
// matrix-vector product, CG's direction update and the FP64 true residual.
//
//   y_s = W x_s + A_s x_{s-1},         W = 1 - kappa H (H: periodic
//   z_s = W y_s + A_{s+1} y_{s+1}           nearest-neighbour adjacency)
//
// Site (n, s) lives at n + Vs*s.  A is the sign-folded time-link
// coefficient (negative except on slice 0, the antiperiodic wrap).
#pragma once

#include "common.h"

namespace hub {

// ---------------------------------------------------------------------------
// Link readers: A_{n,s} at linear index i (slice s).

struct Link64 {
    const double* a;
    __device__ double operator()(int i, int) const { return a[i]; }
};

struct Link32 {
    const float* a;
    __device__ float operator()(int i, int) const { return a[i]; }
};

// Stored sin(sigma) in FP16; A = -+(ls + lb * sin sigma) rebuilt in FP32
// with ls = exp(dtau mu), lb = ls * b, sign + on slice 0.
struct Link16 {
    const _Float16* sn;
    float ls, lb;
    __device__ float operator()(int i, int s) const {
        const float v = fmaf(lb, (float)sn[i], ls);
        return s == 0 ? v : -v;
    }
};

// ---------------------------------------------------------------------------
// Ops.  Interface:
//   acc_t, center_t          arithmetic type; per-site state kept from the
//                            input read to the output write
//   kReduce, kNP             whether out() feeds a grid reduction of kNP sums
//   skip()                   block-uniform early exit (device-side state)
//   begin()                  per-thread set-up from device-side scalars
//   link(i, s)               A at site i of slice s
//   in(i)                    input vector value at any site
//   in_center(i, c)          same, keeping what out() needs in c
//   out(i, z, v, c, part)    consume z = (Q in)_i, v = in_i; add to part[]
//   finish(total)            thread 0 of the last block: reduced totals
// No op writes a buffer that in() reads, so tiles may run in any order.

struct NoCenter {};

// Whether a fold / true-residual kernel of the given mode runs in state done.
__device__ inline bool mode_runs(int mode, int done) {
    if (mode == kModeFinal) return true;
    if (mode == kModeCheck) return done == kDoneIterConverged;
    return done <= kDoneIterConverged;
}

template <class Acc, class Vec, class Lnk>
struct OpApply {
    using acc_t = Acc;
    using center_t = NoCenter;
    static constexpr bool kReduce = false;
    static constexpr int kNP = 1;
    const Vec* x;
    Vec* z;
    Lnk lk;
    __device__ bool skip() const { return false; }
    __device__ void begin() {}
    __device__ Acc link(int i, int s) const { return lk(i, s); }
    __device__ Acc in(int i) const { return (Acc)x[i]; }
    __device__ Acc in_center(int i, NoCenter&) const { return (Acc)x[i]; }
    __device__ void out(int i, Acc zv, Acc, const NoCenter&, double (&)[kNP]) const {
        z[i] = (Vec)zv;
    }
    __device__ void finish(const double (&)[kNP]) const {}
};

// CG direction update fused with q = Q p (Sec. 4.1, CG on Q):
//   p_new = gamma r + beta p_old,  q = Q p_new,  x += alpha_prev p_old,
//   partial p_new . q  (FP64 accumulation); gamma = 1 except right after a
//   reliable update, where it removes the component of p along the new r.
// p is double-buffered by iteration parity so halo reads never see a p_new.
template <class Acc, class Vec, class XVec, class Lnk>
struct OpPhaseA {
    using acc_t = Acc;
    struct center_t { Acc pold; };
    static constexpr bool kReduce = true;
    static constexpr int kNP = 1;
    CGScalars* sc;
    const Vec* r;
    Vec* pbuf0;
    Vec* pbuf1;
    Vec* q;
    XVec* x;
    Lnk lk;
    // set by begin()
    const Vec* pold;
    Vec* pnew;
    Acc beta, alpha, gamma;
    __device__ bool skip() const { return sc->done != kRunning; }
    __device__ void begin() {
        const int it = sc->iter;
        pold = (it & 1) ? pbuf1 : pbuf0;
        pnew = (it & 1) ? pbuf0 : pbuf1;
        beta = (Acc)sc->beta;
        alpha = (Acc)sc->alpha;
        gamma = (Acc)sc->gamma;
    }
    __device__ Acc link(int i, int s) const { return lk(i, s); }
    __device__ Acc in(int i) const { return gamma * (Acc)r[i] + beta * (Acc)pold[i]; }
    __device__ Acc in_center(int i, center_t& c) const {
        c.pold = (Acc)pold[i];
        return gamma * (Acc)r[i] + beta * c.pold;
    }
    __device__ void out(int i, Acc zv, Acc v, const center_t& c, double (&part)[kNP]) const {
        pnew[i] = (Vec)v;
        q[i] = (Vec)zv;
        x[i] = (XVec)((Acc)x[i] + alpha * c.pold);
        part[0] += (double)v * (double)zv;
    }
    __device__ void finish(const double (&tot)[kNP]) const {
        const double pq = tot[0];
        sc->pq = pq;
        sc->gamma = 1.0;
        if (!(pq > 0.0) || !isfinite(pq)) {
            sc->done = kDoneBreakdown;
            sc->alpha = 0.0;  // alpha_prev was applied above
        } else {
            sc->alpha = sc->rho / pq;
        }
    }
};

// FP64 true residual r = phi - Q x (Q with FP64 links); reduces |r|^2 and
// r.p.  The result replaces CG's residual (FP64, or rounded to FP32 in the
// mixed solver) and decides convergence.  In the mixed solver (delta2 > 0)
// the next direction is also made orthogonal to the new residual, the
// reliable-update rule of Clark et al. (2010) for mixed-precision CG.
template <class RVec>
struct OpResidual {
    using acc_t = double;
    using center_t = NoCenter;
    static constexpr bool kReduce = true;
    static constexpr int kNP = 2;
    CGScalars* sc;
    const double* x;
    const double* phi;
    RVec* r;
    const RVec* pbuf0;
    const RVec* pbuf1;
    Link64 lk;
    int mode;
    const RVec* pcur;  // set by begin()
    __device__ bool skip() const { return !mode_runs(mode, sc->done); }
    __device__ void begin() { pcur = (sc->iter & 1) ? pbuf1 : pbuf0; }
    __device__ double link(int i, int s) const { return lk(i, s); }
    __device__ double in(int i) const { return x[i]; }
    __device__ double in_center(int i, NoCenter&) const { return x[i]; }
    __device__ void out(int i, double zv, double, const NoCenter&, double (&part)[kNP]) const {
        const double d = phi[i] - zv;
        const RVec rd = (RVec)d;
        r[i] = rd;
        part[0] += d * d;
        part[1] += (double)rd * (double)pcur[i];
    }
    __device__ void finish(const double (&tot)[kNP]) const {
        const double rr = tot[0];
        sc->rho_true = rr;
        sc->alpha = 0.0;  // folded into x by the preceding fold kernel
        if (mode == kModeFinal) return;
        sc->reliable_updates += 1;
        if (rr <= sc->tol2phi2) {
            sc->done = kDoneConverged;
        } else if (!isfinite(rr)) {
            sc->done = kDoneBreakdown;
        } else if (sc->iter >= sc->max_iter) {
            sc->done = kDoneMaxIter;
        } else {
            // Continue from the true residual, keeping the direction p.
            const double beta = rr / sc->rho_prev;
            double gamma = 1.0;
            if (sc->delta2 > 0.0 && rr > 0.0) gamma = 1.0 - beta * (tot[1] / rr);
            sc->beta = beta;
            sc->gamma = gamma;
            sc->rho = rr;
            sc->rho_ru = rr;
            sc->done = kRunning;
        }
    }
};

// ---------------------------------------------------------------------------
// Fused Q = M^T M sweep for d = 1.
//
// A block owns a strip of TX consecutive sites in x and TT consecutive time
// slices.  It stages the input on slices s0-1 .. s0+TT (sites n0-2 .. n0+w+1)
// in LDS, keeps A at its own sites in registers, forms y = M in one slice at
// a time (own sites plus one halo site each side) in a 3-deep LDS ring, and
// emits z = M^T y for slice s-1 as soon as y_s exists.  HBM traffic is the
// input and A once (halo rows and columns are shared with neighbouring
// tiles through L2) plus the outputs.
template <class Op, int TX, int TT>
__global__ __launch_bounds__(TX) void k_mtm_d1(Geom g, Op op, int tiles_x,
                                               double* partials, uint32_t* ticket) {
    using Acc = typename Op::acc_t;
    using Center = typename Op::center_t;
    __shared__ Acc xs[TT + 2][TX + 4];
    __shared__ Acc ys[3][TX + 2];
    if (op.skip()) return;
    op.begin();
    const int nx = g.nx, nt = g.nt;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = b % tiles_x, tt = b / tiles_x;
    const int n0 = tx * TX, s0 = tt * TT;
    const int w = min(TX, nx - n0), h = min(TT, nt - s0);
    const int t = threadIdx.x;
    const bool own = t < w;
    const Acc kappa = (Acc)g.kappa;

    Center cen[TT];
    Acc cval[TT];
    Acc acen[TT + 1];
    Acc ahalo[TT + 1];

    // x halo lanes 0..3 fill LDS positions 0, 1, w+2, w+3.
    const int hpos = t < 2 ? t : w + t;
    const int hsite = wrap1(n0 - 2 + hpos, nx);
    // A halo lanes 0, 1 hold A at sites n0-1 and n0+w.
    const int asite = wrap1(t == 0 ? n0 - 1 : n0 + w, nx);

#pragma unroll
    for (int rho = 0; rho < TT + 2; ++rho) {
        if (rho < h + 2) {
            const int row = wrap1(s0 - 1 + rho, nt) * nx;
            if (own) {
                Acc v;
                if (rho >= 1 && rho <= TT && rho <= h) {
                    v = op.in_center(row + n0 + t, cen[rho - 1]);
                    cval[rho - 1] = v;
                } else {
                    v = op.in(row + n0 + t);
                }
                xs[rho][t + 2] = v;
            }
            if (t < 4) xs[rho][hpos] = op.in(row + hsite);
        }
    }
#pragma unroll
    for (int rho = 0; rho < TT + 1; ++rho) {
        if (rho <= h) {
            const int s = wrap1(s0 + rho, nt);
            const int row = s * nx;
            if (own) acen[rho] = op.link(row + n0 + t, s);
            if (t < 2) ahalo[rho] = op.link(row + asite, s);
        }
    }
    __syncthreads();

    double part[Op::kNP] = {};
#pragma unroll
    for (int rho = 0; rho < TT + 1; ++rho) {
        if (rho <= h) {
            Acc* yb = ys[rho % 3];
            if (own)
                yb[t + 1] = xs[rho + 1][t + 2] -
                            kappa * (xs[rho + 1][t + 1] + xs[rho + 1][t + 3]) +
                            acen[rho] * xs[rho][t + 2];
            if (t < 2) {
                const int j = t == 0 ? 0 : w + 1;
                yb[j] = xs[rho + 1][j + 1] -
                        kappa * (xs[rho + 1][j] + xs[rho + 1][j + 2]) +
                        ahalo[rho] * xs[rho][j + 1];
            }
            __syncthreads();
            if (rho >= 1 && own) {
                const Acc* yp = ys[(rho - 1) % 3];
                const Acc zv = yp[t + 1] - kappa * (yp[t] + yp[t + 2]) +
                               acen[rho] * yb[t + 1];
                op.out((s0 + rho - 1) * nx + n0 + t, zv, cval[rho - 1],
                       cen[rho - 1], part);
            }
        }
    }
    if constexpr (Op::kReduce) {
        double total[Op::kNP];
        if (grid_sum_last<TX, Op::kNP>(part, partials, ticket, total) && t == 0)
            op.finish(total);
    }
}

// ---------------------------------------------------------------------------
// Generic two-pass path for any d and any extents: y = M in (pass 1, into a
// scratch vector), then z = M^T y with the op's epilogue (pass 2).

template <class Op>
__device__ inline typename Op::acc_t gen_M_at(const Geom& g, const Op& op, int i) {
    using Acc = typename Op::acc_t;
    const int n = i % g.vs, s = i / g.vs;
    Acc hop = 0;
    int stride = 1;
    for (int j = 0; j < g.d; ++j) {
        const int c = (n / stride) % g.nx;
        const int cp = c + 1 == g.nx ? 0 : c + 1;
        const int cm = c == 0 ? g.nx - 1 : c - 1;
        hop += op.in(i + (cp - c) * stride) + op.in(i + (cm - c) * stride);
        stride *= g.nx;
    }
    const int sm = s == 0 ? g.nt - 1 : s - 1;
    return op.in(i) - (Acc)g.kappa * hop + op.link(i, s) * op.in(n + sm * g.vs);
}

template <class Op>
__global__ __launch_bounds__(256) void k_gen_pass1(Geom g, Op op, typename Op::acc_t* y) {
    if (op.skip()) return;
    op.begin();
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < g.V) y[i] = gen_M_at(g, op, i);
}

template <class Op>
__global__ __launch_bounds__(256) void k_gen_pass2(Geom g, Op op,
                                                   const typename Op::acc_t* y,
                                                   double* partials, uint32_t* ticket) {
    using Acc = typename Op::acc_t;
    if (op.skip()) return;
    op.begin();
    const int i = blockIdx.x * 256 + threadIdx.x;
    double part[Op::kNP] = {};
    if (i < g.V) {
        const int n = i % g.vs, s = i / g.vs;
        Acc hop = 0;
        int stride = 1;
        for (int j = 0; j < g.d; ++j) {
            const int c = (n / stride) % g.nx;
            const int cp = c + 1 == g.nx ? 0 : c + 1;
            const int cm = c == 0 ? g.nx - 1 : c - 1;
            hop += y[i + (cp - c) * stride] + y[i + (cm - c) * stride];
            stride *= g.nx;
        }
        const int sp = s == g.nt - 1 ? 0 : s + 1;
        const int ip = n + sp * g.vs;
        const Acc zv = y[i] - (Acc)g.kappa * hop + op.link(ip, sp) * y[ip];
        typename Op::center_t c;
        const Acc v = op.in_center(i, c);
        op.out(i, zv, v, c, part);
    }
    if constexpr (Op::kReduce) {
        double total[Op::kNP];
        if (grid_sum_last<256, Op::kNP>(part, partials, ticket, total) && threadIdx.x == 0)
            op.finish(total);
    }
}

// ---------------------------------------------------------------------------
// Single M or M^T (hub_apply_M): one lane per site, neighbours through L1/L2.
template <class Acc, class Vec, class Lnk, bool TRANSPOSE>
__global__ __launch_bounds__(256) void k_apply_M(Geom g, Lnk lk, const Vec* x, Vec* y) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= g.V) return;
    const int n = i % g.vs, s = i / g.vs;
    Acc hop = 0;
    int stride = 1;
    for (int j = 0; j < g.d; ++j) {
        const int c = (n / stride) % g.nx;
        const int cp = c + 1 == g.nx ? 0 : c + 1;
        const int cm = c == 0 ? g.nx - 1 : c - 1;
        hop += (Acc)x[i + (cp - c) * stride] + (Acc)x[i + (cm - c) * stride];
        stride *= g.nx;
    }
    Acc v = (Acc)x[i] - (Acc)g.kappa * hop;
    if (!TRANSPOSE) {
        const int sm = s == 0 ? g.nt - 1 : s - 1;
        v += (Acc)lk(i, s) * (Acc)x[n + sm * g.vs];
    } else {
        const int sp = s == g.nt - 1 ? 0 : s + 1;
        const int ip = n + sp * g.vs;
        v += (Acc)lk(ip, sp) * (Acc)x[ip];
    }
    y[i] = (Vec)v;
}

}  // namespace hub
