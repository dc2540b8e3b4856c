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

#include <type_traits>

#include "common.h"

namespace hub {

// ---------------------------------------------------------------------------
// Link readers: A_{n,s} at linear index i (slice s).

// Two consecutive FP64 values (sites i, i+1 with i even) moved as one
// 16-byte access; the pair sweep of d = 1 uses these.
struct D2 {
    double a, b;
};
__device__ __forceinline__ D2 ld2(const double* p) {
    const double2 w = *reinterpret_cast<const double2*>(p);
    return {w.x, w.y};
}
// The same load with the non-temporal hint (streamed input, not kept).
__device__ __forceinline__ D2 ld2_nt(const double* p) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 w = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return {w.x, w.y};
}
__device__ __forceinline__ void st2(double* p, double a, double b) {
    *reinterpret_cast<double2*>(p) = make_double2(a, b);
}
typedef double d2_vec __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st2_nt(double* p, double a, double b) {
    const d2_vec v = {a, b};
    __builtin_nontemporal_store(v, reinterpret_cast<d2_vec*>(p));
}

// Every link reader splits the access into the load (raw) and the value
// (val), so that a sweep can issue the loads of a later slice early and form
// the values when it needs them.
struct Link64 {
    const double* a;
    using raw_t = double;
    __device__ double raw(int i) const { return a[i]; }
    __device__ double val(double r, int) const { return r; }
    __device__ D2 pair(int i, int) const { return ld2(a + i); }
};

struct Link32 {
    const float* a;
    using raw_t = float;
    __device__ float raw(int i) const { return a[i]; }
    __device__ float val(float r, int) const { return r; }
};

// Stored sin(sigma) in FP16; A = -+(ls + lb * sin sigma) rebuilt in FP32
// with ls = exp(dtau mu), lb = ls * b, sign + on slice 0.
struct Link16 {
    const _Float16* sn;
    float ls, lb;
    using raw_t = _Float16;
    __device__ _Float16 raw(int i) const { return sn[i]; }
    __device__ float val(_Float16 r, int s) const {
        const float v = fmaf(lb, (float)r, ls);
        return s == 0 ? v : -v;
    }
};

// ---------------------------------------------------------------------------
// Ops.  Interface:
//   acc_t, center_t          arithmetic type; per-site state kept from the
//                            input read to the output write
//   raw_t, craw_t, lraw_t    what load_h / load_c / lraw return
//   kReduce, kNP             whether out() feeds a grid reduction of kNP sums
//   skip()                   block-uniform early exit (device-side state)
//   begin()                  per-thread set-up from device-side scalars
//   load_h(i), val_h(raw)    input vector value at any site (halo sites):
//                            the loads, then the value formed from them
//   load_c(i), val_c(raw, c) the same at a site the tile owns, also loading
//                            everything out() needs into c
//   lraw(i), lval(raw, s)    A at site i of slice s, load and value
//   out(i, z, v, c, part)    consume z = (Q in)_i, v = in_i; stores only;
//                            add to part[]
//   finish(total)            thread 0 of the last block: reduced totals
//   kPair                    FP64 ops that also provide in2 / in_center2 /
//                            link2 / out2, the same for sites i, i+1 (i even)
//                            with 16-byte accesses (the d = 1 pair sweep)
// No op writes a buffer that another site's input reads, so tiles may run in
// any order; out() at site i writes only buffers that load_c(i) of the same
// lane has already read.

struct NoCenter {};

template <class Op>
__device__ __forceinline__ typename Op::acc_t op_in(const Op& op, int i) {
    return op.val_h(op.load_h(i));
}
template <class Op>
__device__ __forceinline__ typename Op::acc_t op_in_center(const Op& op, int i,
                                                           typename Op::center_t& c) {
    return op.val_c(op.load_c(i), c);
}
template <class Op>
__device__ __forceinline__ typename Op::acc_t op_link(const Op& op, int i, int s) {
    return op.lval(op.lraw(i), s);
}

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
    using raw_t = Vec;
    using craw_t = Vec;
    using lraw_t = typename Lnk::raw_t;
    static constexpr bool kReduce = false;
    static constexpr int kNP = 1;
    const Vec* x;
    Vec* z;
    Lnk lk;
    __device__ bool skip() const { return false; }
    __device__ bool begin() { return true; }
    __device__ Vec load_h(int i) const { return x[i]; }
    __device__ Acc val_h(Vec r) const { return (Acc)r; }
    __device__ Vec load_c(int i) const { return x[i]; }
    __device__ Acc val_c(Vec r, NoCenter&) const { return (Acc)r; }
    __device__ lraw_t lraw(int i) const { return lk.raw(i); }
    __device__ Acc lval(lraw_t r, int s) const { return (Acc)lk.val(r, s); }
    // The result is not read again by this sweep: stream it past the caches
    // (non-temporal stores), so that it does not wait in L2 for the
    // write-back at the end of the kernel.
    __device__ void out(int i, Acc zv, Acc, const NoCenter&, double (&)[kNP]) const {
        __builtin_nontemporal_store((Vec)zv, z + i);
    }
    __device__ void finish(const double (&)[kNP]) const {}
    static constexpr bool kPair = sizeof(Acc) == 8 && sizeof(Vec) == 8 &&
                                  std::is_same<Lnk, Link64>::value;
    static constexpr bool kMarch = kPair;
    // The input rows of the pair tiles are loaded with the non-temporal hint
    // (d=1 2048x512: 6.83 -> 6.50 us, 8192x1024: 40.8 -> 34.7 us); the
    // links are not (the same hint on them made both slower again).
    __device__ D2 in2(int i) const { return ld2_nt((const double*)x + i); }
    __device__ D2 in_center2(int i, NoCenter&, NoCenter&) const { return in2(i); }
    __device__ D2 link2(int i, int s) const { return lk.pair(i, s); }
    __device__ void out2(int i, D2 zv, D2, const NoCenter&, const NoCenter&,
                         double (&)[kNP]) const {
        st2_nt((double*)z + i, zv.a, zv.b);
    }
};

// CG direction update fused with q = Q p (Sec. 4.1, CG on Q):
//   p_new = gamma r + beta p_old,  q = Q p_new,  x += alpha_prev p_old,
//   partial p_new . q  (FP64 accumulation); gamma = 1 except right after a
//   reliable update, where it removes the component of p along the new r.
// p is double-buffered by iteration parity so halo reads never see a p_new.
// The p.q deposits are added either by a one-block finalize (finish(), which
// sets alpha) or by the next kernel's blocks themselves.
template <class Acc, class Vec, class XVec, class Lnk>
struct OpPhaseA {
    using acc_t = Acc;
    struct center_t {
        Acc pold;
        XVec xold;
    };
    struct raw_t {
        Vec r, p;
    };
    struct craw_t {
        Vec r, p;
        XVec x;
    };
    using lraw_t = typename Lnk::raw_t;
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
    __device__ bool begin() {
        const int it = sc->iter;
        pold = (it & 1) ? pbuf1 : pbuf0;
        pnew = (it & 1) ? pbuf0 : pbuf1;
        beta = (Acc)sc->beta;
        alpha = (Acc)sc->alpha;
        gamma = (Acc)sc->gamma;
        return true;
    }
    __device__ raw_t load_h(int i) const { return {r[i], pold[i]}; }
    __device__ Acc val_h(const raw_t& v) const { return gamma * (Acc)v.r + beta * (Acc)v.p; }
    __device__ craw_t load_c(int i) const { return {r[i], pold[i], x[i]}; }
    __device__ Acc val_c(const craw_t& v, center_t& c) const {
        c.pold = (Acc)v.p;
        c.xold = v.x;
        return gamma * (Acc)v.r + beta * c.pold;
    }
    __device__ lraw_t lraw(int i) const { return lk.raw(i); }
    __device__ Acc lval(lraw_t v, int s) const { return (Acc)lk.val(v, s); }
    __device__ void out(int i, Acc zv, Acc v, const center_t& c, double (&part)[kNP]) const {
        pnew[i] = (Vec)v;
        q[i] = (Vec)zv;
        x[i] = (XVec)((Acc)c.xold + alpha * c.pold);
        part[0] += (double)v * (double)zv;
    }
    static constexpr bool kPair = sizeof(Acc) == 8 && sizeof(Vec) == 8 && sizeof(XVec) == 8 &&
                                  std::is_same<Lnk, Link64>::value;
    __device__ D2 in2(int i) const {
        const D2 rv = ld2((const double*)r + i), pv = ld2((const double*)pold + i);
        return {gamma * rv.a + beta * pv.a, gamma * rv.b + beta * pv.b};
    }
    __device__ D2 in_center2(int i, center_t& c0, center_t& c1) const {
        const D2 rv = ld2((const double*)r + i), pv = ld2((const double*)pold + i);
        c0.pold = pv.a;
        c1.pold = pv.b;
        return {gamma * rv.a + beta * pv.a, gamma * rv.b + beta * pv.b};
    }
    __device__ D2 link2(int i, int s) const { return lk.pair(i, s); }
    __device__ void out2(int i, D2 zv, D2 v, const center_t& c0, const center_t& c1,
                         double (&part)[kNP]) const {
        st2((double*)pnew + i, v.a, v.b);
        st2((double*)q + i, zv.a, zv.b);
        const D2 xv = ld2((const double*)x + i);
        st2((double*)x + i, xv.a + alpha * c0.pold, xv.b + alpha * c1.pold);
        part[0] += v.a * zv.a;
        part[0] += v.b * zv.b;
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
    struct center_t {
        double phi;
        RVec pc;
    };
    using raw_t = double;
    struct craw_t {
        double x, phi;
        RVec pc;
    };
    using lraw_t = double;
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
    __device__ bool begin() {
        pcur = (sc->iter & 1) ? pbuf1 : pbuf0;
        return true;
    }
    __device__ double load_h(int i) const { return x[i]; }
    __device__ double val_h(double v) const { return v; }
    __device__ craw_t load_c(int i) const { return {x[i], phi[i], pcur[i]}; }
    __device__ double val_c(const craw_t& v, center_t& c) const {
        c.phi = v.phi;
        c.pc = v.pc;
        return v.x;
    }
    __device__ double lraw(int i) const { return lk.raw(i); }
    __device__ double lval(double v, int s) const { return lk.val(v, s); }
    __device__ void out(int i, double zv, double, const center_t& c, double (&part)[kNP]) const {
        const double d = c.phi - zv;
        const RVec rd = (RVec)d;
        r[i] = rd;
        part[0] += d * d;
        part[1] += (double)rd * (double)c.pc;
    }
    static constexpr bool kPair = sizeof(RVec) == 8;
    __device__ D2 in2(int i) const { return ld2(x + i); }
    __device__ D2 in_center2(int i, center_t&, center_t&) const { return ld2(x + i); }
    __device__ D2 link2(int i, int s) const { return lk.pair(i, s); }
    __device__ void out2(int i, D2 zv, D2, const center_t&, const center_t&,
                         double (&part)[kNP]) const {
        const D2 f = ld2(phi + i), pc = ld2((const double*)pcur + i);
        const double d0 = f.a - zv.a, d1 = f.b - zv.b;
        st2((double*)r + i, d0, d1);
        part[0] += d0 * d0;
        part[0] += d1 * d1;
        part[1] += d0 * pc.a;
        part[1] += d1 * pc.b;
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
            sc->rr = rr;
            sc->restart = 1;  // preconditioned CG restarts from the new r
            sc->done = kRunning;
        }
    }
};

// One quadratic factor of the Chebyshev preconditioner (Sec. 4.2, Eq. (13)):
// a conjugate root pair z, z* of P gives the real factor
//   (Q/s - z)(Q/s - z*) = c2 Q^2 + c1 Q + c0   (times its normalisation),
// applied as two sweeps: w = Q v (OpApply-like, OpChebW), then
// v_out = c2 Q w + c1 w + c0 v (OpChebZ), which reads v only at the site it
// writes, so v_out may be v.  The last factor of a preconditioned CG step also
// reduces r.z and sets beta.  With sc == nullptr the ops never skip.
struct OpChebW {
    using acc_t = double;
    using center_t = NoCenter;
    using raw_t = double;
    using craw_t = double;
    using lraw_t = double;
    static constexpr bool kReduce = false;
    static constexpr int kNP = 1;
    const CGScalars* sc;
    const double* v;
    double* w;
    Link64 lk;
    __device__ bool skip() const { return sc && sc->done != kRunning; }
    __device__ bool begin() { return true; }
    __device__ double load_h(int i) const { return v[i]; }
    __device__ double val_h(double r) const { return r; }
    __device__ double load_c(int i) const { return v[i]; }
    __device__ double val_c(double r, NoCenter&) const { return r; }
    __device__ double lraw(int i) const { return lk.raw(i); }
    __device__ double lval(double r, int s) const { return lk.val(r, s); }
    __device__ void out(int i, double zv, double, const NoCenter&, double (&)[kNP]) const {
        w[i] = zv;
    }
    __device__ void finish(const double (&)[kNP]) const {}
    static constexpr bool kPair = true;
    __device__ D2 in2(int i) const { return ld2(v + i); }
    __device__ D2 in_center2(int i, NoCenter&, NoCenter&) const { return ld2(v + i); }
    __device__ D2 link2(int i, int s) const { return lk.pair(i, s); }
    __device__ void out2(int i, D2 zv, D2, const NoCenter&, const NoCenter&,
                         double (&)[kNP]) const {
        st2(w + i, zv.a, zv.b);
    }
};

template <bool kDot>
struct OpChebZ {
    using acc_t = double;
    struct center_t {
        double v, r;
    };
    using raw_t = double;
    struct craw_t {
        double w, v, r;
    };
    using lraw_t = double;
    static constexpr bool kReduce = kDot;
    static constexpr int kNP = 1;
    CGScalars* sc;
    const double* w;
    const double* v;   // factor input (read at the written site only)
    double* vout;
    const double* r;   // kDot: residual for r.z
    double c2, c1, c0;
    Link64 lk;
    __device__ bool skip() const { return sc && sc->done != kRunning; }
    __device__ bool begin() { return true; }
    __device__ double load_h(int i) const { return w[i]; }
    __device__ double val_h(double x) const { return x; }
    __device__ craw_t load_c(int i) const { return {w[i], v[i], kDot ? r[i] : 0.0}; }
    __device__ double val_c(const craw_t& x, center_t& c) const {
        c.v = x.v;
        c.r = x.r;
        return x.w;
    }
    __device__ double lraw(int i) const { return lk.raw(i); }
    __device__ double lval(double x, int s) const { return lk.val(x, s); }
    __device__ void out(int i, double zv, double wv, const center_t& c, double (&part)[kNP]) const {
        const double o = c2 * zv + c1 * wv + c0 * c.v;
        vout[i] = o;
        if constexpr (kDot) part[0] += c.r * o;
    }
    static constexpr bool kPair = true;
    __device__ D2 in2(int i) const { return ld2(w + i); }
    __device__ D2 in_center2(int i, center_t&, center_t&) const { return ld2(w + i); }
    __device__ D2 link2(int i, int s) const { return lk.pair(i, s); }
    __device__ void out2(int i, D2 zv, D2 wv, const center_t&, const center_t&,
                         double (&part)[kNP]) const {
        const D2 vv = ld2(v + i);
        const double o0 = c2 * zv.a + c1 * wv.a + c0 * vv.a;
        const double o1 = c2 * zv.b + c1 * wv.b + c0 * vv.b;
        st2(vout + i, o0, o1);
        if constexpr (kDot) {
            const D2 rv = ld2(r + i);
            part[0] += rv.a * o0;
            part[0] += rv.b * o1;
        }
    }
    // rho = r.z; beta = 0 after a restart, else r.z / previous r.z.
    __device__ void finish(const double (&tot)[kNP]) const {
        if constexpr (kDot) {
            const double rz = tot[0];
            if (!(rz > 0.0) || !isfinite(rz)) {
                sc->done = kDoneBreakdown;
                return;
            }
            sc->beta = sc->restart ? 0.0 : rz / sc->rho;
            sc->rho_prev = sc->rho;
            sc->rho = rz;
            sc->gamma = 1.0;
            sc->restart = 0;
        }
    }
};

// One-block finalize of an op's reduction: the deposits of n tiles in tile
// order, then op.finish (solver scalar update).
template <class Op>
__global__ __launch_bounds__(256) void k_finish_op(Op op, const double* partials, int n) {
    if (op.skip()) return;
    double total[Op::kNP];
    reduce_deposits<256, Op::kNP>(partials, n, total);
    if (threadIdx.x == 0) op.finish(total);
}

// ---------------------------------------------------------------------------
// Fused Q = M^T M sweep for d = 1.
//
// A tile is a strip of TX consecutive x-sites by TT consecutive time slices;
// each 64-lane wavefront of the block owns 64 of the x-sites and works on
// its own, with no LDS and no block barrier: lane i keeps its site's input
// on slices s0-1 .. s0+TT and A on slices s0 .. s0+TT in registers, takes
// x-neighbours from lanes i-1 and i+1 (cross-lane shuffles), and the first
// and last active lanes load the two sites past each end of the wavefront's
// strip.  Slice by slice it forms y = M in at its site (and the end lanes at
// the halo site next to it) and then z = M^T y one slice behind.  HBM
// traffic is the input and A once (the few halo re-reads hit in cache) plus
// the outputs.  Lanes past a ragged edge and slices past a ragged end
// re-read the last valid site / slice, so every load is unconditional.

template <int TX, int TT>
constexpr int d1_lds_elems() { return 0; }

// Moves by one lane across the 64-wide wavefront as DPP wavefront shifts
// (wave_shr:1 / wave_shl:1, a register move per 32 bits, no LDS round trip).
// The lane without a source (lane 0 up, lane 63 down) keeps its own value.
template <int CTRL, class T>
__device__ __forceinline__ T dpp_wave_shift(T v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        const int w = __builtin_bit_cast(int, v);
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(w, w, CTRL, 0xf, 0xf, false));
    } else {
        const long long w = __builtin_bit_cast(long long, v);
        const int lo = (int)w, hi = (int)(w >> 32);
        const int rlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
        const int rhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
        return __builtin_bit_cast(T, (long long)(((unsigned long long)(unsigned)rhi << 32) |
                                                 (unsigned)rlo));
    }
}
template <class T>
__device__ __forceinline__ T lane_up(T v) { return dpp_wave_shift<0x138>(v); }    // from lane-1
template <class T>
__device__ __forceinline__ T lane_down(T v) { return dpp_wave_shift<0x130>(v); }  // from lane+1

// One tile b of the sweep (block of >= TX lanes, TX a multiple of 64); adds
// this lane's share of the op's sums to part.
template <class Op, int TX, int TT>
__device__ __forceinline__ void tile_mtm_d1(const Geom& g, const Op& op, int tiles_x, int b,
                                            typename Op::acc_t* /*lds*/,
                                            double (&part)[Op::kNP]) {
    static_assert(TX % 64 == 0, "tile width is whole wavefronts");
    using Acc = typename Op::acc_t;
    using Center = typename Op::center_t;
    const int nx = g.nx, nt = g.nt;
    const int tx = b % tiles_x, tt = b / tiles_x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave >= TX / 64) return;
    const int n0 = tx * TX + 64 * wave;            // first site of this wavefront
    const int w = min(64, nx - n0);                // its active lanes
    if (w <= 0) return;
    const int s0 = tt * TT, h = min(TT, nt - s0);
    const Acc kappa = (Acc)g.kappa;
    const bool own = lane < w;
    const int site = n0 + (own ? lane : w - 1);
    // A one-site strip (nx = 1 mod 64) lends lane 1 the right end: it loads
    // the right halo and lane 0 takes those values by shuffle.
    const bool solo = w == 1;
    const bool left = lane == 0, right = lane == (solo ? 1 : w - 1);
    // End lanes: h1 = the site next to the strip, h2 = the one after it.
    const int h1 = wrap1(left ? n0 - 1 : n0 + w, nx);
    const int h2 = wrap1(left ? n0 - 2 : n0 + w + 1, nx);

    Acc xv[TT + 2], av[TT + 1];
    Acc x1[TT + 2], x2[TT + 2], a1[TT + 1];
    Center cen[TT];
#pragma unroll
    for (int rho = 0; rho < TT + 2; ++rho) {
        const int row = wrap1(s0 - 1 + (rho < h + 2 ? rho : h + 1), nt) * nx;
        if (rho >= 1 && rho <= TT)
            xv[rho] = op_in_center(op, row + site, cen[rho - 1]);
        else
            xv[rho] = op_in(op, row + site);
    }
#pragma unroll
    for (int rho = 0; rho < TT + 1; ++rho) {
        const int sl = wrap1(s0 + (rho <= h ? rho : h), nt);
        av[rho] = op_link(op, sl * nx + site, sl);
    }
    if (left || right) {
#pragma unroll
        for (int rho = 0; rho < TT + 2; ++rho) {
            const int row = wrap1(s0 - 1 + (rho < h + 2 ? rho : h + 1), nt) * nx;
            x1[rho] = op_in(op, row + h1);
            x2[rho] = op_in(op, row + h2);
        }
#pragma unroll
        for (int rho = 0; rho < TT + 1; ++rho) {
            const int sl = wrap1(s0 + (rho <= h ? rho : h), nt);
            a1[rho] = op_link(op, sl * nx + h1, sl);
        }
    }

    Acc y_prev = 0, yh_prev = 0;
#pragma unroll
    for (int rho = 0; rho < TT + 1; ++rho) {
        if (rho <= h) {
            // y on slice s0+rho at the lane's site, and at the halo site
            // next to the end lanes.
            const Acc xc = xv[rho + 1];
            Acc xm = lane_up(xc), xp = lane_down(xc);
            if (left) xm = x1[rho + 1];
            if (right) xp = x1[rho + 1];
            if (solo) {
                const Acc xr = lane_down(x1[rho + 1]);
                if (left) xp = xr;
            }
            const Acc y = xc - kappa * (xm + xp) + av[rho] * xv[rho];
            Acc yh = 0;
            if (left || right)
                yh = x1[rho + 1] - kappa * (x2[rho + 1] + xc) + a1[rho] * x1[rho];
            if (rho >= 1) {
                // z on slice s0+rho-1 from y there (and its neighbours) and y here.
                Acc ym = lane_up(y_prev), yp = lane_down(y_prev);
                if (left) ym = yh_prev;
                if (right) yp = yh_prev;
                if (solo) {
                    const Acc yr = lane_down(yh_prev);
                    if (left) yp = yr;
                }
                const Acc zv = y_prev - kappa * (ym + yp) + av[rho] * y;
                if (own)
                    op.out((s0 + rho - 1) * nx + n0 + lane, zv, xv[rho], cen[rho - 1], part);
            }
            y_prev = y;
            yh_prev = yh;
        }
    }
}

template <class Op, int TX, int TT>
__global__ __launch_bounds__(TX) void k_mtm_d1(Geom g, Op op, int tiles_x, int ntiles,
                                               double* partials) {
    if (op.skip()) return;
    if (!op.begin()) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    double part[Op::kNP] = {};
    if (b < ntiles) tile_mtm_d1<Op, TX, TT>(g, op, tiles_x, b, nullptr, part);
    if constexpr (Op::kReduce) deposit<TX, Op::kNP>(part, partials, b);
}

// Whether an op provides the pair accessors (kPair, default false).
template <class Op, class = void>
struct op_has_pair : std::false_type {};
template <class Op>
struct op_has_pair<Op, std::void_t<decltype(Op::kPair)>> : std::bool_constant<Op::kPair> {};

// ---------------------------------------------------------------------------
// Pair variant of the d = 1 sweep (FP64 ops, nx even).
//
// As tile_mtm_d1, but each lane owns two adjacent x-sites, so a wavefront
// covers 128 sites and every access of the owned sites is one 16-byte load
// or store.  Inside a pair the x-neighbours are the lane's own values; across
// pairs one cross-lane shuffle per direction and slice suffices (the left
// neighbour of site 2l is the second site of lane l-1).  With nx even every
// row starts at an even index, so pairs stay 16-byte aligned.
template <class Op, int TX, int TT>
__device__ __forceinline__ void tile_mtm_d1p(const Geom& g, const Op& op, int tiles_x, int b,
                                             double (&part)[Op::kNP]) {
    static_assert(TX % 128 == 0, "tile width is whole pair wavefronts");
    using Center = typename Op::center_t;
    const int nx = g.nx, nt = g.nt;
    const int tx = b % tiles_x, tt = b / tiles_x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave >= TX / 128) return;
    const int n0 = tx * TX + 128 * wave;            // first site of this wavefront
    const int w = min(128, nx - n0);                // its sites (even)
    if (w <= 0) return;
    const int np = w >> 1;                          // its active lanes
    const int s0 = tt * TT, h = min(TT, nt - s0);
    const double kappa = g.kappa;
    const bool own = lane < np;
    const int site = n0 + 2 * (own ? lane : np - 1);
    // A one-pair strip (nx = 2 mod 128) lends lane 1 the right end, as in
    // tile_mtm_d1.
    const bool solo = np == 1;
    const bool left = lane == 0, right = lane == (solo ? 1 : np - 1);
    const int h1 = wrap1(left ? n0 - 1 : n0 + w, nx);
    const int h2 = wrap1(left ? n0 - 2 : n0 + w + 1, nx);

    D2 xv[TT + 2], av[TT + 1];
    double x1[TT + 2], x2[TT + 2], a1[TT + 1];
    Center cen[TT][2];
#pragma unroll
    for (int rho = 0; rho < TT + 2; ++rho) {
        const int row = wrap1(s0 - 1 + (rho < h + 2 ? rho : h + 1), nt) * nx;
        if (rho >= 1 && rho <= TT)
            xv[rho] = op.in_center2(row + site, cen[rho - 1][0], cen[rho - 1][1]);
        else
            xv[rho] = op.in2(row + site);
    }
#pragma unroll
    for (int rho = 0; rho < TT + 1; ++rho) {
        const int sl = wrap1(s0 + (rho <= h ? rho : h), nt);
        av[rho] = op.link2(sl * nx + site, sl);
    }
    if (left || right) {
#pragma unroll
        for (int rho = 0; rho < TT + 2; ++rho) {
            const int row = wrap1(s0 - 1 + (rho < h + 2 ? rho : h + 1), nt) * nx;
            x1[rho] = op_in(op, row + h1);
            x2[rho] = op_in(op, row + h2);
        }
#pragma unroll
        for (int rho = 0; rho < TT + 1; ++rho) {
            const int sl = wrap1(s0 + (rho <= h ? rho : h), nt);
            a1[rho] = op_link(op, sl * nx + h1, sl);
        }
    }

    D2 y_prev{0.0, 0.0};
    double yh_prev = 0.0;
#pragma unroll
    for (int rho = 0; rho < TT + 1; ++rho) {
        if (rho <= h) {
            const D2 xc = xv[rho + 1];
            double xm = lane_up(xc.b), xp = lane_down(xc.a);
            if (left) xm = x1[rho + 1];
            if (right) xp = x1[rho + 1];
            if (solo) {
                const double xr = lane_down(x1[rho + 1]);
                if (left) xp = xr;
            }
            D2 y;
            y.a = xc.a - kappa * (xm + xc.b) + av[rho].a * xv[rho].a;
            y.b = xc.b - kappa * (xc.a + xp) + av[rho].b * xv[rho].b;
            double yh = 0.0;
            if (left || right)
                yh = x1[rho + 1] - kappa * (x2[rho + 1] + (left ? xc.a : xc.b)) +
                     a1[rho] * x1[rho];
            if (rho >= 1) {
                double ym = lane_up(y_prev.b), yp = lane_down(y_prev.a);
                if (left) ym = yh_prev;
                if (right) yp = yh_prev;
                if (solo) {
                    const double yr = lane_down(yh_prev);
                    if (left) yp = yr;
                }
                D2 zv;
                zv.a = y_prev.a - kappa * (ym + y_prev.b) + av[rho].a * y.a;
                zv.b = y_prev.b - kappa * (y_prev.a + yp) + av[rho].b * y.b;
                if (own)
                    op.out2((s0 + rho - 1) * nx + site, zv, xv[rho], cen[rho - 1][0],
                            cen[rho - 1][1], part);
            }
            y_prev = y;
            yh_prev = yh;
        }
    }
}

template <class Op, int TX, int TT>
__global__ __launch_bounds__(TX / 2) void k_mtm_d1p(Geom g, Op op, int tiles_x, int ntiles,
                                                    double* partials) {
    if (op.skip()) return;
    if (!op.begin()) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    double part[Op::kNP] = {};
    if (b < ntiles) tile_mtm_d1p<Op, TX, TT>(g, op, tiles_x, b, part);
    if constexpr (Op::kReduce) deposit<TX / 2, Op::kNP>(part, partials, b);
}

// ---------------------------------------------------------------------------
// Marching variant of the pair sweep (the bare FP64 product, d = 1, nx even).
//
// Each wavefront owns 128 x-sites, as in tile_mtm_d1p, but covers TS
// consecutive slices, taking them in "stages": stage j holds the input row
// of slice s0-1+j (j = 0 .. h+1) and the A row of the same slice (j >= 1).
// Stage j gives y on slice s0-1+j and, from stage 2 on, z on slice s0+j-2;
// the loads of stage j+PF are issued before stage j is consumed.  Over TS
// slices a wavefront reads TS+2 input rows and TS+1 A rows through L1
// instead of 2 and 1.5 per slice for the two-slice tile, and its stores
// overlap the loads of later stages.
template <class Op, int TX, int TS, int PF>
__device__ __forceinline__ void tile_mtm_d1m(const Geom& g, const Op& op, int tiles_x, int b,
                                             double (&part)[Op::kNP]) {
    static_assert(TX % 128 == 0, "tile width is whole pair wavefronts");
    using Center = typename Op::center_t;
    const int nx = g.nx, nt = g.nt;
    const int tx = b % tiles_x, tt = b / tiles_x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave >= TX / 128) return;
    const int n0 = tx * TX + 128 * wave;
    const int w = min(128, nx - n0);
    if (w <= 0) return;
    const int np = w >> 1;
    const int s0 = tt * TS, h = min(TS, nt - s0);
    const double kappa = g.kappa;
    const bool own = lane < np;
    const int site = n0 + 2 * (own ? lane : np - 1);
    const bool solo = np == 1;
    const bool left = lane == 0, right = lane == (solo ? 1 : np - 1);
    const bool edge = left || right;
    const int h1 = wrap1(left ? n0 - 1 : n0 + w, nx);
    const int h2 = wrap1(left ? n0 - 2 : n0 + w + 1, nx);

    D2 xv[TS + 2], av[TS + 2];
    double x1[TS + 2], x2[TS + 2], a1[TS + 2];
    Center cen[TS + 2][2];
    auto load = [&](int j) {
        const int sl = wrap1(s0 - 1 + j, nt);
        const int row = sl * nx;
        if (j >= 1 && j <= h)
            xv[j] = op.in_center2(row + site, cen[j][0], cen[j][1]);
        else
            xv[j] = op.in2(row + site);
        if (j >= 1) av[j] = op.link2(row + site, sl);
        if (edge) {
            x1[j] = op_in(op, row + h1);
            x2[j] = op_in(op, row + h2);
            if (j >= 1) a1[j] = op_link(op, row + h1, sl);
        }
    };
#pragma unroll
    for (int j = 0; j < PF && j < TS + 2; ++j)
        if (j <= h + 1) load(j);
    D2 y_prev{0.0, 0.0};
    double yh_prev = 0.0;
#pragma unroll
    for (int j = 0; j < TS + 2; ++j) {
        if (j + PF < TS + 2 && j + PF <= h + 1) load(j + PF);
        if (j == 0 || j > h + 1) continue;
        const D2 xc = xv[j];
        double xm = lane_up(xc.b), xp = lane_down(xc.a);
        if (left) xm = x1[j];
        if (right) xp = x1[j];
        if (solo) {
            const double xr = lane_down(x1[j]);
            if (left) xp = xr;
        }
        D2 y;
        y.a = xc.a - kappa * (xm + xc.b) + av[j].a * xv[j - 1].a;
        y.b = xc.b - kappa * (xc.a + xp) + av[j].b * xv[j - 1].b;
        double yh = 0.0;
        if (edge) yh = x1[j] - kappa * (x2[j] + (left ? xc.a : xc.b)) + a1[j] * x1[j - 1];
        if (j >= 2) {
            double ym = lane_up(y_prev.b), yp = lane_down(y_prev.a);
            if (left) ym = yh_prev;
            if (right) yp = yh_prev;
            if (solo) {
                const double yr = lane_down(yh_prev);
                if (left) yp = yr;
            }
            D2 zv;
            zv.a = y_prev.a - kappa * (ym + y_prev.b) + av[j].a * y.a;
            zv.b = y_prev.b - kappa * (y_prev.a + yp) + av[j].b * y.b;
            if (own)
                op.out2((s0 + j - 2) * nx + site, zv, xv[j - 1], cen[j - 1][0], cen[j - 1][1],
                        part);
        }
        y_prev = y;
        yh_prev = yh;
    }
}

template <class Op, int TX, int TS, int PF>
__global__ __launch_bounds__(TX / 2) void k_mtm_d1m(Geom g, Op op, int tiles_x, int ntiles,
                                                    double* partials) {
    if (op.skip()) return;
    if (!op.begin()) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    double part[Op::kNP] = {};
    if (b < ntiles) tile_mtm_d1m<Op, TX, TS, PF>(g, op, tiles_x, b, part);
    if constexpr (Op::kReduce) deposit<TX / 2, Op::kNP>(part, partials, b);
}

// Whether an op takes the marching d = 1 tile (kMarch, default false): ops
// whose output is not read again soon (the bare product).
template <class Op, class = void>
struct op_marches : std::false_type {};
template <class Op>
struct op_marches<Op, std::void_t<decltype(Op::kMarch)>> : std::bool_constant<Op::kMarch> {};

// ---------------------------------------------------------------------------
// Fused Q = M^T M sweep for d = 3, nx = NX.
//
// A block of BLOCK lanes owns a tile of whole x rows (NX sites) times TY
// y-rows times TZ z-planes and marches over a chunk of consecutive time
// slices.  Step s (z emitted on slice s):
//   1. the input of slice s+1, loaded one step earlier, goes into LDS (X) on
//      the tile plus a two-site halo in y and z (x is periodic inside a row,
//      so rows need no halo), and the loads of slice s+2 are issued;
//   2. y_{s+1} = W x_{s+1} + A_{s+1} x_s is formed in registers on the tile
//      and on its one-site halo;
//   3. z_s = W y_s + A_{s+1} y_{s+1} is formed on the tile, with y_s from
//      LDS (Y) and y_{s+1} from the lane's registers, and handed to the op;
//   4. y_{s+1} replaces y_s in Y.
// Two barriers per step.  The tile's PZ = NX*TY*TZ sites are owned by fixed
// lanes (site q by lane q mod BLOCK), which keep their input value and op
// state in registers from the load of slice s+1 to the output of slice s+1,
// so the op's output is stores only.  The loads of a slice are issued a step
// before it is staged and stay in flight while the slice before it is
// computed: a barrier on gfx950 waits for LDS traffic only, not for
// outstanding global loads.
template <int NX, int TY, int TZ>
constexpr int d3_lds_elems() {
    // X, Y and one spare element that lanes without a halo position write
    // to, so that every LDS write is unconditional (no divergent branch in
    // the march, whose join would make the compiler wait for all
    // outstanding memory operations, stores included).
    return NX * (TY + 4) * (TZ + 4) + NX * (TY + 2) * (TZ + 2) + 1;
}

// One tile b of the sweep (block of BLOCK lanes); adds this lane's share of
// the op's sums to part.  lds: d3_lds_elems<NX, TY, TZ>() elements.
// TCU > 0: every block marches exactly TCU slices (the caller guarantees
// tc == TCU and nt % TCU == 0), and the march is unrolled completely, so
// that no register holding a load in flight has to be copied where the loop
// would close.
template <class Op, int NX, int TY, int TZ, int BLOCK, int PD = 1, int TCU = 0>
__device__ __forceinline__ void tile_mtm_d3(const Geom& g, const Op& op, int tiles_y,
                                            int tiles_z, int tc, int b,
                                            typename Op::acc_t* lds,
                                            double (&part)[Op::kNP]) {
    static_assert(PD == 1 || PD == 2, "prefetch depth 1 or 2 slices");
    static_assert(TCU == 0 || TCU >= PD, "an unrolled march covers the prefetch depth");
    using Acc = typename Op::acc_t;
    using Center = typename Op::center_t;
    using Raw = typename Op::raw_t;
    using CRaw = typename Op::craw_t;
    using LRaw = typename Op::lraw_t;
    constexpr int XY = TY + 4, XZ = TZ + 4, YY = TY + 2, YZ = TZ + 2;
    constexpr int PX = NX * XY * XZ, PZ = NX * TY * TZ;
    static_assert((NX & (NX - 1)) == 0, "NX must be a power of two");
    static_assert(PZ % BLOCK == 0, "tile must be whole multiples of the block");
    constexpr int NC = PZ / BLOCK;
    // Halo rows (y, z pairs outside the tile) of the X and Y stages.
    constexpr int HRX = XY * XZ - TY * TZ, HRY = YY * YZ - TY * TZ;
    constexpr int NHX = (NX * HRX + BLOCK - 1) / BLOCK, NHY = (NX * HRY + BLOCK - 1) / BLOCK;
    Acc* X = lds;
    Acc* Y = lds + PX;
    constexpr int kSink = PX + NX * YY * YZ;  // spare element, index into lds
    const int nt = g.nt, vs = g.vs;
    const int iy = b % tiles_y;
    b /= tiles_y;
    const int iz = b % tiles_z;
    const int ch = b / tiles_z;
    const int y0 = iy * TY, z0 = iz * TZ, s0 = ch * tc;
    const int h = TCU > 0 ? TCU : min(tc, nt - s0);
    const int t = threadIdx.x;
    const Acc kappa = (Acc)g.kappa;

    // Owned tile sites: spatial index, x coordinate, LDS index in X and Y.
    int cn[NC], cx[NC], cxi[NC], cyi[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const int q = t + BLOCK * k;
        const int x = q % NX, r = q / NX, ty = r % TY, tz = r / TY;
        cx[k] = x;
        cn[k] = x + NX * ((y0 + ty) + NX * (z0 + tz));
        cxi[k] = x + NX * ((ty + 2) + XY * (tz + 2));
        cyi[k] = x + NX * ((ty + 1) + YY * (tz + 1));
    }
    // X halo positions of this lane: spatial index and X index.  Lanes past
    // the end repeat the last position (loads stay unconditional; the LDS
    // write is skipped).
    int hxs[NHX], hxi[NHX];
    bool hxo[NHX];
#pragma unroll
    for (int k = 0; k < NHX; ++k) {
        int q = t + BLOCK * k;
        hxo[k] = q < NX * HRX;
        if (!hxo[k]) q = NX * HRX - 1;
        const int x = q % NX, hr = q / NX;
        int yx, zx;
        if (hr < 2 * XY) {
            zx = hr / XY;
            yx = hr % XY;
        } else if (hr < 4 * XY) {
            zx = TZ + 2 + (hr - 2 * XY) / XY;
            yx = (hr - 2 * XY) % XY;
        } else {
            const int r = hr - 4 * XY, c = r % 4;
            zx = 2 + r / 4;
            yx = c < 2 ? c : TY + c;
        }
        hxi[k] = hxo[k] ? x + NX * (yx + XY * zx) : kSink;
        hxs[k] = x + NX * (wrap1(y0 - 2 + yx, NX) + NX * wrap1(z0 - 2 + zx, NX));
    }
    // Y halo positions: spatial index, Y index, X index of the same site.
    int hys[NHY], hyi[NHY], hyx[NHY], hyc[NHY];
    bool hyo[NHY];
#pragma unroll
    for (int k = 0; k < NHY; ++k) {
        int q = t + BLOCK * k;
        hyo[k] = q < NX * HRY;
        if (!hyo[k]) q = NX * HRY - 1;
        const int x = q % NX, hr = q / NX;
        int yy, zz;
        if (hr < 2 * YY) {
            zz = hr < YY ? 0 : TZ + 1;
            yy = hr % YY;
        } else {
            const int r = hr - 2 * YY;
            zz = 1 + r / 2;
            yy = (r & 1) ? TY + 1 : 0;
        }
        hyc[k] = x;
        hyi[k] = hyo[k] ? x + NX * (yy + YY * zz) : kSink - PX;
        hyx[k] = x + NX * ((yy + 1) + XY * (zz + 1));
        hys[k] = x + NX * (wrap1(y0 - 1 + yy, NX) + NX * wrap1(z0 - 1 + zz, NX));
    }
    // W applied to X around X index j (x coordinate x).
    auto wx = [&](int x, int j) {
        const int xm = (x - 1) & (NX - 1), xp = (x + 1) & (NX - 1);
        return X[j] - kappa * (X[j - x + xm] + X[j - x + xp] + X[j - NX] + X[j + NX] +
                               X[j - NX * XY] + X[j + NX * XY]);
    };

    // Loads of one slice, issued PD steps before they are used (PD = 2: two
    // buffers, alternating by step parity).
    struct Pre {
        CRaw pc[NC];
        LRaw pa[NC];
        Raw ph[NHX];
        LRaw pah[NHY];
    };
    Pre pre0, pre1;
    auto prefetch = [&](Pre& P, int sl) {
        const int off = vs * sl;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            P.pc[k] = op.load_c(cn[k] + off);
            P.pa[k] = op.lraw(cn[k] + off);
        }
#pragma unroll
        for (int k = 0; k < NHX; ++k) P.ph[k] = op.load_h(hxs[k] + off);
#pragma unroll
        for (int k = 0; k < NHY; ++k) P.pah[k] = op.lraw(hys[k] + off);
    };
    // x_s, x_{s+1} and op state at the owned sites; x_s at the Y-halo
    // positions; A_{s+1} at both.
    Acc xs_c[NC], xn_c[NC], an_c[NC], xs_h[NHY], an_h[NHY];
    Center cs_c[NC], cn_c[NC];
    // The prefetched slice sl into X, xn_c / cn_c and an_c / an_h.
    auto stage = [&](const Pre& P, int sl) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            xn_c[k] = op.val_c(P.pc[k], cn_c[k]);
            an_c[k] = op.lval(P.pa[k], sl);
            X[cxi[k]] = xn_c[k];
        }
#pragma unroll
        for (int k = 0; k < NHX; ++k) X[hxi[k]] = op.val_h(P.ph[k]);
#pragma unroll
        for (int k = 0; k < NHY; ++k) an_h[k] = op.lval(P.pah[k], sl);
    };

    // Prologue: x_{s0-1} at the owned and Y-halo positions, slice s0 into X,
    // y_{s0} into Y, slice s0+1 in flight.
    {
        const int offm = vs * wrap1(s0 - 1, nt);
#pragma unroll
        for (int k = 0; k < NC; ++k) xs_c[k] = op_in(op, cn[k] + offm);
#pragma unroll
        for (int k = 0; k < NHY; ++k) xs_h[k] = op_in(op, hys[k] + offm);
        prefetch(pre0, s0);
        stage(pre0, s0);
        prefetch(pre0, wrap1(s0 + 1, nt));
        if (PD == 2 && h > 1) prefetch(pre1, wrap1(s0 + 2, nt));
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NC; ++k) Y[cyi[k]] = wx(cx[k], cxi[k]) + an_c[k] * xs_c[k];
#pragma unroll
        for (int k = 0; k < NHY; ++k) {
            Y[hyi[k]] = wx(hyc[k], hyx[k]) + an_h[k] * xs_h[k];
            xs_h[k] = X[hyx[k]];
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            xs_c[k] = xn_c[k];
            cs_c[k] = cn_c[k];
        }
        __syncthreads();
    }

    // Step r emits z on slice s0 + r; the slice it stages was loaded PD
    // steps earlier into the buffer of parity r (PD = 2) or the one buffer.
    auto step = [&](int r, Pre& P, bool more) {
        const int s = s0 + r;
        stage(P, wrap1(s + 1, nt));
        if (more) prefetch(P, wrap1(s + 1 + PD, nt));
        __syncthreads();
        Acc yo[NC], yh[NHY];
#pragma unroll
        for (int k = 0; k < NC; ++k) yo[k] = wx(cx[k], cxi[k]) + an_c[k] * xs_c[k];
#pragma unroll
        for (int k = 0; k < NHY; ++k) {
            yh[k] = wx(hyc[k], hyx[k]) + an_h[k] * xs_h[k];
            xs_h[k] = X[hyx[k]];
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int j = cyi[k], x = cx[k];
            const int xm = (x - 1) & (NX - 1), xp = (x + 1) & (NX - 1);
            const Acc zv = Y[j] - kappa * (Y[j - x + xm] + Y[j - x + xp] + Y[j - NX] +
                                           Y[j + NX] + Y[j - NX * YY] + Y[j + NX * YY]) +
                           an_c[k] * yo[k];
            op.out(cn[k] + vs * s, zv, xs_c[k], cs_c[k], part);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            Y[cyi[k]] = yo[k];
            xs_c[k] = xn_c[k];
            cs_c[k] = cn_c[k];
        }
#pragma unroll
        for (int k = 0; k < NHY; ++k) Y[hyi[k]] = yh[k];
    };
    if constexpr (TCU > 0) {
#pragma unroll
        for (int r = 0; r < TCU; ++r) step(r, (PD == 2 && (r & 1)) ? pre1 : pre0, r + PD < TCU);
    } else if constexpr (PD == 1) {
        for (int r = 0; r < h; ++r) step(r, pre0, r + 1 < h);
    } else {
        for (int r = 0; r < h; r += 2) {
            step(r, pre0, r + 2 < h);
            if (r + 1 < h) step(r + 1, pre1, r + 3 < h);
        }
    }
}

template <class Op, int NX, int TY, int TZ, int BLOCK, int PD = 1, int TCU = 0>
__global__ __launch_bounds__(BLOCK) void k_mtm_d3(Geom g, Op op, int tiles_y, int tiles_z,
                                                  int tc, double* partials) {
    using Acc = typename Op::acc_t;
    __shared__ Acc lds[d3_lds_elems<NX, TY, TZ>()];
    if (op.skip()) return;
    if (!op.begin()) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    double part[Op::kNP] = {};
    tile_mtm_d3<Op, NX, TY, TZ, BLOCK, PD, TCU>(g, op, tiles_y, tiles_z, tc, b, lds, part);
    if constexpr (Op::kReduce) deposit<BLOCK, Op::kNP>(part, partials, b);
}

// ---------------------------------------------------------------------------
// Generic two-pass path for any d and any extents: y = M in (pass 1, into a
// scratch vector), then z = M^T y with the op's epilogue (pass 2).

template <class Op>
__device__ inline typename Op::acc_t gen_M_at(const Geom& g, const Op& op, int i) {
    using Acc = typename Op::acc_t;
    const int s = fdiv(i, g.fvs), n = i - s * g.vs;
    Acc hop = 0;
    int stride = 1, rest = n;
    for (int j = 0; j < g.d; ++j) {
        const int q = fdiv(rest, g.fnx);
        const int c = rest - q * g.nx;
        rest = q;
        const int cp = c + 1 == g.nx ? 0 : c + 1;
        const int cm = c == 0 ? g.nx - 1 : c - 1;
        hop += op_in(op, i + (cp - c) * stride) + op_in(op, i + (cm - c) * stride);
        stride *= g.nx;
    }
    const int sm = s == 0 ? g.nt - 1 : s - 1;
    return op_in(op, i) - (Acc)g.kappa * hop + op_link(op, i, s) * op_in(op, n + sm * g.vs);
}

template <class Op>
__global__ __launch_bounds__(256) void k_gen_pass1(Geom g, Op op, typename Op::acc_t* y) {
    if (op.skip()) return;
    if (!op.begin()) return;
    const int i = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (i < g.V) y[i] = gen_M_at(g, op, i);
}

template <class Op>
__global__ __launch_bounds__(256) void k_gen_pass2(Geom g, Op op,
                                                   const typename Op::acc_t* y,
                                                   double* partials) {
    using Acc = typename Op::acc_t;
    if (op.skip()) return;
    if (!op.begin()) return;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int i = tile * 256 + threadIdx.x;
    double part[Op::kNP] = {};
    if (i < g.V) {
        const int s = fdiv(i, g.fvs), n = i - s * g.vs;
        Acc hop = 0;
        int stride = 1, rest = n;
        for (int j = 0; j < g.d; ++j) {
            const int q = fdiv(rest, g.fnx);
            const int c = rest - q * g.nx;
            rest = q;
            const int cp = c + 1 == g.nx ? 0 : c + 1;
            const int cm = c == 0 ? g.nx - 1 : c - 1;
            hop += y[i + (cp - c) * stride] + y[i + (cm - c) * stride];
            stride *= g.nx;
        }
        const int sp = s == g.nt - 1 ? 0 : s + 1;
        const int ip = n + sp * g.vs;
        const Acc zv = y[i] - (Acc)g.kappa * hop + op_link(op, ip, sp) * y[ip];
        typename Op::center_t c;
        const Acc v = op_in_center(op, i, c);
        op.out(i, zv, v, c, part);
    }
    if constexpr (Op::kReduce) deposit<256, Op::kNP>(part, partials, tile);
}

// ---------------------------------------------------------------------------
// Single M or M^T (hub_apply_M): one lane per site, neighbours through L1/L2.
template <class Acc, class Vec, class Lnk, bool TRANSPOSE>
__global__ __launch_bounds__(256) void k_apply_M(Geom g, Lnk lk, const Vec* x, Vec* y) {
    const int i = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (i >= g.V) return;
    const int s = fdiv(i, g.fvs), n = i - s * g.vs;
    Acc hop = 0;
    int stride = 1, rest = n;
    for (int j = 0; j < g.d; ++j) {
        const int q = fdiv(rest, g.fnx);
        const int c = rest - q * g.nx;
        rest = q;
        const int cp = c + 1 == g.nx ? 0 : c + 1;
        const int cm = c == 0 ? g.nx - 1 : c - 1;
        hop += (Acc)x[i + (cp - c) * stride] + (Acc)x[i + (cm - c) * stride];
        stride *= g.nx;
    }
    Acc v = (Acc)x[i] - (Acc)g.kappa * hop;
    if (!TRANSPOSE) {
        const int sm = s == 0 ? g.nt - 1 : s - 1;
        v += (Acc)lk.val(lk.raw(i), s) * (Acc)x[n + sm * g.vs];
    } else {
        const int sp = s == g.nt - 1 ? 0 : s + 1;
        const int ip = n + sp * g.vs;
        v += (Acc)lk.val(lk.raw(ip), sp) * (Acc)x[ip];
    }
    y[i] = (Vec)v;
}

// The same in FP64 for even nx, two x-adjacent sites per lane with 16-byte
// accesses; each site's arithmetic is that of k_apply_M, in the same order.
template <bool TRANSPOSE, int D>
__global__ __launch_bounds__(256) void k_apply_M2(Geom g, const double* __restrict__ A,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ y) {
    const int i = 2 * (xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x);  // first site of the pair
    if (i >= g.V) return;
    const int s = fdiv(i, g.fvs), n = i - s * g.vs;
    const D2 xc = ld2(x + i);
    double hop_a = 0.0, hop_b = 0.0;
    int rest = n, stride = 1;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const int q = j + 1 < D ? fdiv(rest, g.fnx) : 0;
        const int cj = j + 1 < D ? rest - q * g.nx : rest;
        if (j == 0) {
            // cj is even: a = cj, b = cj + 1 < nx
            const double left_a = x[i + (cj == 0 ? g.nx - 1 : -1)];
            const double right_b = x[i + (cj + 2 == g.nx ? 2 - g.nx : 2)];
            hop_a += xc.b + left_a;
            hop_b += right_b + xc.a;
        } else {
            const int cpj = cj + 1 == g.nx ? 0 : cj + 1;
            const int cmj = cj == 0 ? g.nx - 1 : cj - 1;
            const D2 pl = ld2(x + i + (cpj - cj) * stride);
            const D2 mi = ld2(x + i + (cmj - cj) * stride);
            hop_a += pl.a + mi.a;
            hop_b += pl.b + mi.b;
        }
        stride *= g.nx;
        rest = q;
    }
    double va = xc.a - g.kappa * hop_a;
    double vb = xc.b - g.kappa * hop_b;
    if (!TRANSPOSE) {
        const int sm = s == 0 ? g.nt - 1 : s - 1;
        const D2 a = ld2(A + i), xm = ld2(x + n + sm * g.vs);
        va += a.a * xm.a;
        vb += a.b * xm.b;
    } else {
        const int sp = s == g.nt - 1 ? 0 : s + 1;
        const int ip = n + sp * g.vs;
        const D2 a = ld2(A + ip), xp = ld2(x + ip);
        va += a.a * xp.a;
        vb += a.b * xp.b;
    }
    st2(y + i, va, vb);
}

}  // namespace hub
