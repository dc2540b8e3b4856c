// Conjugate gradient on Q = M^T M (Sec. 4.1) for small lattices, in one
// workgroup.  Up to kSmallSitesMax sites the whole solve fits one block: the
// direction vector, M p and the links live in LDS, every other vector in the
// lanes' registers, and an iteration is two stencil passes and two block
// sums separated by barriers instead of three kernel launches.  The method
// is the FP64 CG of the multi-kernel solver: x0 = 0, convergence decided on
// the FP64 true residual |phi - Q x| / |phi| <= tol, and when the iterated
// residual meets tol but the true one does not, the iteration continues from
// the true residual keeping p.
#include <cmath>

#include "internal.h"

namespace hub {

namespace {

constexpr int kSB = 512;                   // lanes of the block (8 waves: measured faster than 4 or 16)
constexpr int kNPT = 4;                    // sites per lane
constexpr int kSmallSitesMax = kSB * kNPT;

struct SmallResult {
    int32_t iters;
    int32_t done;         // kDone* of common.h
    int32_t recomputes;   // true-residual recomputes
    int32_t pad;
    double rho_true;      // |phi - Q x|^2 of the returned x
    double phi2;
};

// Sums over the block in a fixed order (wave sums, then the waves' sums in
// wave order), the same value in every lane.  Consecutive sums alternate
// between two LDS slots, so one barrier per sum suffices: a slot is written
// again only after every lane has passed the other slot's barrier, that is
// after it has read this slot.  Every lane makes the same sequence of calls.
struct BlockSum {
    double* red;  // 2 * kSB / 64 doubles of LDS
    int turn;
    __device__ double operator()(double v) {
        double* r = red + turn * (kSB / 64);
        turn ^= 1;
        v = wave_sum(v);
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        if (lane == 0) r[w] = v;
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kSB / 64; ++k) s += r[k];
        return s;
    }
};

struct Site {
    int i;        // linear index (0 for a lane past the end)
    bool ok;      // i < V
    int nb[6];    // spatial neighbours +-e_j, j < d
    int im, ip;   // same n on slice s-1 and s+1 (periodic in the index)
};

__device__ inline Site make_site(const Geom& g, int i) {
    Site S;
    S.ok = i < g.V;
    S.i = S.ok ? i : 0;
    const int n = S.i % g.vs, s = S.i / g.vs;
    int stride = 1;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (j < g.d) {
            const int c = (n / stride) % g.nx;
            const int cp = c + 1 == g.nx ? 0 : c + 1;
            const int cm = c == 0 ? g.nx - 1 : c - 1;
            S.nb[2 * j] = S.i + (cp - c) * stride;
            S.nb[2 * j + 1] = S.i + (cm - c) * stride;
            stride *= g.nx;
        } else {
            S.nb[2 * j] = S.nb[2 * j + 1] = S.i;
        }
    }
    S.im = n + g.vs * (s == 0 ? g.nt - 1 : s - 1);
    S.ip = n + g.vs * (s + 1 == g.nt ? 0 : s + 1);
    return S;
}

// (M v)_i = v_i - kappa sum_j (v_{i+e_j} + v_{i-e_j}) + A_i v_{i, s-1}
__device__ inline double apply_M_at(const Geom& g, const Site& S, const double* v,
                                    const double* A) {
    double hop = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j)
        if (j < 2 * g.d) hop += v[S.nb[j]];
    return v[S.i] - g.kappa * hop + A[S.i] * v[S.im];
}

// (M^T v)_i = v_i - kappa sum_j (v_{i+e_j} + v_{i-e_j}) + A_{i, s+1} v_{i, s+1}
__device__ inline double apply_Mt_at(const Geom& g, const Site& S, const double* v,
                                     const double* A) {
    double hop = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j)
        if (j < 2 * g.d) hop += v[S.nb[j]];
    return v[S.i] - g.kappa * hop + A[S.ip] * v[S.ip];
}

__global__ __launch_bounds__(kSB) void k_cg_small(Geom g, const double* __restrict__ A,
                                                  const double* __restrict__ phi,
                                                  double* __restrict__ x_out, double tol2,
                                                  int max_iter, SmallResult* res) {
    __shared__ double P[kSmallSitesMax], Y[kSmallSitesMax], AL[kSmallSitesMax];
    __shared__ double red[2 * (kSB / 64)];
    BlockSum sum_block{red, 0};
    Site S[kNPT];
    double x[kNPT], r[kNPT], p[kNPT], f[kNPT];
#pragma unroll
    for (int k = 0; k < kNPT; ++k) {
        S[k] = make_site(g, threadIdx.x + kSB * k);
        f[k] = S[k].ok ? phi[S[k].i] : 0.0;
        if (S[k].ok) AL[S[k].i] = A[S[k].i];
        x[k] = 0.0;
        r[k] = f[k];
        p[k] = f[k];
    }
    // |phi - Q v|^2 with v from the lanes' registers; r = phi - Q v.
    auto true_residual = [&](const double (&v)[kNPT]) {
#pragma unroll
        for (int k = 0; k < kNPT; ++k)
            if (S[k].ok) P[S[k].i] = v[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kNPT; ++k)
            if (S[k].ok) Y[S[k].i] = apply_M_at(g, S[k], P, AL);
        __syncthreads();
        double part = 0.0;
#pragma unroll
        for (int k = 0; k < kNPT; ++k) {
            if (S[k].ok) {
                const double d = f[k] - apply_Mt_at(g, S[k], Y, AL);
                r[k] = d;
                part += d * d;
            }
        }
        return sum_block(part);
    };

    double part = 0.0;
#pragma unroll
    for (int k = 0; k < kNPT; ++k) part += f[k] * f[k];
    const double phi2 = sum_block(part);
    double rho = phi2, rho_true = phi2;
    int done = !isfinite(phi2) ? kDoneBreakdown : (phi2 == 0.0 ? kDoneConverged : kRunning);
    int it = 0, recomputes = 0;
    while (done == kRunning) {
        // q = Q p, p.q
#pragma unroll
        for (int k = 0; k < kNPT; ++k)
            if (S[k].ok) P[S[k].i] = p[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kNPT; ++k)
            if (S[k].ok) Y[S[k].i] = apply_M_at(g, S[k], P, AL);
        __syncthreads();
        double q[kNPT];
        part = 0.0;
#pragma unroll
        for (int k = 0; k < kNPT; ++k) {
            q[k] = S[k].ok ? apply_Mt_at(g, S[k], Y, AL) : 0.0;
            part += p[k] * q[k];
        }
        const double pq = sum_block(part);
        if (!(pq > 0.0) || !isfinite(pq)) {
            done = kDoneBreakdown;
            break;
        }
        // x += alpha p, r -= alpha q, r.r; a step that overflows is not
        // taken, so a breakdown returns the last finite iterate.
        const double alpha = rho / pq;
        if (!isfinite(alpha)) {
            done = kDoneBreakdown;
            break;
        }
        double xn[kNPT], rn[kNPT];
        part = 0.0;
#pragma unroll
        for (int k = 0; k < kNPT; ++k) {
            xn[k] = x[k] + alpha * p[k];
            rn[k] = r[k] - alpha * q[k];
            part += rn[k] * rn[k];
        }
        double rho_new = sum_block(part);
        if (!isfinite(rho_new)) {
            done = kDoneBreakdown;
            break;
        }
        ++it;
#pragma unroll
        for (int k = 0; k < kNPT; ++k) {
            x[k] = xn[k];
            r[k] = rn[k];
        }
        if (rho_new <= tol2 * phi2) {
            ++recomputes;
            rho_true = true_residual(x);
            if (rho_true <= tol2 * phi2) {
                done = kDoneConverged;
                break;
            }
            rho_new = rho_true;  // continue from the true residual, keeping p
        }
        if (it >= max_iter) {
            done = kDoneMaxIter;
            break;
        }
        const double beta = rho_new / rho;
        rho = rho_new;
#pragma unroll
        for (int k = 0; k < kNPT; ++k) p[k] = r[k] + beta * p[k];
    }
    if (done != kDoneConverged) rho_true = true_residual(x);
#pragma unroll
    for (int k = 0; k < kNPT; ++k)
        if (S[k].ok) x_out[S[k].i] = x[k];
    if (threadIdx.x == 0) {
        res->iters = it;
        res->done = done;
        res->recomputes = recomputes;
        res->rho_true = rho_true;
        res->phi2 = phi2;
    }
}

}  // namespace

bool cg_small_fits(const Geom& g) { return g.V <= kSmallSitesMax; }

hub_status cg_solve_small(const Geom& g, const double* sigma, const double* phi, double* x,
                          const hub_cg_opts& o, hub_cg_stats* out, hipStream_t st) {
    const size_t bytes = (8 * (size_t)g.V + 255) / 256 * 256 + 256;
    char* ws = nullptr;
    const hub_status wr = solver_workspace(bytes, &ws);
    if (wr != HUB_OK) return wr;
    double* A = (double*)ws;
    SmallResult* dres = (SmallResult*)(ws + bytes - 256);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    SmallResult h{};
    float ms = 0.0f;
    hub_status r = launch_links(g, sigma, A, HUB_F64, st);
    auto step = [&](hipError_t e) {
        if (r == HUB_OK && e != hipSuccess)
            r = set_error(HUB_E_DEVICE, "hub_cg_solve: %s", hipGetErrorString(e));
    };
    step(hipEventCreate(&t0));
    step(hipEventCreate(&t1));
    if (r == HUB_OK) {
        step(hipEventRecord(t0, st));
        k_cg_small<<<1, kSB, 0, st>>>(g, A, phi, x, o.tol * o.tol, o.max_iter, dres);
        step(hipGetLastError());
        step(hipEventRecord(t1, st));
        step(hipMemcpyAsync(&h, dres, sizeof(h), hipMemcpyDeviceToHost, st));
        step(hipStreamSynchronize(st));
        if (r == HUB_OK) step(hipEventElapsedTime(&ms, t0, t1));
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    step(hipStreamSynchronize(st));  // the workspace is free again once st has drained
    if (r != HUB_OK) return r;
    hub_cg_stats stats{};
    stats.iters = h.iters;
    stats.reliable_updates = h.recomputes;
    stats.true_rel_resid = h.phi2 > 0 ? std::sqrt(h.rho_true / h.phi2) : 0.0;
    stats.ms = ms;
    stats.status = h.done == kDoneConverged ? HUB_OK : HUB_E_NOCONV;
    if (out) *out = stats;
    if (stats.status != HUB_OK)
        return set_error(HUB_E_NOCONV,
                         "CG did not converge: %d iterations, true relative residual %.3e%s",
                         h.iters, stats.true_rel_resid,
                         h.done == kDoneBreakdown ? " (breakdown)" : "");
    return HUB_OK;
}

}  // namespace hub
