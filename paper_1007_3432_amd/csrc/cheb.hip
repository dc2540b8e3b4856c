// Chebyshev polynomial preconditioner (Sec. 4.2, Eqs. (13)-(15)).
//
// P(l) = c_{2n} prod_{k=1}^{2n} (l - z_{2n,k}) approximates 1/l on (eps, 1]
// for l an eigenvalue of Q / scale.  The roots come in conjugate pairs
// (z_{2n,2n+1-k} = conj z_{2n,k}), so P is applied as n real quadratic
// factors in Q, each two fused sweeps (w = Q v; v' = c2 Q w + c1 w + c0 v).
// Each factor is normalised to 1 at l = (1 + eps)/2, where P = 2/(1 + eps).
//
// Order of the factors.  Each sweep adds rounding error of relative size u
// (about 1e-16) in every eigen-direction of Q; the factors still to come
// multiply the error in direction l by their product S_j(l).  The error of the
// whole product is therefore about u max_j [max_l |prefix_j(l)|] [max_l S_j(l)]:
// for the order k = 1 .. n this reaches 1e41 at n = 48 (eps = 0.01), for an
// alternating order 1, n, 2, n-1, ... still 1e18.  The order used here is
// built greedily: at each step the factor that minimises
// max(1, max_l prefix) * max_l suffix on a grid over [0, 1] comes next; in a
// dense emulation its error stays at 1e-12 or below up to n = 128 for
// eps >= 1e-5 (2e-11 at n = 256), against 1e+29 for the alternating order at
// n = 128.  The order is computed once per (n, eps) and cached.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "cheb.h"

namespace hub {

namespace {

// Greedy factor order for (n, eps), n <= kMaxChebN, in k = 1 .. n.  Computed
// without heap allocation (fixed static work arrays under a lock) and kept
// in a fixed-size table, so that every caller -- including the
// no-allocation entry point -- gets it without allocating.
constexpr int kMaxChebN = 256;
constexpr int kGrid = 1024;
constexpr int kOrderCache = 64;

struct OrderEntry {
    int n;
    double eps;
    uint16_t order[kMaxChebN];
};

std::mutex g_order_mu;
OrderEntry g_orders[kOrderCache];
int g_orders_used = 0, g_orders_next = 0;
double g_lf[kMaxChebN * kGrid];  // log f_k(lambda_i), under g_order_mu
double g_lam[kGrid], g_total[kGrid], g_pre[kGrid];

void factor_order(int n, double eps, uint16_t* order) {
    std::lock_guard<std::mutex> lk(g_order_mu);
    for (int e = 0; e < g_orders_used; ++e)
        if (g_orders[e].n == n && g_orders[e].eps == eps) {
            std::copy(g_orders[e].order, g_orders[e].order + n, order);
            return;
        }
    const double pi = 3.14159265358979323846;
    const double h = 0.5 * (1.0 + eps);
    // Grid: 512 points uniform on [0, 1] and 512 log-spaced on [eps/64, 1].
    for (int i = 0; i < 512; ++i) g_lam[i] = i / 511.0;
    const double l0 = std::log(eps / 64.0);
    for (int i = 0; i < 512; ++i) g_lam[512 + i] = std::exp(l0 * (1.0 - i / 511.0));
    const int L = kGrid;
    // log f_k(l) of the normalised pair factors, and their sum.
    std::fill(g_total, g_total + L, 0.0);
    for (int k = 1; k <= n; ++k) {
        const double th = 2.0 * pi * k / (2 * n + 1);
        const double a = h * (1.0 - std::cos(th));
        const double bi = std::sqrt(eps) * std::sin(th);
        const double norm = 1.0 / ((h - a) * (h - a) + bi * bi);
        for (int i = 0; i < L; ++i) {
            const double v = std::log(((g_lam[i] - a) * (g_lam[i] - a) + bi * bi) * norm);
            g_lf[(size_t)(k - 1) * L + i] = v;
            g_total[i] += v;
        }
    }
    std::fill(g_pre, g_pre + L, 0.0);
    bool used[kMaxChebN] = {};
    for (int step = 0; step < n; ++step) {
        int best = -1;
        double best_m = 0.0;
        for (int k = 0; k < n; ++k) {
            if (used[k]) continue;
            const double* f = &g_lf[(size_t)k * L];
            double mp = 0.0, ms = -1e300;
            for (int i = 0; i < L; ++i) {
                const double p = g_pre[i] + f[i];
                mp = std::max(mp, p);
                ms = std::max(ms, g_total[i] - p);
            }
            const double m = mp + ms;
            if (best < 0 || m < best_m) {
                best = k;
                best_m = m;
            }
        }
        used[best] = true;
        order[step] = (uint16_t)(best + 1);
        for (int i = 0; i < L; ++i) g_pre[i] += g_lf[(size_t)best * L + i];
    }
    OrderEntry& e = g_orders[g_orders_next];
    g_orders_next = (g_orders_next + 1) % kOrderCache;
    if (g_orders_used < kOrderCache) ++g_orders_used;
    e.n = n;
    e.eps = eps;
    std::copy(order, order + n, e.order);
}

}  // namespace

void cheb_factors(int n, double eps, double scale, ChebFactor* f) {
    const double pi = 3.14159265358979323846;
    const double h = 0.5 * (1.0 + eps);
    uint16_t order[kMaxChebN];
    factor_order(n, eps, order);
    for (int j = 0; j < n; ++j) {
        const int k = order[j];
        const double th = 2.0 * pi * k / (2 * n + 1);
        const double a = h * (1.0 - std::cos(th));       // Re z_{2n,k}
        const double bi = std::sqrt(eps) * std::sin(th);  // -Im z_{2n,k}
        const double norm = 1.0 / ((h - a) * (h - a) + bi * bi);
        ChebFactor& c = f[j];
        c.c2 = norm / (scale * scale);
        c.c1 = -2.0 * a * norm / scale;
        c.c0 = (a * a + bi * bi) * norm;
    }
    // The remaining constant of c_{2n}: 1 / h.
    f[n - 1].c2 /= h;
    f[n - 1].c1 /= h;
    f[n - 1].c0 /= h;
}

std::vector<ChebFactor> cheb_factors(int n, double eps, double scale) {
    std::vector<ChebFactor> f((size_t)n);
    cheb_factors(n, eps, scale, f.data());
    return f;
}

double cheb_default_scale(const Geom& g) {
    // |M| <= 1 + 2 d kappa + max|A| by the triangle inequality over the
    // stencil's terms, max|A| <= exp(dtau mu)(1 + b); |Q| <= |M|^2.
    const double m = 1.0 + 2.0 * g.d * g.kappa + g.lscale * (1.0 + g.b);
    return m * m;
}

hub_status launch_cheb(const Geom& g, const SweepPlan& P, const double* A64, CGScalars* sc,
                       const double* r, double* z, double* w, double* yscratch,
                       double* partials, const ChebFactor* f, int n, bool dot,
                       hipStream_t st) {
    for (int j = 0; j < n; ++j) {
        const double* v = j == 0 ? r : z;
        OpChebW opw{sc, v, w, Link64{A64}};
        hub_status s = launch_q(g, P, opw, yscratch, nullptr, st);
        if (s != HUB_OK) return s;
        if (dot && j == n - 1) {
            OpChebZ<true> opz{sc, w, v, z, r, f[j].c2, f[j].c1, f[j].c0, Link64{A64}};
            s = launch_q(g, P, opz, yscratch, partials, st);
        } else {
            OpChebZ<false> opz{sc, w, v, z, r, f[j].c2, f[j].c1, f[j].c0, Link64{A64}};
            s = launch_q(g, P, opz, yscratch, nullptr, st);
        }
        if (s != HUB_OK) return s;
    }
    return HUB_OK;
}

hub_status cheb_apply(const Geom& g, const double* links, const double* r, double* z,
                      const hub_cheb_opts& c, hipStream_t st) {
    const SweepPlan P = plan_sweep(g, true);
    const double scale = c.scale > 0 ? c.scale : cheb_default_scale(g);
    ChebFactor f[kMaxChebN];
    cheb_factors(c.n, c.eps, scale, f);
    const size_t vb = ((size_t)g.V * 8 + 255) & ~size_t(255);
    char* ws = nullptr;
    const size_t bytes = vb * (P.fused ? 1 : 2);
    if (hipMallocAsync((void**)&ws, bytes, st) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(HUB_E_NOMEM, "hub_apply_cheb: cannot allocate %zu bytes", bytes);
    }
    double* w = (double*)ws;
    double* y = P.fused ? nullptr : (double*)(ws + vb);
    const hub_status s = launch_cheb(g, P, links, nullptr, r, z, w, y, nullptr, f, c.n, false, st);
    const hipError_t e = hipFreeAsync(ws, st);
    if (s != HUB_OK) return s;
    if (e != hipSuccess) return set_error(HUB_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
    return HUB_OK;
}

// ---------------------------------------------------------------------------
// No-allocation variant: the workspace (w, and y for two-pass plans) lives in
// a fixed array of kNoAllocBytes that every GPU running the library holds
// until the process ends.  Host code never passes the array's name to a
// kernel: its device address on the current GPU is looked up once per device
// (hipGetSymbolAddress) and kept in g_scratch_ptr.  All calls on one GPU
// share the array, so calls that overlap in time on one GPU race.  Nothing in
// it must start at zero: every sweep writes its whole output before the next
// one reads it.

static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

hub_status noalloc_scratch(double** out) {
    int dev = 0;
    HUB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(HUB_E_DEVICE, "device ordinal %d beyond the %d supported", dev,
                         kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(HUB_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                             hipGetErrorString(e));
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return HUB_OK;
}

}  // namespace

size_t cheb_noalloc_bytes(const Geom& g) {
    const SweepPlan P = plan_sweep(g, true);
    const size_t vb = ((size_t)g.V * 8 + 255) & ~size_t(255);
    return vb * (P.fused ? 1 : 2);
}

hub_status cheb_apply_noalloc(const Geom& g, const double* links, const double* r, double* z,
                              const hub_cheb_opts& c, hipStream_t st) {
    const size_t need = cheb_noalloc_bytes(g);
    if (need > kNoAllocBytes)
        return set_error(HUB_E_NOMEM,
                         "hub_apply_cheb_noalloc: %d sites need %zu bytes of workspace, the "
                         "fixed array holds %zu",
                         g.V, need, kNoAllocBytes);
    double* ws = nullptr;
    hub_status s = noalloc_scratch(&ws);
    if (s != HUB_OK) return s;
    const SweepPlan P = plan_sweep(g, true);
    const double scale = c.scale > 0 ? c.scale : cheb_default_scale(g);
    ChebFactor f[kMaxChebN];
    cheb_factors(c.n, c.eps, scale, f);
    const size_t vb = ((size_t)g.V * 8 + 255) & ~size_t(255);
    double* w = ws;
    double* y = P.fused ? nullptr : (double*)((char*)ws + vb);
    return launch_cheb(g, P, links, nullptr, r, z, w, y, nullptr, f, c.n, false, st);
}

}  // namespace hub
