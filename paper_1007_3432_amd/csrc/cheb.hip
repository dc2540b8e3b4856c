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
#include <map>
#include <mutex>
#include <vector>

#include "cheb.h"

namespace hub {

namespace {

// Greedy factor order for (n, eps) in k = 1 .. n, cached per process.
std::vector<int> factor_order(int n, double eps) {
    static std::mutex mu;
    static std::map<std::pair<int, double>, std::vector<int>> cache;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find({n, eps});
        if (it != cache.end()) return it->second;
    }
    const double pi = 3.14159265358979323846;
    const double h = 0.5 * (1.0 + eps);
    // Grid: 512 points uniform on [0, 1] and 512 log-spaced on [eps/64, 1].
    std::vector<double> lam;
    for (int i = 0; i < 512; ++i) lam.push_back(i / 511.0);
    const double l0 = std::log(eps / 64.0);
    for (int i = 0; i < 512; ++i) lam.push_back(std::exp(l0 * (1.0 - i / 511.0)));
    const int L = (int)lam.size();
    // log f_k(l) of the normalised pair factors, and their sum.
    std::vector<double> lf((size_t)n * L), total(L, 0.0);
    for (int k = 1; k <= n; ++k) {
        const double th = 2.0 * pi * k / (2 * n + 1);
        const double a = h * (1.0 - std::cos(th));
        const double bi = std::sqrt(eps) * std::sin(th);
        const double norm = 1.0 / ((h - a) * (h - a) + bi * bi);
        for (int i = 0; i < L; ++i) {
            const double v = std::log(((lam[i] - a) * (lam[i] - a) + bi * bi) * norm);
            lf[(size_t)(k - 1) * L + i] = v;
            total[i] += v;
        }
    }
    std::vector<double> pre(L, 0.0);
    std::vector<char> used(n, 0);
    std::vector<int> order;
    order.reserve(n);
    for (int step = 0; step < n; ++step) {
        int best = -1;
        double best_m = 0.0;
        for (int k = 0; k < n; ++k) {
            if (used[k]) continue;
            const double* f = &lf[(size_t)k * L];
            double mp = 0.0, ms = -1e300;
            for (int i = 0; i < L; ++i) {
                const double p = pre[i] + f[i];
                mp = std::max(mp, p);
                ms = std::max(ms, total[i] - p);
            }
            const double m = mp + ms;
            if (best < 0 || m < best_m) {
                best = k;
                best_m = m;
            }
        }
        used[best] = 1;
        order.push_back(best + 1);
        for (int i = 0; i < L; ++i) pre[i] += lf[(size_t)best * L + i];
    }
    std::lock_guard<std::mutex> lk(mu);
    cache[{n, eps}] = order;
    return order;
}

}  // namespace

std::vector<ChebFactor> cheb_factors(int n, double eps, double scale) {
    const double pi = 3.14159265358979323846;
    const double h = 0.5 * (1.0 + eps);
    const std::vector<int> order = factor_order(n, eps);
    std::vector<ChebFactor> f;
    f.reserve(n);
    for (int k : order) {
        const double th = 2.0 * pi * k / (2 * n + 1);
        const double a = h * (1.0 - std::cos(th));       // Re z_{2n,k}
        const double bi = std::sqrt(eps) * std::sin(th);  // -Im z_{2n,k}
        const double norm = 1.0 / ((h - a) * (h - a) + bi * bi);
        ChebFactor c;
        c.c2 = norm / (scale * scale);
        c.c1 = -2.0 * a * norm / scale;
        c.c0 = (a * a + bi * bi) * norm;
        f.push_back(c);
    }
    // The remaining constant of c_{2n}: 1 / h.
    f.back().c2 /= h;
    f.back().c1 /= h;
    f.back().c0 /= h;
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
                       double* partials, const std::vector<ChebFactor>& f, bool dot,
                       hipStream_t st) {
    const int n = (int)f.size();
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
    const std::vector<ChebFactor> f = cheb_factors(c.n, c.eps, scale);
    const size_t vb = ((size_t)g.V * 8 + 255) & ~size_t(255);
    char* ws = nullptr;
    const size_t bytes = vb * (P.fused ? 1 : 2);
    if (hipMallocAsync((void**)&ws, bytes, st) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(HUB_E_NOMEM, "hub_apply_cheb: cannot allocate %zu bytes", bytes);
    }
    double* w = (double*)ws;
    double* y = P.fused ? nullptr : (double*)(ws + vb);
    const hub_status s = launch_cheb(g, P, links, nullptr, r, z, w, y, nullptr, f, false, st);
    const hipError_t e = hipFreeAsync(ws, st);
    if (s != HUB_OK) return s;
    if (e != hipSuccess) return set_error(HUB_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
    return HUB_OK;
}

}  // namespace hub
