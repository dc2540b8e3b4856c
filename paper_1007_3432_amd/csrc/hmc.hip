// Hybrid Monte Carlo, the phi-algorithm of Sec. 4.1: the force of the
// pseudofermion action S_p = phi^T Q^{-1} phi, the leapfrog molecular
// dynamics (MD) trajectory with one CG solve of Q x = phi per force
// evaluation, and the Metropolis step.
//
// The field sigma_{n,s} enters M only through the time link of row s' = s+1
// (mod nt), A_{n,s'} = sg(s') e^{dtau mu} (1 + b sin sigma_{n,s}) with
// sg(0) = +1 (antiperiodic wrap) and sg(s') = -1 otherwise, so with y = M x
//   dS_p/dsigma_{n,s} = -2 y_{n,s'} sg(s') e^{dtau mu} b cos(sigma_{n,s}) x_{n,s}.
// MD Hamiltonian H = 1/2 pi.pi + S_p (the compact field has a flat measure,
// so there is no separate field action), S_p = phi . x.
#include <cmath>

#include "cgtiles.h"
#include "internal.h"

namespace hub {

// What the force kernel does with F at each site.
enum ForceMode : int {
    kForceOut = 0,    // out[i] = F
    kKick = 1,        // pi[i] -= c F
    kKickDrift = 2,   // pi[i] -= c F, then sigma[i] += eps pi[i]
};

// One lane per site; x at the time-neighbour row and its spatial
// neighbours come through L1/L2.  Only sigma[i] and pi[i] of the lane's own
// site are read and written, so the in-place drift is race-free.
template <int MODE, int D>
__global__ __launch_bounds__(256) void k_force(Geom g, double* __restrict__ sigma,
                                               const double* __restrict__ x,
                                               double* __restrict__ out, double c, double eps) {
    const int i = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (i >= g.V) return;
    const int s = fdiv(i, g.fvs), n = i - s * g.vs;
    const int sp = s + 1 == g.nt ? 0 : s + 1;
    const int ip = n + sp * g.vs;
    double hop = 0.0;
    int rest = n, stride = 1;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        // coordinate j of n; the last one is what is left (< nx)
        const int q = j + 1 < D ? fdiv(rest, g.fnx) : 0;
        const int cj = j + 1 < D ? rest - q * g.nx : rest;
        const int cpj = cj + 1 == g.nx ? 0 : cj + 1;
        const int cmj = cj == 0 ? g.nx - 1 : cj - 1;
        hop += x[ip + (cpj - cj) * stride] + x[ip + (cmj - cj) * stride];
        stride *= g.nx;
        rest = q;
    }
    const double sg = sp == 0 ? g.lscale : -g.lscale;
    const double sv = sigma[i];
    double sn, cs;
    sincos(sv, &sn, &cs);
    const double xi = x[i];
    const double y = x[ip] - g.kappa * hop + sg * (1.0 + g.b * sn) * xi;
    const double F = -2.0 * y * (sg * g.b * cs) * xi;
    if constexpr (MODE == kForceOut) {
        out[i] = F;
    } else {
        const double p = out[i] - c * F;
        out[i] = p;
        if constexpr (MODE == kKickDrift) sigma[i] = sv + eps * p;
    }
}

// The same force for even nx, two x-adjacent sites per lane (16-byte loads
// and stores; the x neighbours of the pair are its own two values and one
// more site on each side).  Each site's arithmetic is that of k_force, in
// the same order.
template <int MODE, int D>
__global__ __launch_bounds__(256) void k_force2(Geom g, double* __restrict__ sigma,
                                                const double* __restrict__ x,
                                                double* __restrict__ out, double c, double eps) {
    const int i = 2 * (xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x);  // first site of the pair
    if (i >= g.V) return;
    const int s = fdiv(i, g.fvs), n = i - s * g.vs;
    const int sp = s + 1 == g.nt ? 0 : s + 1;
    const int ip = n + sp * g.vs;
    auto ld2v = [](const double* p) { return *reinterpret_cast<const double2*>(p); };
    const double2 xp = ld2v(x + ip);  // x at the next slice: sites a, b
    double hop_a = 0.0, hop_b = 0.0;
    int rest = n, stride = 1;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const int q = j + 1 < D ? fdiv(rest, g.fnx) : 0;
        const int cj = j + 1 < D ? rest - q * g.nx : rest;
        if (j == 0) {
            // cj is even: a = cj, b = cj + 1 < nx
            const double left_a = x[ip + (cj == 0 ? g.nx - 1 : -1)];
            const double right_b = x[ip + (cj + 2 == g.nx ? 2 - g.nx : 2)];
            hop_a += xp.y + left_a;
            hop_b += right_b + xp.x;
        } else {
            const int cpj = cj + 1 == g.nx ? 0 : cj + 1;
            const int cmj = cj == 0 ? g.nx - 1 : cj - 1;
            const double2 pl = ld2v(x + ip + (cpj - cj) * stride);
            const double2 mi = ld2v(x + ip + (cmj - cj) * stride);
            hop_a += pl.x + mi.x;
            hop_b += pl.y + mi.y;
        }
        stride *= g.nx;
        rest = q;
    }
    const double sg = sp == 0 ? g.lscale : -g.lscale;
    const double2 sv = ld2v(sigma + i), xi = ld2v(x + i);
    double sn_a, cs_a, sn_b, cs_b;
    sincos(sv.x, &sn_a, &cs_a);
    sincos(sv.y, &sn_b, &cs_b);
    const double y_a = xp.x - g.kappa * hop_a + sg * (1.0 + g.b * sn_a) * xi.x;
    const double y_b = xp.y - g.kappa * hop_b + sg * (1.0 + g.b * sn_b) * xi.y;
    const double F_a = -2.0 * y_a * (sg * g.b * cs_a) * xi.x;
    const double F_b = -2.0 * y_b * (sg * g.b * cs_b) * xi.y;
    if constexpr (MODE == kForceOut) {
        *reinterpret_cast<double2*>(out + i) = make_double2(F_a, F_b);
    } else {
        const double2 po = ld2v(out + i);
        const double p_a = po.x - c * F_a, p_b = po.y - c * F_b;
        *reinterpret_cast<double2*>(out + i) = make_double2(p_a, p_b);
        if constexpr (MODE == kKickDrift)
            *reinterpret_cast<double2*>(sigma + i) = make_double2(sv.x + eps * p_a, sv.y + eps * p_b);
    }
}

// Deposits of 1/2 pi.pi and phi.x (FP64, tile order), then the one-block sum.
__global__ __launch_bounds__(256) void k_energy(const double* __restrict__ pi,
                                                const double* __restrict__ phi,
                                                const double* __restrict__ x, int V,
                                                double* partials) {
    const int base = lane_base(blockIdx.x), cnt = lane_count(base, V);
    double a[8], f[8], y[8];
    if (cnt == 8) {
        ld8(pi + base, a);
        ld8(phi + base, f);
        ld8(x + base, y);
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a[k] = k < cnt ? pi[base + eoff(k)] : 0.0;
            f[k] = k < cnt ? phi[base + eoff(k)] : 0.0;
            y[k] = k < cnt ? x[base + eoff(k)] : 0.0;
        }
    }
    double part[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        part[0] += a[k] * a[k];
        part[1] += f[k] * y[k];
    }
    deposit<256, 2>(part, partials, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_energy_finish(const double* partials, int n,
                                                       double* out) {
    double tot[2];
    reduce_deposits<256, 2>(partials, n, tot);
    if (threadIdx.x == 0) {
        out[0] = 0.5 * tot[0];
        out[1] = tot[1];
    }
}

hub_status launch_force(const Geom& g, int mode, double* sigma, const double* x, double* out,
                        double c, double eps, hipStream_t st) {
    // Even nx: two sites per lane (every row, hence V, is even).
    const bool pairs = (g.nx & 1) == 0;
    const int grid = pairs ? ceil_div(g.V / 2, 256) : ceil_div(g.V, 256);
#define HUB_FORCE(M, D)                                                          \
    do {                                                                         \
        if (pairs)                                                               \
            k_force2<M, D><<<grid, 256, 0, st>>>(g, sigma, x, out, c, eps);      \
        else                                                                     \
            k_force<M, D><<<grid, 256, 0, st>>>(g, sigma, x, out, c, eps);       \
    } while (0)
#define HUB_FORCE_D(M)                              \
    switch (g.d) {                                  \
        case 1: HUB_FORCE(M, 1); break;             \
        case 2: HUB_FORCE(M, 2); break;             \
        default: HUB_FORCE(M, 3); break;            \
    }
    switch (mode) {
        case kForceOut:
            HUB_FORCE_D(kForceOut)
            break;
        case kKick:
            HUB_FORCE_D(kKick)
            break;
        default:
            HUB_FORCE_D(kKickDrift)
            break;
    }
#undef HUB_FORCE_D
#undef HUB_FORCE
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

namespace {

#define HUB_TRY(expr)                \
    do {                             \
        hub_status s_ = (expr);      \
        if (s_ != HUB_OK) return s_; \
    } while (0)

struct MDWork {
    double* x;         // V: CG solution of the latest force evaluation
    double* partials;  // 2 * elem_tiles(V)
    double* energy;    // [2]: 1/2 pi.pi, phi.x
};

// H = 1/2 pi.pi + phi.x (x the solution at the current field).
hub_status energy(const Geom& g, const double* pi, const double* phi, const MDWork& w,
                  double* h, hipStream_t st) {
    const int tiles = elem_tiles(g.V);
    k_energy<<<tiles, 256, 0, st>>>(pi, phi, w.x, g.V, w.partials);
    k_energy_finish<<<1, 256, 0, st>>>(w.partials, tiles, w.energy);
    HUB_HIP(hipGetLastError());
    double e[2];
    HUB_HIP(hipMemcpyAsync(e, w.energy, sizeof(e), hipMemcpyDeviceToHost, st));
    HUB_HIP(hipStreamSynchronize(st));
    *h = e[0] + e[1];
    return HUB_OK;
}

hub_status md_solve(const Geom& g, const double* sigma, const double* phi, const MDWork& w,
                    const hub_cg_opts& o, hub_md_stats* s, hipStream_t st) {
    hub_cg_stats cs{};
    const hub_status r = cg_solve(g, sigma, phi, w.x, o, &cs, st);
    s->solves += 1;
    s->cg_iters += cs.iters;
    return r;
}

// Leapfrog from (sigma, pi), both updated in place: a half kick, then
// n_steps drifts each followed by a force evaluation and a full kick (half
// for the last).  The drift after a kick is fused into the kick kernel.
hub_status md_run(const Geom& g, double* sigma, double* pi, const double* phi,
                  const hub_md_opts& o, const MDWork& w, hub_md_stats* s, hipStream_t st) {
    HUB_TRY(md_solve(g, sigma, phi, w, o.cg, s, st));
    HUB_TRY(energy(g, pi, phi, w, &s->h_start, st));
    HUB_TRY(launch_force(g, kKickDrift, sigma, w.x, pi, 0.5 * o.eps, o.eps, st));
    for (int k = 1; k <= o.n_steps; ++k) {
        HUB_TRY(md_solve(g, sigma, phi, w, o.cg, s, st));
        if (k < o.n_steps)
            HUB_TRY(launch_force(g, kKickDrift, sigma, w.x, pi, o.eps, o.eps, st));
        else
            HUB_TRY(launch_force(g, kKick, sigma, w.x, pi, 0.5 * o.eps, 0.0, st));
    }
    return energy(g, pi, phi, w, &s->h_end, st);
}

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

hub_status hmc_force(const Geom& g, const double* sigma, const double* x, double* F,
                     hipStream_t st) {
    return launch_force(g, kForceOut, const_cast<double*>(sigma), x, F, 0.0, 0.0, st);
}

// hub_md_trajectory / hub_hmc_trajectory (arguments already validated).
// eta == nullptr: MD only, phi given, sigma and pi updated in place.
// eta != nullptr: phi = M^T eta, MD on copies of sigma and pi0, Metropolis.
hub_status md_trajectory(const Geom& g, double* sigma, double* pi, const double* phi,
                         const double* eta, const double* pi0, double u, const hub_md_opts& o,
                         hub_md_stats* out, hipStream_t st) {
    const size_t V = (size_t)g.V;
    const bool hmc = eta != nullptr;
    size_t off = 0;
    const size_t o_x = off; off += al256(8 * V);
    const size_t o_part = off; off += al256(16 * (size_t)elem_tiles(g.V));
    const size_t o_e = off; off += 256;
    const size_t o_phi = off; off += hmc ? al256(8 * V) : 0;
    const size_t o_sig = off; off += hmc ? al256(8 * V) : 0;
    const size_t o_pi = off; off += hmc ? al256(8 * V) : 0;
    char* ws = nullptr;
    if (hipMallocAsync((void**)&ws, off, st) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(HUB_E_NOMEM, "MD trajectory: cannot allocate %zu bytes", off);
    }
    MDWork w{(double*)(ws + o_x), (double*)(ws + o_part), (double*)(ws + o_e)};
    hub_md_stats s{};
    hub_status r = HUB_OK;
    if (!hmc) {
        r = md_run(g, sigma, pi, phi, o, w, &s, st);
    } else {
        double* phi_w = (double*)(ws + o_phi);
        double* sig_w = (double*)(ws + o_sig);
        double* pi_w = (double*)(ws + o_pi);
        // Heatbath phi = M^T eta at the starting field (links into sig_w,
        // which the copy below then overwrites).
        r = launch_links(g, sigma, sig_w, HUB_F64, st);
        if (r == HUB_OK) r = launch_apply_M(g, sig_w, HUB_F64, HUB_F64, eta, phi_w, 1, st);
        if (r == HUB_OK) {
            const hipError_t e1 = hipMemcpyAsync(sig_w, sigma, 8 * V, hipMemcpyDeviceToDevice, st);
            const hipError_t e2 = hipMemcpyAsync(pi_w, pi0, 8 * V, hipMemcpyDeviceToDevice, st);
            if (e1 != hipSuccess || e2 != hipSuccess)
                r = set_error(HUB_E_DEVICE, "MD trajectory: copy failed");
        }
        if (r == HUB_OK) r = md_run(g, sig_w, pi_w, phi_w, o, w, &s, st);
        if (r == HUB_OK) {
            s.accepted = u < std::exp(-(s.h_end - s.h_start)) ? 1 : 0;
            if (s.accepted &&
                hipMemcpyAsync(sigma, sig_w, 8 * V, hipMemcpyDeviceToDevice, st) != hipSuccess)
                r = set_error(HUB_E_DEVICE, "MD trajectory: copy failed");
        }
    }
    const hipError_t ef = hipFreeAsync(ws, st);
    const hipError_t es = hipStreamSynchronize(st);
    s.status = r;
    if (out) *out = s;
    if (r != HUB_OK) return r;
    if (ef != hipSuccess || es != hipSuccess)
        return set_error(HUB_E_DEVICE, "MD trajectory: %s",
                         hipGetErrorString(ef != hipSuccess ? ef : es));
    return HUB_OK;
}

}  // namespace hub
