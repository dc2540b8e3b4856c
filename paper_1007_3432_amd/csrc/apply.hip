// Link precompute and matrix-vector launchers of libhub.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "internal.h"
#include "stencil.h"

namespace hub {

// ---------------------------------------------------------------------------
// Errors

static thread_local char g_err[512];

hub_status set_error(hub_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

void clear_error() { g_err[0] = '\0'; }

const char* last_error() { return g_err; }

// ---------------------------------------------------------------------------
// Validation

hub_status make_geom(const hub_lattice* lat, Geom* g) {
    if (!lat) return set_error(HUB_E_INVALID, "lattice descriptor is NULL");
    if (lat->d < 1 || lat->d > 3)
        return set_error(HUB_E_INVALID, "d = %d, expected 1..3", lat->d);
    if (lat->nx < 2) return set_error(HUB_E_INVALID, "nx = %d, expected >= 2", lat->nx);
    if (lat->nt < 2) return set_error(HUB_E_INVALID, "nt = %d, expected >= 2", lat->nt);
    if (lat->reserved != 0)
        return set_error(HUB_E_INVALID, "lattice.reserved must be 0");
    if (!std::isfinite(lat->t_hop) || lat->t_hop < 0)
        return set_error(HUB_E_INVALID, "t_hop = %g, expected finite >= 0", lat->t_hop);
    if (!std::isfinite(lat->dtau) || !(lat->dtau > 0))
        return set_error(HUB_E_INVALID, "dtau = %g, expected finite > 0", lat->dtau);
    if (!std::isfinite(lat->U) || lat->U > 0)
        return set_error(HUB_E_INVALID,
                         "U = %g: the compact HS field needs an attractive U <= 0",
                         lat->U);
    if (!std::isfinite(lat->mu))
        return set_error(HUB_E_INVALID, "mu is not finite");
    long long vs = 1;
    for (int j = 0; j < lat->d; ++j) vs *= lat->nx;
    const long long V = vs * lat->nt;
    if (vs > 0x7fffffffLL || V > 0x7fffffffLL)
        return set_error(HUB_E_INVALID, "volume %lld exceeds 2^31 - 1 sites", V);
    g->d = lat->d;
    g->nx = lat->nx;
    g->nt = lat->nt;
    g->vs = (int)vs;
    g->V = (int)V;
    g->kappa = lat->dtau * lat->t_hop;
    g->lscale = std::exp(lat->dtau * lat->mu);
    g->b = std::sqrt(2.0 * (std::exp(-lat->dtau * lat->U) - 1.0));
    g->fnx = make_fastdiv((uint32_t)g->nx);
    g->fvs = make_fastdiv((uint32_t)g->vs);
    if (!std::isfinite(g->b) || !std::isfinite(g->lscale))
        return set_error(HUB_E_INVALID, "coupling or chemical potential overflows");
    return HUB_OK;
}

size_t dtype_size(hub_dtype t) {
    switch (t) {
        case HUB_F64: return 8;
        case HUB_F32: return 4;
        case HUB_F16: return 2;
    }
    return 0;
}

bool valid_pair(hub_dtype vec, hub_dtype link) {
    return (vec == HUB_F64 && link == HUB_F64) ||
           (vec == HUB_F32 && (link == HUB_F32 || link == HUB_F16));
}

// ---------------------------------------------------------------------------
// Links (Sec. 2, Eqs. (8), (10)): A_{n,s} = -+exp(dtau mu)(1 + b sin sigma_{n,s-1}).

template <class T>
__global__ __launch_bounds__(256) void k_links(Geom g, const double* __restrict__ sigma,
                                               T* __restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= g.V) return;
    const int s = fdiv(i, g.fvs), n = i - s * g.vs;
    const int sm = s == 0 ? g.nt - 1 : s - 1;
    const double sn = sin(sigma[n + sm * g.vs]);
    if constexpr (sizeof(T) == 2) {
        out[i] = (T)sn;  // single round-to-nearest double -> half
    } else {
        const double l = g.lscale * (1.0 + g.b * sn);
        out[i] = (T)(s == 0 ? l : -l);
    }
}

// The same for even nx, two x-adjacent sites per lane (one 16-byte load of
// sigma, one store of both links); each site's arithmetic is k_links'.
template <class T>
__global__ __launch_bounds__(256) void k_links2(Geom g, const double* __restrict__ sigma,
                                                T* __restrict__ out) {
    const int i = 2 * (blockIdx.x * 256 + threadIdx.x);  // first site of the pair
    if (i >= g.V) return;
    const int s = fdiv(i, g.fvs), n = i - s * g.vs;
    const int sm = s == 0 ? g.nt - 1 : s - 1;
    const double2 sg = *reinterpret_cast<const double2*>(sigma + n + sm * g.vs);
    const double sa = sin(sg.x), sb = sin(sg.y);
    typedef T t2 __attribute__((ext_vector_type(2)));
    t2 v;
    if constexpr (sizeof(T) == 2) {
        v.x = (T)sa;  // single round-to-nearest double -> half
        v.y = (T)sb;
    } else {
        const double la = g.lscale * (1.0 + g.b * sa);
        const double lb = g.lscale * (1.0 + g.b * sb);
        v.x = (T)(s == 0 ? la : -la);
        v.y = (T)(s == 0 ? lb : -lb);
    }
    *reinterpret_cast<t2*>(out + i) = v;
}

hub_status launch_links(const Geom& g, const double* sigma, void* links,
                        hub_dtype link, hipStream_t st) {
    // Even nx: two sites per lane (every row, hence V, is even).
    const bool pairs = (g.nx & 1) == 0;
    const int grid = pairs ? ceil_div(g.V / 2, 256) : ceil_div(g.V, 256);
    switch (link) {
        case HUB_F64:
            if (pairs)
                k_links2<double><<<grid, 256, 0, st>>>(g, sigma, (double*)links);
            else
                k_links<double><<<grid, 256, 0, st>>>(g, sigma, (double*)links);
            break;
        case HUB_F32:
            if (pairs)
                k_links2<float><<<grid, 256, 0, st>>>(g, sigma, (float*)links);
            else
                k_links<float><<<grid, 256, 0, st>>>(g, sigma, (float*)links);
            break;
        case HUB_F16:
            if (pairs)
                k_links2<_Float16><<<grid, 256, 0, st>>>(g, sigma, (_Float16*)links);
            else
                k_links<_Float16><<<grid, 256, 0, st>>>(g, sigma, (_Float16*)links);
            break;
    }
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

// ---------------------------------------------------------------------------
// M and M^T

template <class Acc, class Vec, class Lnk>
static hub_status apply_M_t(const Geom& g, Lnk lk, const void* x, void* y,
                            int transpose, hipStream_t st) {
    const int grid = ceil_div(g.V, 256);
    if (transpose)
        k_apply_M<Acc, Vec, Lnk, true><<<grid, 256, 0, st>>>(g, lk, (const Vec*)x, (Vec*)y);
    else
        k_apply_M<Acc, Vec, Lnk, false><<<grid, 256, 0, st>>>(g, lk, (const Vec*)x, (Vec*)y);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

// FP64 with even nx: two sites per lane (every row, hence V, is even).
template <bool TRANSPOSE>
static void apply_M2_d(const Geom& g, const double* A, const double* x, double* y,
                       hipStream_t st) {
    const int grid = ceil_div(g.V / 2, 256);
    switch (g.d) {
        case 1: k_apply_M2<TRANSPOSE, 1><<<grid, 256, 0, st>>>(g, A, x, y); break;
        case 2: k_apply_M2<TRANSPOSE, 2><<<grid, 256, 0, st>>>(g, A, x, y); break;
        default: k_apply_M2<TRANSPOSE, 3><<<grid, 256, 0, st>>>(g, A, x, y); break;
    }
}

Link16 make_link16(const Geom& g, const void* links) {
    Link16 l;
    l.sn = (const _Float16*)links;
    l.ls = (float)g.lscale;
    l.lb = (float)(g.lscale * g.b);
    return l;
}

hub_status launch_apply_M(const Geom& g, const void* links, hub_dtype link,
                          hub_dtype vec, const void* x, void* y, int transpose,
                          hipStream_t st) {
    if (vec == HUB_F64 && (g.nx & 1) == 0) {
        if (transpose)
            apply_M2_d<true>(g, (const double*)links, (const double*)x, (double*)y, st);
        else
            apply_M2_d<false>(g, (const double*)links, (const double*)x, (double*)y, st);
        HUB_HIP(hipGetLastError());
        return HUB_OK;
    }
    if (vec == HUB_F64)
        return apply_M_t<double, double>(g, Link64{(const double*)links}, x, y, transpose, st);
    if (link == HUB_F32)
        return apply_M_t<float, float>(g, Link32{(const float*)links}, x, y, transpose, st);
    return apply_M_t<float, float>(g, make_link16(g, links), x, y, transpose, st);
}

}  // namespace hub
