// Host-side planning and launch of one Q = M^T M sweep with a given op.
#pragma once

#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "internal.h"
#include "stencil.h"

namespace hub {

// Tile shapes of the fused d = 1 kernel: TX sites in x x TT slices.
enum D1Tile { kD1_256x8 = 0, kD1_128x8, kD1_64x8, kD1_256x4, kD1_256x16, kD1_128x16,
              kD1_Count };
struct D1Shape { int tx, tt; };
static constexpr D1Shape kD1Shapes[kD1_Count] = {
    {256, 8}, {128, 8}, {64, 8}, {256, 4}, {256, 16}, {128, 16}};

struct SweepPlan {
    bool fused;
    int variant;   // D1Tile when fused
    int tiles_x;
    int grid;      // blocks of the sweep kernel (pass 2 when generic)
};

// HUB_D1_TILE=<TX>x<TT> forces a d = 1 tile shape (tuning aid).
inline int d1_tile_override() {
    static int v = [] {
        const char* e = std::getenv("HUB_D1_TILE");
        if (!e) return -1;
        for (int k = 0; k < kD1_Count; ++k) {
            char buf[32];
            std::snprintf(buf, sizeof(buf), "%dx%d", kD1Shapes[k].tx, kD1Shapes[k].tt);
            if (std::strcmp(buf, e) == 0) return k;
        }
        return -1;
    }();
    return v;
}

inline SweepPlan plan_sweep(const Geom& g) {
    SweepPlan p{};
    if (g.d == 1) {
        int v = d1_tile_override();
        if (v < 0) v = g.nx >= 256 ? kD1_256x8 : (g.nx >= 128 ? kD1_128x8 : kD1_64x8);
        p.fused = true;
        p.variant = v;
        p.tiles_x = ceil_div(g.nx, kD1Shapes[v].tx);
        p.grid = p.tiles_x * ceil_div(g.nt, kD1Shapes[v].tt);
    } else {
        p.fused = false;
        p.variant = -1;
        p.tiles_x = 0;
        p.grid = ceil_div(g.V, 256);
    }
    return p;
}

// Blocks of the grid-stride elementwise kernels: a function of V only, so
// that reductions are summed in the same order on every call.
inline int elementwise_grid(const Geom& g) {
    int b = ceil_div(g.V, 256 * 4);
    return b < 1 ? 1 : (b > 2048 ? 2048 : b);
}

// Deposit slots any reduction over this geometry may need.
inline int max_partials(const Geom& g) {
    const SweepPlan p = plan_sweep(g);
    int m = p.grid;
    const int e = elementwise_grid(g);
    return m > e ? m : e;
}

// One sweep: z = Q in, consumed by op.out().  y: scratch of g.V acc_t
// elements, used by the generic path only.
template <class Op>
hub_status launch_q(const Geom& g, const SweepPlan& P, const Op& op,
                    typename Op::acc_t* y, double* partials, uint32_t* ticket,
                    hipStream_t st) {
    if (P.fused) {
        switch (P.variant) {
#define HUB_D1_CASE(K, TX, TT)                                                   \
    case K:                                                                      \
        k_mtm_d1<Op, TX, TT><<<P.grid, TX, 0, st>>>(g, op, P.tiles_x, partials,  \
                                                     ticket);                    \
        break;
            HUB_D1_CASE(kD1_256x8, 256, 8)
            HUB_D1_CASE(kD1_128x8, 128, 8)
            HUB_D1_CASE(kD1_64x8, 64, 8)
            HUB_D1_CASE(kD1_256x4, 256, 4)
            HUB_D1_CASE(kD1_256x16, 256, 16)
            HUB_D1_CASE(kD1_128x16, 128, 16)
#undef HUB_D1_CASE
            default:
                return set_error(HUB_E_INVALID, "internal: bad tile variant");
        }
    } else {
        if (!y) return set_error(HUB_E_INVALID, "internal: generic sweep needs scratch");
        const int grid = ceil_div(g.V, 256);
        k_gen_pass1<Op><<<grid, 256, 0, st>>>(g, op, y);
        k_gen_pass2<Op><<<grid, 256, 0, st>>>(g, op, y, partials, ticket);
    }
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

}  // namespace hub
