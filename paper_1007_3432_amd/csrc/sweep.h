// Host-side planning and launch of one Q = M^T M sweep with a given op.
#pragma once

#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "cgtiles.h"
#include "internal.h"
#include "stencil.h"

namespace hub {

// Tile shapes of the fused d = 1 kernel: TX sites in x x TT slices.
enum D1Tile { kD1_256x8 = 0, kD1_128x8, kD1_64x8, kD1_256x4, kD1_256x16, kD1_128x16,
              kD1_256x2, kD1_256x1, kD1_128x4, kD1_64x4, kD1_Count };
struct D1Shape { int tx, tt; };
static constexpr D1Shape kD1Shapes[kD1_Count] = {
    {256, 8}, {128, 8}, {64, 8}, {256, 4}, {256, 16}, {128, 16},
    {256, 2}, {256, 1}, {128, 4}, {64, 4}};

// Tile shapes of the fused d = 3 kernel: whole rows of NX x TY x TZ, swept
// by blocks of `block` lanes.  Mixed-precision solves (and with them the
// serving kernel, which must take the same steps) use 256-lane tiles only.
enum D3Tile { kD3_8x8x8 = 0, kD3_16x4x4, kD3_16x8x8, kD3_32x4x4, kD3_32x8x4, kD3_64x4x4,
              kD3_16x8x4, kD3_32x8x8_512, kD3_64x4x4_512, kD3_64x8x4_512, kD3_16x8x8_512,
              kD3_32x8x4_512, kD3_32x4x4_512, kD3_16x8x4_512, kD3_8x8x8_512, kD3_Count };
struct D3Shape { int nx, ty, tz, block; };
static constexpr D3Shape kD3Shapes[kD3_Count] = {
    {8, 8, 8, 256}, {16, 4, 4, 256}, {16, 8, 8, 256}, {32, 4, 4, 256}, {32, 8, 4, 256},
    {64, 4, 4, 256}, {16, 8, 4, 256}, {32, 8, 8, 512}, {64, 4, 4, 512}, {64, 8, 4, 512},
    {16, 8, 8, 512}, {32, 8, 4, 512}, {32, 4, 4, 512}, {16, 8, 4, 512}, {8, 8, 8, 512}};

enum SweepKind { kSweepD1 = 0, kSweepD3, kSweepGeneric };

// Pair tiles of the d = 1 sweep (FP64, nx even): TX sites x TT slices.
enum D1PTile { kD1P_512x2 = 0, kD1P_256x2, kD1P_128x2, kD1P_512x4, kD1P_512x1, kD1P_Count };
static constexpr D1Shape kD1PShapes[kD1P_Count] = {
    {512, 2}, {256, 2}, {128, 2}, {512, 4}, {512, 1}};

struct SweepPlan {
    int kind;      // SweepKind
    bool fused;    // single pass (kSweepD1 / kSweepD3)
    bool pair;     // kSweepD1 with the pair tile (variant is a D1PTile)
    int variant;   // D1Tile, D1PTile or D3Tile
    int tiles_x;   // d = 1
    int tiles_y, tiles_z, tc;  // d = 3: tiles and slices per block
    int ntiles;    // tiles of one sweep = deposits of its reductions
    int grid;      // blocks of the sweep kernel (pass 2 when generic)
};

// Tuning aids: HUB_D1_TILE=<TX>x<TT>,
// HUB_D3_TILE=<NX>x<TY>x<TZ>[@512], HUB_D3_TC=<slices per block>, HUB_SWEEP=generic.
inline const char* env_or_null(const char* k) { return std::getenv(k); }

inline int d1_tile_override() {
    static int v = [] {
        const char* e = env_or_null("HUB_D1_TILE");
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

inline int d3_tile_override() {
    static int v = [] {
        const char* e = env_or_null("HUB_D3_TILE");
        if (!e) return -1;
        for (int k = 0; k < kD3_Count; ++k) {
            char buf[32];
            if (kD3Shapes[k].block == 256)
                std::snprintf(buf, sizeof(buf), "%dx%dx%d", kD3Shapes[k].nx, kD3Shapes[k].ty,
                              kD3Shapes[k].tz);
            else
                std::snprintf(buf, sizeof(buf), "%dx%dx%d@%d", kD3Shapes[k].nx, kD3Shapes[k].ty,
                              kD3Shapes[k].tz, kD3Shapes[k].block);
            if (std::strcmp(buf, e) == 0) return k;
        }
        return -1;
    }();
    return v;
}

inline int d1p_tile_override() {
    static int v = [] {
        const char* e = env_or_null("HUB_D1P_TILE");
        if (!e) return -1;
        if (std::strcmp(e, "off") == 0) return -2;
        for (int k = 0; k < kD1P_Count; ++k) {
            char buf[32];
            std::snprintf(buf, sizeof(buf), "%dx%d", kD1PShapes[k].tx, kD1PShapes[k].tt);
            if (std::strcmp(buf, e) == 0) return k;
        }
        return -1;
    }();
    return v;
}

inline int env_int(const char* k, int dflt) {
    const char* e = env_or_null(k);
    return e ? std::atoi(e) : dflt;
}

inline bool force_generic() {
    static bool v = [] {
        const char* e = env_or_null("HUB_SWEEP");
        return e && std::strcmp(e, "generic") == 0;
    }();
    return v;
}

// f64: the sweep's ops are FP64 throughout, so the pair tile may serve d = 1.
// solve: the plan of an FP64 solver (CG phase A and the true residual), which
// may take another d = 3 tile than the bare product.
inline SweepPlan plan_sweep(const Geom& g, bool f64, bool solve = false) {
    SweepPlan p{};
    p.kind = kSweepGeneric;
    p.variant = -1;
    p.pair = false;
    const int pv = d1p_tile_override();
    if (!force_generic() && g.d == 1 && f64 && g.nx % 2 == 0 && pv != -2) {
        int v = pv;
        if (v < 0) v = g.nx >= 512 ? kD1P_512x2 : (g.nx >= 256 ? kD1P_256x2 : kD1P_128x2);
        p.kind = kSweepD1;
        p.pair = true;
        p.variant = v;
        p.tiles_x = ceil_div(g.nx, kD1PShapes[v].tx);
        p.ntiles = p.tiles_x * ceil_div(g.nt, kD1PShapes[v].tt);
        p.grid = p.ntiles;
    } else if (!force_generic() && g.d == 1) {
        int v = d1_tile_override();
        if (v < 0) v = g.nx >= 256 ? kD1_256x4 : (g.nx >= 128 ? kD1_128x4 : kD1_64x4);
        p.kind = kSweepD1;
        p.variant = v;
        p.tiles_x = ceil_div(g.nx, kD1Shapes[v].tx);
        p.ntiles = p.tiles_x * ceil_div(g.nt, kD1Shapes[v].tt);
        p.grid = p.ntiles;
    } else if (!force_generic() && g.d == 3) {
        int v = d3_tile_override();
        if (v >= 0 && (kD3Shapes[v].nx != g.nx || (!f64 && kD3Shapes[v].block != 256))) v = -1;
        if (v < 0) {
            // Measured on MI355X (bare FP64 and FP32 sweeps on 8^3 x 80,
            // 16^3 x 160, 32^3 x 256, 64^3 x 32): FP64 sweeps run best on
            // 512-lane blocks for nx = 16, 32 (fewer registers per lane than
            // the 256-lane tiles, whose FP64 CG variant needs 256 VGPRs);
            // mixed-precision plans stay on 256-lane tiles.
            switch (g.nx) {
                case 8: v = kD3_8x8x8; break;
                case 16: v = f64 ? kD3_16x8x4_512 : kD3_16x4x4; break;
                // The FP64 CG iteration on 32^3 x 256 ran faster on 32x8x8
                // (143.7 vs 150.6 us), the bare FP64 sweep on 32x8x4 (59 vs
                // 63 us).
                case 32: v = f64 ? (solve ? kD3_32x8x8_512 : kD3_32x8x4_512) : kD3_32x8x4; break;
                case 64: v = f64 ? kD3_64x4x4_512 : kD3_64x4x4; break;
                default: v = -1;
            }
        }
        if (v >= 0) {
            const D3Shape sh = kD3Shapes[v];
            p.kind = kSweepD3;
            p.variant = v;
            p.tiles_y = g.nx / sh.ty;
            p.tiles_z = g.nx / sh.tz;
            const int tiles = p.tiles_y * p.tiles_z;
            // Slices per block: the sweeps ran best with about 128K lanes in
            // the grid (one 512-lane or two 256-lane blocks per CU), long
            // marches amortising each block's prologue slice.
            long long tcl = ((long long)g.nt * tiles * sh.block + 131071) / 131072;
            int tc = (int)(tcl < 2 ? 2 : (tcl > 16 ? 16 : tcl));
            tc = env_int("HUB_D3_TC", tc);
            if (tc < 1) tc = 1;
            p.tc = tc;
            p.ntiles = tiles * ceil_div(g.nt, tc);
            p.grid = p.ntiles;
        }
    }
    if (p.kind == kSweepGeneric) p.ntiles = p.grid = ceil_div(g.V, 256);
    p.fused = p.kind != kSweepGeneric;
    return p;
}

// Doubles of deposit space any reduction over this geometry may need:
// kMaxNP sums for each tile of the largest grid (sweep or element-wise).
inline int max_partials(const Geom& g) {
    const SweepPlan p = plan_sweep(g, false), q = plan_sweep(g, true),
                    r = plan_sweep(g, true, true);
    const int e = elem_tiles(g.V);
    int m = p.ntiles > e ? p.ntiles : e;
    m = q.ntiles > m ? q.ntiles : m;
    m = r.ntiles > m ? r.ntiles : m;
    return kMaxNP * m;
}

// Slices in flight per block of the d = 3 sweep.  Measured on MI355X: FP32
// ops gain from loading two slices ahead (the mixed-precision CG iteration
// on 32^3 x 256 with FP16 links: 75.6 -> 67.0 us); FP64 ops do not (the
// FP64 sweep and CG on the same lattice: 57.3 -> 58.9 us, 154 -> 159 us).
template <class Op>
constexpr int d3_prefetch_depth() {
    return sizeof(typename Op::acc_t) == 4 ? 2 : 1;
}

// Slices per block of the completely unrolled d = 3 march, and whether a
// plan can take it (every block marching exactly that many slices).  Only
// the bare FP64 product takes it, with two slices in flight: 32^3 x 256
// 58.0 -> 55.0 us; the FP64 CG phase A would spill registers on it (140 ->
// 198 us per iteration), the mixed one gains nothing.
constexpr int kD3Unroll = 16;
inline bool d3_unrolled_ok(const Geom& g, const SweepPlan& P) {
    return P.tc == kD3Unroll && g.nt % kD3Unroll == 0;
}
template <class Op>
constexpr int d3_unrolled_depth() {
    return 2;
}

// One sweep: z = Q in, consumed by op.out().  y: scratch of g.V acc_t
// elements, used by the generic path only.  A reducing op's deposits go to
// partials; with finalize, a one-block kernel then adds them (op.finish),
// otherwise the next kernel does.
template <class Op>
hub_status launch_q(const Geom& g, const SweepPlan& P, const Op& op,
                    typename Op::acc_t* y, double* partials, hipStream_t st,
                    bool finalize = true) {
    if (P.kind == kSweepD1 && P.pair) {
        if constexpr (op_marches<Op>::value) {
            // The bare product takes the marching tile (8 slices per
            // wavefront, all but the last stage's loads issued up front) on
            // lattices of 2^19 sites and more, unless a pair tile is forced
            // for tuning.  Measured on MI355X: at 2^20 sites and above the
            // marching tile is faster (d=1 2048x512 streamed from HBM 8.0 ->
            // 6.8 us), at 2^18 and below the shorter chains of the two-slice
            // tile win (d=1 1024x256: 2.8 vs 4.2 us).  The plan's deposit
            // count is the pair tile's, so only ops without a reduction may
            // march.
            static_assert(!Op::kReduce, "a marching sweep leaves no pair-tile deposits");
            if (d1p_tile_override() < 0 && g.V >= (1 << 19)) {
                constexpr int kTS = 8, kPF = 8;
                const int tx = kD1PShapes[P.variant].tx;
                const int ntiles = P.tiles_x * ceil_div(g.nt, kTS);
                switch (tx) {
                    case 512:
                        k_mtm_d1m<Op, 512, kTS, kPF><<<ntiles, 256, 0, st>>>(g, op, P.tiles_x,
                                                                             ntiles, partials);
                        break;
                    case 256:
                        k_mtm_d1m<Op, 256, kTS, kPF><<<ntiles, 128, 0, st>>>(g, op, P.tiles_x,
                                                                             ntiles, partials);
                        break;
                    default:
                        k_mtm_d1m<Op, 128, kTS, kPF><<<ntiles, 64, 0, st>>>(g, op, P.tiles_x,
                                                                            ntiles, partials);
                        break;
                }
                HUB_HIP(hipGetLastError());
                return HUB_OK;
            }
        }
        if constexpr (op_has_pair<Op>::value) {
            switch (P.variant) {
#define HUB_D1P_CASE(K, TX, TT)                                                         \
    case K:                                                                             \
        k_mtm_d1p<Op, TX, TT><<<P.grid, TX / 2, 0, st>>>(g, op, P.tiles_x, P.ntiles,     \
                                                          partials);                     \
        break;
                HUB_D1P_CASE(kD1P_512x2, 512, 2)
                HUB_D1P_CASE(kD1P_256x2, 256, 2)
                HUB_D1P_CASE(kD1P_128x2, 128, 2)
                HUB_D1P_CASE(kD1P_512x4, 512, 4)
                HUB_D1P_CASE(kD1P_512x1, 512, 1)
#undef HUB_D1P_CASE
                default:
                    return set_error(HUB_E_INVALID, "internal: bad d=1 pair tile variant");
            }
        } else {
            return set_error(HUB_E_INVALID, "internal: op has no pair access");
        }
    } else if (P.kind == kSweepD1) {
        switch (P.variant) {
#define HUB_D1_CASE(K, TX, TT)                                                             \
    case K:                                                                                \
        k_mtm_d1<Op, TX, TT><<<P.grid, TX, 0, st>>>(g, op, P.tiles_x, P.ntiles, partials); \
        break;
            HUB_D1_CASE(kD1_256x8, 256, 8)
            HUB_D1_CASE(kD1_128x8, 128, 8)
            HUB_D1_CASE(kD1_64x8, 64, 8)
            HUB_D1_CASE(kD1_256x4, 256, 4)
            HUB_D1_CASE(kD1_256x16, 256, 16)
            HUB_D1_CASE(kD1_128x16, 128, 16)
            HUB_D1_CASE(kD1_256x2, 256, 2)
            HUB_D1_CASE(kD1_256x1, 256, 1)
            HUB_D1_CASE(kD1_128x4, 128, 4)
            HUB_D1_CASE(kD1_64x4, 64, 4)
#undef HUB_D1_CASE
            default:
                return set_error(HUB_E_INVALID, "internal: bad d=1 tile variant");
        }
    } else if (P.kind == kSweepD3) {
        if (g.nx != kD3Shapes[P.variant].nx)
            return set_error(HUB_E_INVALID, "internal: d=3 tile does not fit nx");
        switch (P.variant) {
#define HUB_D3_CASE(K, NX, TY, TZ, B)                                                    \
    case K:                                                                              \
        if constexpr (NX >= 32 && op_marches<Op>::value) {                               \
            if (d3_unrolled_ok(g, P)) {                                                  \
                k_mtm_d3<Op, NX, TY, TZ, B, d3_unrolled_depth<Op>(), kD3Unroll>            \
                    <<<P.grid, B, 0, st>>>(g, op, P.tiles_y, P.tiles_z, P.tc, partials);  \
                break;                                                                   \
            }                                                                            \
        }                                                                                \
        k_mtm_d3<Op, NX, TY, TZ, B, d3_prefetch_depth<Op>()>                              \
            <<<P.grid, B, 0, st>>>(g, op, P.tiles_y, P.tiles_z, P.tc, partials);          \
        break;
            HUB_D3_CASE(kD3_8x8x8, 8, 8, 8, 256)
            HUB_D3_CASE(kD3_16x4x4, 16, 4, 4, 256)
            HUB_D3_CASE(kD3_16x8x8, 16, 8, 8, 256)
            HUB_D3_CASE(kD3_32x4x4, 32, 4, 4, 256)
            HUB_D3_CASE(kD3_32x8x4, 32, 8, 4, 256)
            HUB_D3_CASE(kD3_64x4x4, 64, 4, 4, 256)
            HUB_D3_CASE(kD3_16x8x4, 16, 8, 4, 256)
            HUB_D3_CASE(kD3_32x8x8_512, 32, 8, 8, 512)
            HUB_D3_CASE(kD3_64x4x4_512, 64, 4, 4, 512)
            HUB_D3_CASE(kD3_64x8x4_512, 64, 8, 4, 512)
            HUB_D3_CASE(kD3_16x8x8_512, 16, 8, 8, 512)
            HUB_D3_CASE(kD3_32x8x4_512, 32, 8, 4, 512)
            HUB_D3_CASE(kD3_32x4x4_512, 32, 4, 4, 512)
            HUB_D3_CASE(kD3_16x8x4_512, 16, 8, 4, 512)
            HUB_D3_CASE(kD3_8x8x8_512, 8, 8, 8, 512)
#undef HUB_D3_CASE
            default:
                return set_error(HUB_E_INVALID, "internal: bad d=3 tile variant");
        }
    } else {
        if (!y) return set_error(HUB_E_INVALID, "internal: generic sweep needs scratch");
        const int grid = ceil_div(g.V, 256);
        k_gen_pass1<Op><<<grid, 256, 0, st>>>(g, op, y);
        k_gen_pass2<Op><<<grid, 256, 0, st>>>(g, op, y, partials);
    }
    if constexpr (Op::kReduce) {
        if (!partials) return set_error(HUB_E_INVALID, "internal: reduction needs deposits");
        if (finalize) k_finish_op<Op><<<1, 256, 0, st>>>(op, partials, P.ntiles);
    }
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

}  // namespace hub
