// hub_apply_MtM launcher: one fused sweep z = M^T M x.
#include "sweep.h"

namespace hub {

Link16 make_link16(const Geom& g, const void* links);

bool mtm_fused(const Geom& g, hub_dtype vec) { return plan_sweep(g, vec == HUB_F64).fused; }

size_t mtm_scratch_bytes(const Geom& g, hub_dtype vec) {
    return mtm_fused(g, vec) ? 0 : (size_t)g.V * dtype_size(vec);
}

template <class Acc, class Vec, class Lnk>
static hub_status mtm_t(const Geom& g, Lnk lk, const void* x, void* z, void* scratch,
                        hipStream_t st) {
    const SweepPlan P = plan_sweep(g, sizeof(Vec) == 8);
    OpApply<Acc, Vec, Lnk> op{(const Vec*)x, (Vec*)z, lk};
    Acc* y = (Acc*)scratch;
    bool own = false;
    if (!P.fused && !y) {
        HUB_HIP(hipMallocAsync((void**)&y, (size_t)g.V * sizeof(Acc), st));
        own = true;
    }
    hub_status s = launch_q(g, P, op, y, nullptr, st);
    if (own) {
        hipError_t e = hipFreeAsync(y, st);
        if (s == HUB_OK && e != hipSuccess)
            return set_error(HUB_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
    }
    return s;
}

hub_status launch_apply_MtM(const Geom& g, const void* links, hub_dtype link,
                            hub_dtype vec, const void* x, void* z, void* scratch,
                            hipStream_t st) {
    if (vec == HUB_F64)
        return mtm_t<double, double>(g, Link64{(const double*)links}, x, z, scratch, st);
    if (link == HUB_F32)
        return mtm_t<float, float>(g, Link32{(const float*)links}, x, z, scratch, st);
    return mtm_t<float, float>(g, make_link16(g, links), x, z, scratch, st);
}

}  // namespace hub
