// Serving: continuous batching of CG solves (placeholder until the
// persistent multi-solve kernel lands).
#include "internal.h"

using namespace hub;

extern "C" {

hub_status hub_serve_create(const hub_serve_opts*, hub_server** out) {
    if (out) *out = nullptr;
    return set_error(HUB_E_INVALID, "serving is not available in this build");
}

hub_status hub_serve_submit(hub_server*, int32_t, const hub_lattice*, const double*,
                            const double*, uint64_t*) {
    return set_error(HUB_E_INVALID, "serving is not available in this build");
}

hub_status hub_serve_poll(hub_server*, uint64_t, double*, hub_cg_stats*) {
    return set_error(HUB_E_NOTFOUND, "serving is not available in this build");
}

hub_status hub_serve_destroy(hub_server*) { return HUB_OK; }

}  // extern "C"
