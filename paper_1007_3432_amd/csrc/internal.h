// Host-side internals of libhub shared between translation units.
#pragma once

#include <string>

#include "common.h"

namespace hub {

// Error reporting: thread-local message behind hub_last_error().
hub_status set_error(hub_status st, const char* fmt, ...)
    __attribute__((format(printf, 2, 3)));
void clear_error();

#define HUB_HIP(call)                                                        \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess)                                                \
            return ::hub::set_error(HUB_E_DEVICE, "%s failed: %s (%s:%d)",   \
                                    #call, hipGetErrorString(e_), __FILE__,  \
                                    __LINE__);                               \
    } while (0)

// Validates a lattice descriptor and fills the kernel geometry.
hub_status make_geom(const hub_lattice* lat, Geom* g);

// Bytes of one element of dtype.
size_t dtype_size(hub_dtype t);

// Accepted (vector, link) precision pairs of the apply calls.
bool valid_pair(hub_dtype vec, hub_dtype link);

// Kernel launchers (asynchronous on st; arguments already validated).
hub_status launch_links(const Geom& g, const double* sigma, void* links,
                        hub_dtype link, hipStream_t st);
hub_status launch_apply_M(const Geom& g, const void* links, hub_dtype link,
                          hub_dtype vec, const void* x, void* y, int transpose,
                          hipStream_t st);
// scratch: NULL, or at least mtm_scratch_bytes(g, vec) bytes of device memory.
hub_status launch_apply_MtM(const Geom& g, const void* links, hub_dtype link,
                            hub_dtype vec, const void* x, void* z, void* scratch,
                            hipStream_t st);
size_t mtm_scratch_bytes(const Geom& g, hub_dtype vec);

// True when Q sweeps on this geometry use the fused single-pass kernel.
bool mtm_fused(const Geom& g, hub_dtype vec);

// Blocking CG solve (arguments already validated).
hub_status cg_solve(const Geom& g, const double* sigma, const double* phi,
                    double* x, const hub_cg_opts& o, hub_cg_stats* out,
                    hipStream_t st);

// The calling thread's solver workspace, at least `bytes` long (cg.hip): kept
// between solves, grown when a solve needs more; valid until the next call
// that grows it or solver_release().  Solves only: one solve at a time per
// thread uses it.
hub_status solver_workspace(size_t bytes, char** out);
// Frees the calling thread's solver workspace and cached chunk graphs.
void solver_release();

// FP64 CG in one workgroup for lattices that fit it (cgsmall.hip).
bool cg_small_fits(const Geom& g);
hub_status cg_solve_small(const Geom& g, const double* sigma, const double* phi, double* x,
                          const hub_cg_opts& o, hub_cg_stats* out, hipStream_t st);

// HMC (hmc.hip; arguments already validated).
hub_status hmc_force(const Geom& g, const double* sigma, const double* x, double* F,
                     hipStream_t st);
hub_status md_trajectory(const Geom& g, double* sigma, double* pi, const double* phi,
                         const double* eta, const double* pi0, double u, const hub_md_opts& o,
                         hub_md_stats* out, hipStream_t st);

}  // namespace hub
