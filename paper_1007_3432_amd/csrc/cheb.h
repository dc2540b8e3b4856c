// Chebyshev polynomial preconditioner (Sec. 4.2, Eqs. (13)-(15)): host-side
// factor table and sweep launcher, shared by hub_apply_cheb and the
// preconditioned CG solve.
#pragma once

#include <vector>

#include "sweep.h"

namespace hub {

// One real quadratic factor c2 Q^2 + c1 Q + c0 (Q unnormalised).
struct ChebFactor {
    double c2, c1, c0;
};

// The n factors of P(Q / scale) in the order they are applied (into f[0..n),
// n <= 256, without heap allocation); their product is P including c_{2n}.
void cheb_factors(int n, double eps, double scale, ChebFactor* f);
std::vector<ChebFactor> cheb_factors(int n, double eps, double scale);

// Upper bound on the largest eigenvalue of Q: (1 + 2 d kappa + e^{dtau mu}(1 + b))^2.
double cheb_default_scale(const Geom& g);

// z = P r with the factors f (2 sweeps each); w: V doubles of scratch;
// yscratch: V doubles when the plan is not fused.  With dot, the last factor
// reduces r.z into sc (rho, beta); with sc == nullptr nothing is skipped.
hub_status launch_cheb(const Geom& g, const SweepPlan& P, const double* A64, CGScalars* sc,
                       const double* r, double* z, double* w, double* yscratch,
                       double* partials, const ChebFactor* f, int n, bool dot,
                       hipStream_t st);

// hub_apply_cheb (arguments already validated).
hub_status cheb_apply(const Geom& g, const double* links, const double* r, double* z,
                      const hub_cheb_opts& c, hipStream_t st);

// Size of the fixed workspace array of hub_apply_cheb_noalloc (per GPU).
constexpr size_t kNoAllocBytes = size_t(64) << 20;

// Workspace bytes hub_apply_cheb needs on this geometry.
size_t cheb_noalloc_bytes(const Geom& g);

// hub_apply_cheb_noalloc (arguments already validated): as cheb_apply, with
// the workspace in the fixed per-GPU array; allocates nothing.
hub_status cheb_apply_noalloc(const Geom& g, const double* links, const double* r, double* z,
                              const hub_cheb_opts& c, hipStream_t st);

// hub_pcg_solve (arguments already validated).
hub_status pcg_solve(const Geom& g, const double* sigma, const double* phi, double* x,
                     const hub_cg_opts& o, const hub_cheb_opts& c, hub_cg_stats* out,
                     hipStream_t st);

}  // namespace hub
