/*
 * hub.h -- C ABI of libhub, the MI355X (gfx950) library for the fermion
 * matrix of the spin-symmetric Hubbard model and for conjugate-gradient
 * solves of Q x = phi, Q = M^T M, on the (d+1)-dimensional space-time
 * lattice (Wendt, Drut, Laehde, "Toward large-scale Hybrid Monte Carlo
 * simulations of the Hubbard model on graphics processing units").
 *
 * Operator (Sec. 2: block form of M, Eq. (7); transfer blocks, Eq. (8);
 * stencil form, Eq. (10)).  Site (n, s) of a lattice with d spatial
 * dimensions of extent nx (periodic) and nt time slices (antiperiodic) has
 * linear index n + nx^d * s, n = c_0 + nx c_1 + nx^2 c_2 (c_0 fastest):
 *
 *   (M x)_{n,s}   = x_{n,s} - kappa sum_j (x_{n+e_j,s} + x_{n-e_j,s})
 *                   + A_{n,s} x_{n,s-1 mod nt}
 *   (M^T y)_{n,s} = y_{n,s} - kappa sum_j (y_{n+e_j,s} + y_{n-e_j,s})
 *                   + A_{n,s+1 mod nt} y_{n,s+1 mod nt}
 *   kappa   = dtau * t_hop
 *   A_{n,s} = -exp(dtau mu) (1 + b sin sigma_{n,s-1})  for s >= 1
 *   A_{n,0} = +exp(dtau mu) (1 + b sin sigma_{n,nt-1}) (antiperiodic wrap)
 *   b       = sqrt(2 (exp(-dtau U) - 1)), U <= 0 (compact continuous
 *             Hubbard-Stratonovich field, attractive coupling)
 *
 * i.e. Eq. (10) with B = 1/d, C = D = -dtau t and the time-link coefficient
 * A carrying the field: block row s of Eq. (7) multiplied on the left by
 * 1 + dtau K, the first-order expansion of exp(dtau K).
 *
 * Conventions for every call:
 *   - Device pointers are caller-owned device memory (hipMalloc or a torch
 *     tensor), contiguous, site-major, 16-byte aligned, and must stay valid
 *     until the stream reaches the work.  Input and output may not alias.
 *   - `stream` is a hipStream_t; NULL is the legacy default stream.
 *   - Arguments are validated before anything is launched; on any error the
 *     outputs are untouched and hub_last_error() describes the problem.
 *   - Lattice limits: 1 <= d <= 3, nx >= 2, nt >= 2, nx^d * nt <= 2^31 - 1,
 *     t_hop >= 0, dtau > 0, U <= 0, all values finite.
 *   - Precision pairs (vector dtype, link dtype) accepted by the apply calls:
 *     (HUB_F64, HUB_F64), (HUB_F32, HUB_F32), (HUB_F32, HUB_F16).
 *   - The solvers (hub_cg_solve, hub_pcg_solve, the HMC calls) run on the
 *     device current on the calling host thread; a host thread keeps to one
 *     device for them (a solve on another device returns HUB_E_INVALID;
 *     use another thread).
 *   - No C++ exception crosses this interface.
 */
#ifndef HUB_H
#define HUB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HUB_API __attribute__((visibility("default")))

typedef enum {
    HUB_OK = 0,
    HUB_PENDING = 1,      /* serve: the ticket's solve has not finished */
    HUB_E_INVALID = -1,   /* bad descriptor, pointer, dtype, option */
    HUB_E_NOMEM = -2,     /* allocation failed, or larger than a budget */
    HUB_E_NOCONV = -3,    /* max_iter reached, CG breakdown, NaN/Inf */
    HUB_E_DEVICE = -4,    /* a HIP runtime call failed */
    HUB_E_NOTFOUND = -5   /* serve: unknown or already retired ticket */
} hub_status;

typedef enum { HUB_F64 = 0, HUB_F32 = 1, HUB_F16 = 2 } hub_dtype;

typedef struct {
    int32_t d;        /* spatial dimensions, 1..3 */
    int32_t nx;       /* spatial extent in every direction (periodic), >= 2 */
    int32_t nt;       /* time slices (antiperiodic), >= 2 */
    int32_t reserved; /* must be 0 */
    double t_hop;     /* hopping t >= 0 */
    double dtau;      /* Trotter step > 0 */
    double U;         /* on-site coupling <= 0 */
    double mu;        /* chemical potential */
} hub_lattice;

typedef struct {
    hub_dtype bulk;          /* HUB_F64: plain CG; HUB_F32: mixed CG */
    hub_dtype link;          /* links of the bulk operator: F64 (with bulk
                                F64), F32 or F16 (with bulk F32) */
    double tol;              /* stop when |phi - Q x|_2 / |phi|_2 <= tol,
                                evaluated in FP64 on the true residual */
    int32_t max_iter;        /* iteration cap, >= 1 */
    int32_t reliable_every;  /* mixed: FP64 residual recompute period, >= 1 */
} hub_cg_opts;

typedef struct {
    int32_t iters;            /* CG iterations performed */
    int32_t reliable_updates; /* FP64 true-residual recomputes */
    double true_rel_resid;    /* |phi - Q x|_2 / |phi|_2 in FP64 at exit */
    double ms;                /* wall time of the call (device-timed) */
    int32_t status;           /* hub_status of the solve */
    int32_t reserved;
} hub_cg_stats;

/* Time-link coefficients from the auxiliary field (Sec. 2, Eqs. (8), (10)).
 * sigma: device, FP64[nx^d * nt], sigma[n + nx^d s] is the field on slice s.
 * links: device, written with nx^d * nt elements of `link`:
 *   HUB_F64 / HUB_F32: the sign-folded A_{n,s} above;
 *   HUB_F16: s_{n,s} = sin(sigma_{n,s-1 mod nt}) rounded to nearest, from
 *            which the stencil rebuilds A = -+exp(dtau mu)(1 + b s) in FP32.
 * Asynchronous on `stream`. */
HUB_API hub_status hub_links_from_sigma(const hub_lattice* lat, const double* sigma,
                                void* links, hub_dtype link, void* stream);

/* y = M x (transpose = 0) or y = M^T x (transpose = 1), Eq. (10).
 * links: from hub_links_from_sigma with dtype `link`; x, y: device,
 * nx^d * nt elements of `vec`.  Asynchronous on `stream`. */
HUB_API hub_status hub_apply_M(const hub_lattice* lat, const void* links,
                       hub_dtype link, hub_dtype vec, const void* x, void* y,
                       int transpose, void* stream);

/* z = M^T (M x) in one fused pass: the matrix-vector operation with
 * Q = M^T M of Sec. 4.2/4.3.  Same argument rules as hub_apply_M.
 * Asynchronous on `stream`. */
HUB_API hub_status hub_apply_MtM(const hub_lattice* lat, const void* links,
                         hub_dtype link, hub_dtype vec, const void* x, void* z,
                         void* stream);

/* Solve (M^T M) x = phi by conjugate gradient from x = 0 (Sec. 4.1).
 * sigma, phi: device FP64[nx^d * nt]; x: device FP64[nx^d * nt], output.
 * opts->bulk = HUB_F64: Hestenes-Stiefel CG in FP64 throughout.
 * opts->bulk = HUB_F32: mixed precision with reliable updates: vectors r, p,
 *   q and the correction x_lo in FP32, links per opts->link, dot products
 *   accumulated in FP64; every opts->reliable_every iterations (and whenever
 *   the iterated residual meets tol) x += x_lo is folded into the FP64
 *   solution and r is replaced by the FP64 true residual phi - Q x.
 * Convergence is always decided on the FP64 true residual.  With bulk =
 * HUB_F64 on a lattice of at most 2048 sites the whole solve runs in one
 * workgroup (one kernel launch, no graphs); otherwise each iteration is a few
 * kernels replayed in chunks from HIP graphs.  The device workspace (about
 * five V-vectors of `bulk` plus the links) and the chunk graphs are kept per
 * host thread after the call: the next solve on that thread reuses the
 * workspace when it is large enough (else frees it and allocates a larger
 * one, which synchronizes the device) and replays the graphs when lattice,
 * options, phi and x are the same (else captures them again).
 * hub_solver_release frees them.  Blocks until done, and until `stream` has
 * drained.  stats.reliable_updates counts the true-residual recomputes.
 * Returns HUB_OK, or HUB_E_NOCONV with x holding the last iterate and
 * `out` filled; `out` may be NULL. */
HUB_API hub_status hub_cg_solve(const hub_lattice* lat, const double* sigma,
                        const double* phi, double* x, const hub_cg_opts* opts,
                        hub_cg_stats* out, void* stream);

/* ---- Chebyshev polynomial preconditioning (Sec. 4.2, Eqs. (13)-(17)) ----
 * P(Q) = c_{2n} prod_{k=1}^{2n} (Q/scale - z_{2n,k}), with the roots
 * z_{2n,k} = (1+eps)/2 [1 - cos(2 pi k/(2n+1))] - i sqrt(eps) sin(2 pi k/(2n+1))
 * and 1/c_{2n} = (1+eps)/2 prod_k ((1+eps)/2 - z_{2n,k}), approximates
 * scale * Q^{-1} with relative error at most 2((1-sqrt eps)/(1+sqrt eps))^{2n+1}
 * on the eigenvalues of Q/scale in (eps, 1] (Eq. (16)).  P is positive for
 * every real argument, so P(Q) is symmetric positive definite whatever the
 * spectrum; eps and scale only affect how well it approximates. */
typedef struct {
    int32_t n;        /* half the polynomial degree, 1 <= n <= 256: P(Q) costs
                         2n applications of Q */
    int32_t reserved; /* must be 0 */
    double eps;       /* lower end of the approximation interval, 0 < eps < 1 */
    double scale;     /* normalisation of Q; <= 0 selects the bound
                         (1 + 2 d dtau t + e^{dtau mu}(1 + b))^2 >= lambda_max(Q) */
} hub_cheb_opts;

/* z = P(Q) r.  links: FP64 time links (hub_links_from_sigma, HUB_F64);
 * r, z: device FP64[nx^d * nt], distinct.  The conjugate root pairs are
 * applied as n real quadratic factors, two fused M^T M sweeps each.
 * Asynchronous on `stream` (allocates one V-vector of workspace
 * stream-ordered). */
HUB_API hub_status hub_apply_cheb(const hub_lattice* lat, const double* links,
                          const double* r, double* z, const hub_cheb_opts* cheb,
                          void* stream);

/* z = P(Q) r exactly as hub_apply_cheb (same kernels, same factor order,
 * bitwise the same result), for callers that cannot allocate: code under HIP
 * graph capture, serving loops, harnesses that forbid allocation.  The
 * workspace (one FP64 vector of nx^d * nt elements, two when the lattice has
 * no fused sweep: d = 2, or d = 3 with nx not in {8, 16, 32, 64}) lives in a
 * fixed 64 MiB device array that the library holds on every GPU it runs on
 * until the process ends; no device or host memory is allocated by the call.
 * Lattices whose workspace exceeds 64 MiB (more than 8 388 608 sites, or
 * 4 194 304 without a fused sweep) are rejected with HUB_E_NOMEM before
 * anything is launched.  All calls on one GPU share that array: calls that
 * overlap in time on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  Asynchronous on `stream`. */
HUB_API hub_status hub_apply_cheb_noalloc(const hub_lattice* lat, const double* links,
                                  const double* r, double* z, const hub_cheb_opts* cheb,
                                  void* stream);

/* Solve (M^T M) x = phi by conjugate gradient preconditioned with P(Q)
 * (Sec. 4.2; the preconditioned CG of Sec. 5), from x = 0, in FP64:
 * opts->bulk and opts->link must be HUB_F64.  Convergence is decided on
 * |r| <= tol |phi| and confirmed on the FP64 true residual; a failed
 * confirmation restarts from the true residual.  stats->iters counts CG
 * iterations (each costs 2n + 1 applications of Q).  Blocks until done;
 * keeps its workspace and graphs, and returns, as hub_cg_solve. */
HUB_API hub_status hub_pcg_solve(const hub_lattice* lat, const double* sigma,
                         const double* phi, double* x, const hub_cg_opts* opts,
                         const hub_cheb_opts* cheb, hub_cg_stats* out,
                         void* stream);

/* ---- Hybrid Monte Carlo, the phi-algorithm (Sec. 4.1) --------------------
 * (det M)^2 = det Q is represented by a pseudofermion field phi with action
 * S_p = phi^T Q^{-1} phi (Sec. 4.1).  The compact field sigma has a flat
 * measure, so the MD Hamiltonian of sigma and its momenta pi is
 *   H = 1/2 pi.pi + S_p,   S_p = phi . x,   x = Q^{-1} phi,
 * and the force is (sigma_{n,s} enters M only through A_{n,s+1 mod nt})
 *   dS_p/dsigma_{n,s} = -2 (M x)_{n,s+1} (dA_{n,s+1}/dsigma_{n,s}) x_{n,s},
 *   dA_{n,s+1}/dsigma_{n,s} = -+ exp(dtau mu) b cos sigma_{n,s}  (+ on the wrap). */

/* force[i] = dS_p/dsigma_i at every site, for x = Q^{-1} phi (any x is
 * accepted: the formula is evaluated as written).  sigma, x, force: device
 * FP64[nx^d * nt]; force distinct from both inputs.  Asynchronous. */
HUB_API hub_status hub_hmc_force(const hub_lattice* lat, const double* sigma, const double* x,
                         double* force, void* stream);

typedef struct {
    int32_t n_steps;  /* leapfrog steps per trajectory, >= 1 */
    int32_t reserved; /* must be 0 */
    double eps;       /* MD step size, finite and > 0 */
    hub_cg_opts cg;   /* solver of every force evaluation (as hub_cg_solve) */
} hub_md_opts;

typedef struct {
    double h_start;   /* H at the start of the trajectory */
    double h_end;     /* H at its end */
    int32_t solves;   /* CG solves = force evaluations (n_steps + 1) */
    int32_t cg_iters; /* CG iterations over all solves */
    int32_t accepted; /* hub_hmc_trajectory: Metropolis decision */
    int32_t status;   /* hub_status of the call */
} hub_md_stats;

/* One leapfrog MD trajectory from (sigma, pi), both device FP64[V] updated in
 * place: pi -= eps/2 F; then n_steps times { sigma += eps pi; solve
 * Q x = phi; pi -= eps F } with the last kick halved.  Every force
 * evaluation solves Q x = phi from x = 0 with opts->cg (the same solver as
 * hub_cg_solve).  phi: device FP64[V].  Blocks until done.  HUB_E_NOCONV if
 * a solve fails: the trajectory stops there, sigma and pi hold the point
 * reached. */
HUB_API hub_status hub_md_trajectory(const hub_lattice* lat, double* sigma, double* pi,
                             const double* phi, const hub_md_opts* opts,
                             hub_md_stats* out, void* stream);

/* One HMC trajectory: the pseudofermion heatbath phi = M^T eta at the
 * starting field, the MD trajectory of hub_md_trajectory from (sigma, pi0)
 * on copies, and the Metropolis step: the end point replaces sigma when
 * u < exp(-(H_end - H_start)); otherwise sigma is left untouched.  The
 * random numbers come from the caller: eta (device FP64[V], density
 * exp(-eta.eta), i.e. variance 1/2 per component), pi0 (device FP64[V],
 * standard normal; not modified), u (uniform on [0, 1)).  Blocks until done;
 * a failed solve returns HUB_E_NOCONV with sigma untouched. */
HUB_API hub_status hub_hmc_trajectory(const hub_lattice* lat, double* sigma, const double* eta,
                              const double* pi0, double u, const hub_md_opts* opts,
                              hub_md_stats* out, void* stream);

/* ---- Serving: continuous batching of CG solves from many HMC chains ----
 * A server owns one worker thread, one HIP stream and the resident state of
 * every chain it has seen (field, links, Krylov vectors).  Requests are
 * admitted while their footprint fits hbm_budget_bytes and a slot is free;
 * admitted solves step together on the device (all in-flight solves in each
 * launch, or in one persistent kernel), newly
 * admitted ones join between epochs (reliable_every iterations plus the
 * reliable update), finished ones leave.  Every solve takes exactly the
 * steps of hub_cg_solve with the same options, so its result is the same
 * alone and in the mix. */
typedef struct hub_server hub_server;

typedef struct {
    size_t hbm_budget_bytes; /* cap on resident chain + solve memory */
    int32_t max_inflight;    /* cap on concurrently stepped solves, >= 1 */
    int32_t engine;          /* 0: one launch per CG phase for all in-flight
                                solves, kernel boundaries as the device-wide
                                sync (default); 1: one persistent cooperative
                                kernel per epoch with grid barriers */
    hub_cg_opts cg;          /* solver options (bulk must be HUB_F32) */
} hub_serve_opts;

HUB_API hub_status hub_serve_create(const hub_serve_opts* opts, hub_server** out);

/* Queue a solve for chain `chain_id` on lattice `lat`.  sigma_host: host
 * FP64[V], the chain's new field, or NULL to reuse the field of the chain's
 * previous request (same lattice required).  phi_host: host FP64[V].  Both
 * are copied before the call returns.  Writes a ticket; non-blocking.
 * HUB_E_NOMEM if the request alone exceeds the budget. */
HUB_API hub_status hub_serve_submit(hub_server* srv, int32_t chain_id,
                            const hub_lattice* lat, const double* sigma_host,
                            const double* phi_host, uint64_t* ticket);

/* HUB_PENDING while the solve runs; otherwise copies x (host FP64[V]) and
 * the stats out once and retires the ticket, returning the solve's status.
 * HUB_E_NOTFOUND for an unknown or retired ticket.  x_host or out may be
 * NULL. */
HUB_API hub_status hub_serve_poll(hub_server* srv, uint64_t ticket, double* x_host,
                          hub_cg_stats* out);

/* Stops the worker after the in-flight solves finish and frees everything. */
HUB_API hub_status hub_serve_destroy(hub_server* srv);

/* Frees the solver workspace and chunk graphs that hub_cg_solve,
 * hub_pcg_solve and the HMC calls keep for the calling host thread (see
 * hub_cg_solve).  Safe to call at any time between calls; the next solve
 * allocates again.  Returns HUB_OK. */
HUB_API hub_status hub_solver_release(void);

/* Message for the last error on the calling thread ("" if none). */
HUB_API const char* hub_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HUB_H */
