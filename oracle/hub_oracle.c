/*
 * hub_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, obviously correct FP64 CPU implementation of the fermion
 * matrix of the spin-symmetric Hubbard model on a (d+1)-dimensional
 * space-time lattice (Wendt, Drut, Laehde, "Toward large-scale Hybrid Monte
 * Carlo simulations of the Hubbard model on graphics processing units"), and
 * of conjugate gradient on Q = M^T M.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may call it.  It shares no code,
 * header or constant with the GPU library.
 *
 * Conventions (the readings of the paper that this file fixes):
 *   - lattice: d spatial dimensions of extent nx (periodic), nt time slices
 *     (antiperiodic), Sec. 2 after Eq. (10);
 *   - site (n, tau) has linear index n + Vs*tau with Vs = nx^d, and the
 *     spatial index n = c_0 + nx*c_1 + nx^2*c_2 (coordinate c_0 fastest);
 *   - slices are 0-based: slice s of this file is slice s+1 of the block
 *     matrix M of Sec. 2, Eq. (7);
 *   - the auxiliary-field factor exp(-dtau V[sigma]) of Eq. (8) is the
 *     compact continuous Hubbard-Stratonovich form diag(1 + b sin sigma) with
 *     b = sqrt(2 (exp(-dtau U) - 1)), U <= 0 (attractive, Sec. 2 after
 *     Eq. (10)); a chemical potential multiplies it by exp(dtau mu);
 *   - the operator is the stencil form of M, Eq. (10), obtained by
 *     multiplying block row s of Eq. (7) on the left by (1 + dtau K), the
 *     first-order expansion of exp(dtau K); this yields Eq. (10) with
 *     coefficients B = 1/d, C = D = -dtau t and the time-link coefficient
 *     A carrying all the sigma dependence:
 *
 *       (M x)_{n,s} = x_{n,s} - kappa sum_j (x_{n+e_j,s} + x_{n-e_j,s})
 *                     + A_{n,s} x_{n,s-1 mod nt}
 *       kappa   = dtau t
 *       A_{n,s} = -exp(dtau mu) (1 + b sin sigma_{n,s-1})   for s >= 1
 *       A_{n,0} = +exp(dtau mu) (1 + b sin sigma_{n,nt-1})  (the +B_{N_tau}
 *                  wrap of Eq. (7): antiperiodic time boundary)
 *
 *     Row s of M_paper holds -B_{s} x_{s-1} with B_s built from the field
 *     on slice s-1 (0-based), which is why A_{n,s} reads sigma_{n,s-1}.
 *
 *   - M^T follows by transposition:
 *       (M^T y)_{n,s} = y_{n,s} - kappa sum_j (y_{n+e_j,s} + y_{n-e_j,s})
 *                       + A_{n,s+1 mod nt} y_{n,s+1 mod nt}
 *   - Q = M^T M (Sec. 4.1, after Eq. (12)) is applied as M^T(M x).
 *
 * Conjugate gradient (Sec. 4.1: "solution of the linear problem Qx = b" by
 * CG) is the textbook Hestenes-Stiefel recurrence with x0 = 0, stopped when
 * the true residual |phi - Q x|_2 / |phi|_2 <= tol.  Dot products are summed
 * serially in index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t d;      /* spatial dimensions, 1..3 */
    int32_t nx;     /* spatial extent (all directions), >= 2 */
    int32_t nt;     /* time slices, >= 2 */
    int32_t pad;
    double t_hop;   /* hopping t */
    double dtau;    /* Trotter step */
    double U;       /* on-site coupling, <= 0 */
    double mu;      /* chemical potential */
} oracle_lattice;

typedef struct {
    int32_t iters;          /* CG iterations performed */
    int32_t converged;      /* 1 if the true residual met tol */
    int32_t breakdown;      /* 1 if p.Qp <= 0 or not finite */
    int32_t restarts;       /* times the iterated residual was replaced */
    double true_rel_resid;  /* |phi - Qx| / |phi| at exit */
    double iter_rel_resid;  /* sqrt(r.r) / |phi| of the recurrence at exit */
} oracle_cg_result;

static long spatial_volume(const oracle_lattice* L) {
    long v = 1;
    for (int j = 0; j < L->d; ++j) v *= L->nx;
    return v;
}

long oracle_volume(const oracle_lattice* L) {
    return spatial_volume(L) * (long)L->nt;
}

/* Index of n + step*e_j (step = +1 or -1), periodic in every spatial
 * direction. */
static long spatial_shift(const oracle_lattice* L, long n, int j, int step) {
    long stride = 1;
    for (int k = 0; k < j; ++k) stride *= L->nx;
    long c = (n / stride) % L->nx;
    long c2 = (c + step + L->nx) % L->nx;
    return n + (c2 - c) * stride;
}

/* b of the compact Hubbard-Stratonovich transform: the identity
 * (1/2pi) Int dsigma (1 + b sin sigma n_up)(1 + b sin sigma n_dn)
 *     = exp(-dtau U n_up n_dn)                 (n in {0,1})
 * fixes b^2 / 2 = exp(-dtau U) - 1.  Returns NaN for U > 0. */
double oracle_hs_coupling(double dtau, double U) {
    double e = exp(-dtau * U) - 1.0;
    if (e < 0.0) return NAN;
    return sqrt(2.0 * e);
}

/* A[n + Vs*s] from sigma[n + Vs*s], as in the header comment. */
void oracle_links(const oracle_lattice* L, const double* sigma, double* A) {
    long Vs = spatial_volume(L);
    double b = oracle_hs_coupling(L->dtau, L->U);
    double scale = exp(L->dtau * L->mu);
    for (long s = 0; s < L->nt; ++s) {
        long sm = (s - 1 + L->nt) % L->nt;
        double sign = (s == 0) ? 1.0 : -1.0;
        for (long n = 0; n < Vs; ++n)
            A[n + Vs * s] = sign * scale * (1.0 + b * sin(sigma[n + Vs * sm]));
    }
}

/* y = M x. */
void oracle_apply_M(const oracle_lattice* L, const double* A, const double* x,
                    double* y) {
    long Vs = spatial_volume(L);
    double kappa = L->dtau * L->t_hop;
#pragma omp parallel for schedule(static) if (Vs * L->nt >= 65536)
    for (long s = 0; s < L->nt; ++s) {
        long sm = (s - 1 + L->nt) % L->nt;
        for (long n = 0; n < Vs; ++n) {
            double hop = 0.0;
            for (int j = 0; j < L->d; ++j) {
                hop += x[spatial_shift(L, n, j, +1) + Vs * s];
                hop += x[spatial_shift(L, n, j, -1) + Vs * s];
            }
            long i = n + Vs * s;
            y[i] = x[i] - kappa * hop + A[i] * x[n + Vs * sm];
        }
    }
}

/* z = M^T y. */
void oracle_apply_Mt(const oracle_lattice* L, const double* A, const double* y,
                     double* z) {
    long Vs = spatial_volume(L);
    double kappa = L->dtau * L->t_hop;
#pragma omp parallel for schedule(static) if (Vs * L->nt >= 65536)
    for (long s = 0; s < L->nt; ++s) {
        long sp = (s + 1) % L->nt;
        for (long n = 0; n < Vs; ++n) {
            double hop = 0.0;
            for (int j = 0; j < L->d; ++j) {
                hop += y[spatial_shift(L, n, j, +1) + Vs * s];
                hop += y[spatial_shift(L, n, j, -1) + Vs * s];
            }
            long i = n + Vs * s;
            z[i] = y[i] - kappa * hop + A[n + Vs * sp] * y[n + Vs * sp];
        }
    }
}

/* z = M^T (M x), using caller-provided scratch tmp of the lattice volume. */
void oracle_apply_MtM(const oracle_lattice* L, const double* A, const double* x,
                      double* z, double* tmp) {
    oracle_apply_M(L, A, x, tmp);
    oracle_apply_Mt(L, A, tmp, z);
}

/* Serial dot product in index order. */
double oracle_dot(long n, const double* a, const double* b) {
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Conjugate gradient on Q x = phi, Q = M^T M, x0 = 0.  On exit x holds the
 * last iterate.  If alphas / betas are non-NULL (max_iter entries each) the
 * step lengths alpha_k and coefficients beta_k of every iteration are
 * recorded; they define the Lanczos tridiagonal of Q on the Krylov space.
 * Work arrays are allocated here.  Returns 0 if converged, 1 if max_iter was
 * reached or CG broke down, -1 on allocation failure. */
int oracle_cg(const oracle_lattice* L, const double* A, const double* phi,
              double* x, double tol, int32_t max_iter, oracle_cg_result* res,
              double* alphas, double* betas) {
    long V = oracle_volume(L);
    double* r = (double*)malloc(sizeof(double) * V);
    double* p = (double*)malloc(sizeof(double) * V);
    double* q = (double*)malloc(sizeof(double) * V);
    double* tmp = (double*)malloc(sizeof(double) * V);
    if (!r || !p || !q || !tmp) {
        free(r); free(p); free(q); free(tmp);
        return -1;
    }
    memset(res, 0, sizeof(*res));
    double phinorm = sqrt(oracle_dot(V, phi, phi));
    for (long i = 0; i < V; ++i) {
        x[i] = 0.0;
        r[i] = phi[i];
        p[i] = phi[i];
    }
    double rho = oracle_dot(V, r, r);
    int status = 1;
    if (phinorm == 0.0) {
        res->converged = 1;
        status = 0;
        goto out;
    }
    for (int32_t k = 1; k <= max_iter; ++k) {
        oracle_apply_MtM(L, A, p, q, tmp);
        double pq = oracle_dot(V, p, q);
        res->iters = k;
        if (!(pq > 0.0) || !isfinite(pq)) {
            res->breakdown = 1;
            break;
        }
        double alpha = rho / pq;
        if (alphas) alphas[k - 1] = alpha;
        for (long i = 0; i < V; ++i) x[i] += alpha * p[i];
        for (long i = 0; i < V; ++i) r[i] -= alpha * q[i];
        double rho_new = oracle_dot(V, r, r);
        if (!isfinite(rho_new)) {
            res->breakdown = 1;
            break;
        }
        if (sqrt(rho_new) / phinorm <= tol) {
            /* Confirm on the true residual; continue from it otherwise. */
            oracle_apply_MtM(L, A, x, q, tmp);
            for (long i = 0; i < V; ++i) r[i] = phi[i] - q[i];
            rho_new = oracle_dot(V, r, r);
            if (sqrt(rho_new) / phinorm <= tol) {
                res->converged = 1;
                status = 0;
                break;
            }
            res->restarts += 1;
        }
        double beta = rho_new / rho;
        if (betas) betas[k - 1] = beta;
        for (long i = 0; i < V; ++i) p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }
out:
    res->iter_rel_resid = (phinorm > 0.0) ? sqrt(oracle_dot(V, r, r)) / phinorm : 0.0;
    oracle_apply_MtM(L, A, x, q, tmp);
    for (long i = 0; i < V; ++i) q[i] = phi[i] - q[i];
    res->true_rel_resid = (phinorm > 0.0) ? sqrt(oracle_dot(V, q, q)) / phinorm : 0.0;
    free(r); free(p); free(q); free(tmp);
    return status;
}

/* ---------------------------------------------------------------------------
 * Chebyshev polynomial preconditioner (Sec. 4.2, Eqs. (13)-(15)).
 *
 * With Q normalised so that its eigenvalues lie in [0, 1] (Qn = Q / scale),
 *   P(Qn) = c_{2n} prod_{k=1}^{2n} (Qn - z_{2n,k})
 *   z_{2n,k} = (1+eps)/2 [1 - cos(2 pi k/(2n+1))] - i sqrt(eps) sin(2 pi k/(2n+1))
 *   1/c_{2n} = (1+eps)/2 prod_{k=1}^{2n} ((1+eps)/2 - z_{2n,k})
 * approximates Qn^{-1} on (eps, 1].  The oracle applies the 2n complex
 * linear factors one after the other, k = 1 .. 2n, on a complex vector. */

void oracle_cheb_roots(int32_t n, double eps, double* re, double* im) {
    const double pi = 3.14159265358979323846;
    for (int32_t k = 1; k <= 2 * n; ++k) {
        double th = 2.0 * pi * (double)k / (double)(2 * n + 1);
        re[k - 1] = 0.5 * (1.0 + eps) * (1.0 - cos(th));
        im[k - 1] = -sqrt(eps) * sin(th);
    }
}

/* c_{2n} (real: the roots come in conjugate pairs). */
double oracle_cheb_norm(int32_t n, double eps) {
    double* re = (double*)malloc(sizeof(double) * 2 * n);
    double* im = (double*)malloc(sizeof(double) * 2 * n);
    if (!re || !im) { free(re); free(im); return NAN; }
    oracle_cheb_roots(n, eps, re, im);
    double h = 0.5 * (1.0 + eps);
    double pr = h, pi_ = 0.0;   /* running complex product, starts at (1+eps)/2 */
    for (int32_t k = 0; k < 2 * n; ++k) {
        double ar = h - re[k], ai = -im[k];
        double nr = pr * ar - pi_ * ai, ni = pr * ai + pi_ * ar;
        pr = nr;
        pi_ = ni;
    }
    free(re);
    free(im);
    return 1.0 / pr;
}

/* z = P(Q / scale) r. */
int oracle_cheb_apply(const oracle_lattice* L, const double* A, double scale, int32_t n,
                      double eps, const double* r, double* z) {
    long V = oracle_volume(L);
    double* vr = (double*)malloc(sizeof(double) * V);
    double* vi = (double*)malloc(sizeof(double) * V);
    double* qr = (double*)malloc(sizeof(double) * V);
    double* qi = (double*)malloc(sizeof(double) * V);
    double* tmp = (double*)malloc(sizeof(double) * V);
    double* re = (double*)malloc(sizeof(double) * 2 * n);
    double* im = (double*)malloc(sizeof(double) * 2 * n);
    if (!vr || !vi || !qr || !qi || !tmp || !re || !im) {
        free(vr); free(vi); free(qr); free(qi); free(tmp); free(re); free(im);
        return -1;
    }
    oracle_cheb_roots(n, eps, re, im);
    double c = oracle_cheb_norm(n, eps);
    for (long i = 0; i < V; ++i) { vr[i] = r[i]; vi[i] = 0.0; }
    for (int32_t k = 0; k < 2 * n; ++k) {
        /* v <- (Qn - z_k) v, complex v = vr + i vi, real Qn */
        oracle_apply_MtM(L, A, vr, qr, tmp);
        oracle_apply_MtM(L, A, vi, qi, tmp);
        for (long i = 0; i < V; ++i) {
            double ar = qr[i] / scale - (re[k] * vr[i] - im[k] * vi[i]);
            double ai = qi[i] / scale - (re[k] * vi[i] + im[k] * vr[i]);
            vr[i] = ar;
            vi[i] = ai;
        }
    }
    for (long i = 0; i < V; ++i) z[i] = c * vr[i];
    free(vr); free(vi); free(qr); free(qi); free(tmp); free(re); free(im);
    return 0;
}

/* Preconditioned CG on Q x = phi with z = P(Q / scale) r (Sec. 4.2), x0 = 0,
 * stopped on the true residual as oracle_cg.  Returns as oracle_cg. */
int oracle_pcg(const oracle_lattice* L, const double* A, const double* phi, double* x,
               double tol, int32_t max_iter, double scale, int32_t n, double eps,
               oracle_cg_result* res) {
    long V = oracle_volume(L);
    double* r = (double*)malloc(sizeof(double) * V);
    double* z = (double*)malloc(sizeof(double) * V);
    double* p = (double*)malloc(sizeof(double) * V);
    double* q = (double*)malloc(sizeof(double) * V);
    double* tmp = (double*)malloc(sizeof(double) * V);
    if (!r || !z || !p || !q || !tmp) {
        free(r); free(z); free(p); free(q); free(tmp);
        return -1;
    }
    memset(res, 0, sizeof(*res));
    double phinorm = sqrt(oracle_dot(V, phi, phi));
    for (long i = 0; i < V; ++i) {
        x[i] = 0.0;
        r[i] = phi[i];
    }
    int status = 1;
    if (phinorm == 0.0) {
        res->converged = 1;
        status = 0;
        goto out;
    }
    if (oracle_cheb_apply(L, A, scale, n, eps, r, z) != 0) { status = -1; goto out; }
    for (long i = 0; i < V; ++i) p[i] = z[i];
    double rho = oracle_dot(V, r, z);
    for (int32_t k = 1; k <= max_iter; ++k) {
        oracle_apply_MtM(L, A, p, q, tmp);
        double pq = oracle_dot(V, p, q);
        res->iters = k;
        if (!(pq > 0.0) || !isfinite(pq)) { res->breakdown = 1; break; }
        double alpha = rho / pq;
        for (long i = 0; i < V; ++i) x[i] += alpha * p[i];
        for (long i = 0; i < V; ++i) r[i] -= alpha * q[i];
        double rr = oracle_dot(V, r, r);
        if (!isfinite(rr)) { res->breakdown = 1; break; }
        int restart = 0;
        if (sqrt(rr) / phinorm <= tol) {
            oracle_apply_MtM(L, A, x, q, tmp);
            for (long i = 0; i < V; ++i) r[i] = phi[i] - q[i];
            rr = oracle_dot(V, r, r);
            if (sqrt(rr) / phinorm <= tol) { res->converged = 1; status = 0; break; }
            res->restarts += 1;
            restart = 1;
        }
        if (oracle_cheb_apply(L, A, scale, n, eps, r, z) != 0) { status = -1; break; }
        double rho_new = oracle_dot(V, r, z);
        double beta = restart ? 0.0 : rho_new / rho;
        for (long i = 0; i < V; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }
out:
    res->iter_rel_resid = (phinorm > 0.0) ? sqrt(oracle_dot(V, r, r)) / phinorm : 0.0;
    oracle_apply_MtM(L, A, x, q, tmp);
    for (long i = 0; i < V; ++i) q[i] = phi[i] - q[i];
    res->true_rel_resid = (phinorm > 0.0) ? sqrt(oracle_dot(V, q, q)) / phinorm : 0.0;
    free(r); free(z); free(p); free(q); free(tmp);
    return status;
}

/* Number of OpenMP threads the stencil loops use (1 without OpenMP). */
int oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Hybrid Monte Carlo, phi-algorithm (Sec. 4.1).
 *
 * (det M)^2 = det Q = Int Dphi exp(-S_p) with S_p = phi^T Q^{-1} phi, Q = M^T M
 * (Sec. 4.1).  The compact field sigma has a flat measure on [-pi, pi), so
 * the local action S_g of Eq. (5) vanishes and the molecular dynamics (MD)
 * Hamiltonian of the field and its conjugate momenta pi is
 *   H(sigma, pi) = 1/2 sum pi^2 + S_p(sigma),   S_p = phi . x,   x = Q^{-1} phi.
 * Force.  dS_p/dsigma = -x^T (dQ/dsigma) x = -2 (M x)^T (dM/dsigma) x, and
 * sigma_{n,s} enters M only through the time link A_{n,s+1} (row s+1 of M
 * reads the field of slice s), so with y = M x
 *   dS_p/dsigma_{n,s} = -2 y_{n,s'} (dA_{n,s'}/dsigma_{n,s}) x_{n,s},  s' = s+1 mod nt,
 *   dA_{n,s'}/dsigma_{n,s} = -+ exp(dtau mu) b cos sigma_{n,s}  (+ when s' = 0).
 * MD: the leapfrog integrator (half step in pi, alternating full steps in
 * sigma and pi, closing half step in pi); every force evaluation solves
 * Q x = phi by oracle_cg from x = 0.  Metropolis: the end point is accepted
 * when u < exp(-(H_end - H_start)), u uniform on [0, 1) supplied by the
 * caller; otherwise sigma returns to its start.  The pseudofermion heatbath
 * phi = M^T eta takes eta from the caller (density exp(-eta.eta), i.e.
 * variance 1/2 per component, so that phi has density exp(-S_p)).
 */

typedef struct {
    double h_start;      /* H at the start of the trajectory */
    double h_end;        /* H at its end */
    int32_t solves;      /* CG solves (force evaluations) */
    int32_t cg_iters;    /* CG iterations over all solves */
    int32_t accepted;    /* Metropolis decision */
    int32_t failed;      /* a CG solve did not converge */
} oracle_md_result;

/* F[n + Vs s] = dS_p/dsigma_{n,s} for x = Q^{-1} phi. */
void oracle_force(const oracle_lattice* L, const double* sigma, const double* x, double* F) {
    long Vs = spatial_volume(L);
    long V = oracle_volume(L);
    double* A = (double*)malloc(sizeof(double) * V);
    double* y = (double*)malloc(sizeof(double) * V);
    if (!A || !y) {
        free(A); free(y);
        for (long i = 0; i < V; ++i) F[i] = NAN;
        return;
    }
    oracle_links(L, sigma, A);
    oracle_apply_M(L, A, x, y);
    double b = oracle_hs_coupling(L->dtau, L->U);
    double scale = exp(L->dtau * L->mu);
    for (long s = 0; s < L->nt; ++s) {
        long sp = (s + 1) % L->nt;
        double sign = (sp == 0) ? 1.0 : -1.0;
        for (long n = 0; n < Vs; ++n) {
            double dA = sign * scale * b * cos(sigma[n + Vs * s]);
            F[n + Vs * s] = -2.0 * y[n + Vs * sp] * dA * x[n + Vs * s];
        }
    }
    free(A);
    free(y);
}

/* Solve Q(sigma) x = phi and return S_p = phi . x; adds the iterations to
 * *iters; sets *failed when the solve did not converge. */
static double md_solve(const oracle_lattice* L, const double* sigma, const double* phi,
                       double* x, double* A, double tol, int32_t max_iter, int32_t* iters,
                       int32_t* failed) {
    long V = oracle_volume(L);
    oracle_cg_result res;
    oracle_links(L, sigma, A);
    int rc = oracle_cg(L, A, phi, x, tol, max_iter, &res, NULL, NULL);
    *iters += res.iters;
    if (rc != 0) *failed = 1;
    return oracle_dot(V, phi, x);
}

/* One MD trajectory of n_steps leapfrog steps of size eps from (sigma, pi),
 * both updated in place; fills h_start, h_end, solves, cg_iters, failed.
 * Returns 0, or -1 on allocation failure. */
int oracle_md(const oracle_lattice* L, double* sigma, double* pi, const double* phi, double eps,
              int32_t n_steps, double tol, int32_t max_iter, oracle_md_result* res) {
    long V = oracle_volume(L);
    double* x = (double*)malloc(sizeof(double) * V);
    double* A = (double*)malloc(sizeof(double) * V);
    double* F = (double*)malloc(sizeof(double) * V);
    if (!x || !A || !F) {
        free(x); free(A); free(F);
        return -1;
    }
    memset(res, 0, sizeof(*res));
    double sp = md_solve(L, sigma, phi, x, A, tol, max_iter, &res->cg_iters, &res->failed);
    res->solves = 1;
    res->h_start = 0.5 * oracle_dot(V, pi, pi) + sp;
    oracle_force(L, sigma, x, F);
    for (long i = 0; i < V; ++i) pi[i] -= 0.5 * eps * F[i];
    for (int32_t k = 1; k <= n_steps; ++k) {
        for (long i = 0; i < V; ++i) sigma[i] += eps * pi[i];
        sp = md_solve(L, sigma, phi, x, A, tol, max_iter, &res->cg_iters, &res->failed);
        res->solves += 1;
        oracle_force(L, sigma, x, F);
        double c = (k == n_steps) ? 0.5 * eps : eps;
        for (long i = 0; i < V; ++i) pi[i] -= c * F[i];
    }
    res->h_end = 0.5 * oracle_dot(V, pi, pi) + sp;
    free(x);
    free(A);
    free(F);
    return 0;
}

/* One HMC trajectory: phi = M^T eta at the starting field, the MD
 * trajectory from (sigma, pi0), then the Metropolis decision with u.
 * sigma is replaced by the end point when accepted and left unchanged
 * otherwise; pi0 is not modified.  Returns as oracle_md. */
int oracle_hmc(const oracle_lattice* L, double* sigma, const double* eta, const double* pi0,
               double u, double eps, int32_t n_steps, double tol, int32_t max_iter,
               oracle_md_result* res) {
    long V = oracle_volume(L);
    double* A = (double*)malloc(sizeof(double) * V);
    double* phi = (double*)malloc(sizeof(double) * V);
    double* s1 = (double*)malloc(sizeof(double) * V);
    double* p1 = (double*)malloc(sizeof(double) * V);
    if (!A || !phi || !s1 || !p1) {
        free(A); free(phi); free(s1); free(p1);
        return -1;
    }
    oracle_links(L, sigma, A);
    oracle_apply_Mt(L, A, eta, phi);
    memcpy(s1, sigma, sizeof(double) * V);
    memcpy(p1, pi0, sizeof(double) * V);
    int rc = oracle_md(L, s1, p1, phi, eps, n_steps, tol, max_iter, res);
    if (rc == 0) {
        res->accepted = (!res->failed && u < exp(-(res->h_end - res->h_start))) ? 1 : 0;
        if (res->accepted) memcpy(sigma, s1, sizeof(double) * V);
    }
    free(A); free(phi); free(s1); free(p1);
    return rc;
}
