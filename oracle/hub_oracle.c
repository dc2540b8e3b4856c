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
#pragma omp parallel for schedule(static)
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
#pragma omp parallel for schedule(static)
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
