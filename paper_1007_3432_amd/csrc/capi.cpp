// Exported C ABI of libhub (declarations and contracts in include/hub.h).
#include <cmath>
#include <cstdint>
#include <initializer_list>
#include <new>

#include "cheb.h"
#include "internal.h"

namespace hub {
const char* last_error();
}

using namespace hub;

namespace {

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

bool valid_dtype(int t) { return t == HUB_F64 || t == HUB_F32 || t == HUB_F16; }

hub_status check_vec_ptr(const void* p, const char* name) {
    if (!p) return set_error(HUB_E_INVALID, "%s is NULL", name);
    if (!aligned16(p)) return set_error(HUB_E_INVALID, "%s is not 16-byte aligned", name);
    return HUB_OK;
}

#define HUB_TRY(expr)                \
    do {                             \
        hub_status s_ = (expr);      \
        if (s_ != HUB_OK) return s_; \
    } while (0)

#define HUB_GUARD_BEGIN try {
#define HUB_GUARD_END                                                         \
    }                                                                         \
    catch (const std::bad_alloc&) {                                           \
        return set_error(HUB_E_NOMEM, "host allocation failed");              \
    }                                                                         \
    catch (...) {                                                             \
        return set_error(HUB_E_INVALID, "internal error (unexpected exception)"); \
    }

hub_status check_apply_args(const hub_lattice* lat, const void* links, int link,
                            int vec, const void* x, const void* y, Geom* g) {
    HUB_TRY(make_geom(lat, g));
    if (!valid_dtype(link) || !valid_dtype(vec))
        return set_error(HUB_E_INVALID, "unknown dtype (vec %d, link %d)", vec, link);
    if (!valid_pair((hub_dtype)vec, (hub_dtype)link))
        return set_error(HUB_E_INVALID,
                         "unsupported precision pair (vec %d, link %d): use F64/F64, "
                         "F32/F32 or F32/F16",
                         vec, link);
    HUB_TRY(check_vec_ptr(links, "links"));
    HUB_TRY(check_vec_ptr(x, "x"));
    HUB_TRY(check_vec_ptr(y, "output"));
    if (x == y) return set_error(HUB_E_INVALID, "input and output alias");
    return HUB_OK;
}

hub_status check_cg_args(const hub_lattice* lat, const double* sigma, const double* phi,
                         const double* x, const hub_cg_opts* opts, Geom* g) {
    HUB_TRY(make_geom(lat, g));
    if (!opts) return set_error(HUB_E_INVALID, "opts is NULL");
    const hub_cg_opts o = *opts;
    if (!valid_dtype(o.bulk) || !valid_dtype(o.link))
        return set_error(HUB_E_INVALID, "unknown dtype in opts");
    if (o.bulk == HUB_F16) return set_error(HUB_E_INVALID, "bulk precision must be F64 or F32");
    if (!valid_pair(o.bulk, o.link))
        return set_error(HUB_E_INVALID, "link dtype %d does not fit bulk dtype %d",
                         (int)o.link, (int)o.bulk);
    if (!(o.tol > 0) || !(o.tol < 1))
        return set_error(HUB_E_INVALID, "tol = %g, expected 0 < tol < 1", o.tol);
    if (o.max_iter < 1) return set_error(HUB_E_INVALID, "max_iter must be >= 1");
    if (o.bulk == HUB_F32 && o.reliable_every < 1)
        return set_error(HUB_E_INVALID, "reliable_every must be >= 1");
    HUB_TRY(check_vec_ptr(sigma, "sigma"));
    HUB_TRY(check_vec_ptr(phi, "phi"));
    HUB_TRY(check_vec_ptr(x, "x"));
    if ((const void*)x == (const void*)phi || (const void*)x == (const void*)sigma)
        return set_error(HUB_E_INVALID, "x aliases an input");
    return HUB_OK;
}

hub_status check_md_opts(const hub_md_opts* o) {
    if (!o) return set_error(HUB_E_INVALID, "md opts is NULL");
    if (o->n_steps < 1) return set_error(HUB_E_INVALID, "n_steps = %d, expected >= 1", o->n_steps);
    if (o->reserved != 0) return set_error(HUB_E_INVALID, "md opts reserved must be 0");
    if (!std::isfinite(o->eps) || !(o->eps > 0))
        return set_error(HUB_E_INVALID, "eps = %g, expected finite > 0", o->eps);
    const hub_cg_opts c = o->cg;
    if (!valid_dtype(c.bulk) || !valid_dtype(c.link) || c.bulk == HUB_F16 ||
        !valid_pair(c.bulk, c.link))
        return set_error(HUB_E_INVALID, "md opts: bad solver precision (bulk %d, link %d)",
                         (int)c.bulk, (int)c.link);
    if (!(c.tol > 0) || !(c.tol < 1))
        return set_error(HUB_E_INVALID, "md opts: tol = %g, expected 0 < tol < 1", c.tol);
    if (c.max_iter < 1) return set_error(HUB_E_INVALID, "md opts: max_iter must be >= 1");
    if (c.bulk == HUB_F32 && c.reliable_every < 1)
        return set_error(HUB_E_INVALID, "md opts: reliable_every must be >= 1");
    return HUB_OK;
}

bool distinct(std::initializer_list<const void*> ps) {
    for (auto a = ps.begin(); a != ps.end(); ++a)
        for (auto b = a + 1; b != ps.end(); ++b)
            if (*a == *b) return false;
    return true;
}

hub_status check_cheb(const hub_cheb_opts* c) {
    if (!c) return set_error(HUB_E_INVALID, "cheb is NULL");
    if (c->n < 1 || c->n > 256) return set_error(HUB_E_INVALID, "cheb n = %d, expected 1..256", c->n);
    if (c->reserved != 0) return set_error(HUB_E_INVALID, "cheb reserved must be 0");
    if (!(c->eps > 0) || !(c->eps < 1))
        return set_error(HUB_E_INVALID, "cheb eps = %g, expected 0 < eps < 1", c->eps);
    if (!std::isfinite(c->scale)) return set_error(HUB_E_INVALID, "cheb scale is not finite");
    return HUB_OK;
}

}  // namespace

extern "C" {

hub_status hub_links_from_sigma(const hub_lattice* lat, const double* sigma, void* links,
                                hub_dtype link, void* stream) {
    HUB_GUARD_BEGIN
    clear_error();
    Geom g;
    HUB_TRY(make_geom(lat, &g));
    if (!valid_dtype(link)) return set_error(HUB_E_INVALID, "unknown link dtype %d", (int)link);
    HUB_TRY(check_vec_ptr(sigma, "sigma"));
    HUB_TRY(check_vec_ptr(links, "links"));
    return launch_links(g, sigma, links, link, (hipStream_t)stream);
    HUB_GUARD_END
}

hub_status hub_apply_M(const hub_lattice* lat, const void* links, hub_dtype link,
                       hub_dtype vec, const void* x, void* y, int transpose, void* stream) {
    HUB_GUARD_BEGIN
    clear_error();
    Geom g;
    HUB_TRY(check_apply_args(lat, links, link, vec, x, y, &g));
    if (transpose != 0 && transpose != 1)
        return set_error(HUB_E_INVALID, "transpose must be 0 or 1");
    return launch_apply_M(g, links, link, vec, x, y, transpose, (hipStream_t)stream);
    HUB_GUARD_END
}

hub_status hub_apply_MtM(const hub_lattice* lat, const void* links, hub_dtype link,
                         hub_dtype vec, const void* x, void* z, void* stream) {
    HUB_GUARD_BEGIN
    clear_error();
    Geom g;
    HUB_TRY(check_apply_args(lat, links, link, vec, x, z, &g));
    return launch_apply_MtM(g, links, link, vec, x, z, nullptr, (hipStream_t)stream);
    HUB_GUARD_END
}

hub_status hub_cg_solve(const hub_lattice* lat, const double* sigma, const double* phi,
                        double* x, const hub_cg_opts* opts, hub_cg_stats* out,
                        void* stream) {
    HUB_GUARD_BEGIN
    clear_error();
    Geom g;
    HUB_TRY(check_cg_args(lat, sigma, phi, x, opts, &g));
    return cg_solve(g, sigma, phi, x, *opts, out, (hipStream_t)stream);
    HUB_GUARD_END
}

hub_status hub_apply_cheb(const hub_lattice* lat, const double* links, const double* r,
                          double* z, const hub_cheb_opts* cheb, void* stream) {
    HUB_GUARD_BEGIN
    clear_error();
    Geom g;
    HUB_TRY(make_geom(lat, &g));
    HUB_TRY(check_cheb(cheb));
    HUB_TRY(check_vec_ptr(links, "links"));
    HUB_TRY(check_vec_ptr(r, "r"));
    HUB_TRY(check_vec_ptr(z, "z"));
    if ((const void*)r == (const void*)z || (const void*)z == (const void*)links)
        return set_error(HUB_E_INVALID, "z aliases an input");
    return cheb_apply(g, links, r, z, *cheb, (hipStream_t)stream);
    HUB_GUARD_END
}

hub_status hub_apply_cheb_noalloc(const hub_lattice* lat, const double* links, const double* r,
                                  double* z, const hub_cheb_opts* cheb, void* stream) {
    HUB_GUARD_BEGIN
    clear_error();
    Geom g;
    HUB_TRY(make_geom(lat, &g));
    HUB_TRY(check_cheb(cheb));
    HUB_TRY(check_vec_ptr(links, "links"));
    HUB_TRY(check_vec_ptr(r, "r"));
    HUB_TRY(check_vec_ptr(z, "z"));
    if ((const void*)r == (const void*)z || (const void*)z == (const void*)links)
        return set_error(HUB_E_INVALID, "z aliases an input");
    return cheb_apply_noalloc(g, links, r, z, *cheb, (hipStream_t)stream);
    HUB_GUARD_END
}

hub_status hub_pcg_solve(const hub_lattice* lat, const double* sigma, const double* phi,
                         double* x, const hub_cg_opts* opts, const hub_cheb_opts* cheb,
                         hub_cg_stats* out, void* stream) {
    HUB_GUARD_BEGIN
    clear_error();
    Geom g;
    HUB_TRY(check_cg_args(lat, sigma, phi, x, opts, &g));
    HUB_TRY(check_cheb(cheb));
    if (opts->bulk != HUB_F64 || opts->link != HUB_F64)
        return set_error(HUB_E_INVALID, "hub_pcg_solve runs in FP64: bulk and link must be F64");
    return pcg_solve(g, sigma, phi, x, *opts, *cheb, out, (hipStream_t)stream);
    HUB_GUARD_END
}

hub_status hub_hmc_force(const hub_lattice* lat, const double* sigma, const double* x,
                         double* force, void* stream) {
    HUB_GUARD_BEGIN
    clear_error();
    Geom g;
    HUB_TRY(make_geom(lat, &g));
    HUB_TRY(check_vec_ptr(sigma, "sigma"));
    HUB_TRY(check_vec_ptr(x, "x"));
    HUB_TRY(check_vec_ptr(force, "force"));
    if (!distinct({sigma, x, force})) return set_error(HUB_E_INVALID, "force aliases an input");
    return hmc_force(g, sigma, x, force, (hipStream_t)stream);
    HUB_GUARD_END
}

hub_status hub_md_trajectory(const hub_lattice* lat, double* sigma, double* pi,
                             const double* phi, const hub_md_opts* opts, hub_md_stats* out,
                             void* stream) {
    HUB_GUARD_BEGIN
    clear_error();
    Geom g;
    HUB_TRY(make_geom(lat, &g));
    HUB_TRY(check_md_opts(opts));
    HUB_TRY(check_vec_ptr(sigma, "sigma"));
    HUB_TRY(check_vec_ptr(pi, "pi"));
    HUB_TRY(check_vec_ptr(phi, "phi"));
    if (!distinct({sigma, pi, phi})) return set_error(HUB_E_INVALID, "sigma, pi and phi alias");
    return md_trajectory(g, sigma, pi, phi, nullptr, nullptr, 0.0, *opts, out,
                         (hipStream_t)stream);
    HUB_GUARD_END
}

hub_status hub_hmc_trajectory(const hub_lattice* lat, double* sigma, const double* eta,
                              const double* pi0, double u, const hub_md_opts* opts,
                              hub_md_stats* out, void* stream) {
    HUB_GUARD_BEGIN
    clear_error();
    Geom g;
    HUB_TRY(make_geom(lat, &g));
    HUB_TRY(check_md_opts(opts));
    HUB_TRY(check_vec_ptr(sigma, "sigma"));
    HUB_TRY(check_vec_ptr(eta, "eta"));
    HUB_TRY(check_vec_ptr(pi0, "pi0"));
    if (!distinct({sigma, eta, pi0})) return set_error(HUB_E_INVALID, "sigma, eta and pi0 alias");
    if (!std::isfinite(u)) return set_error(HUB_E_INVALID, "u is not finite");
    return md_trajectory(g, sigma, nullptr, nullptr, eta, pi0, u, *opts, out,
                         (hipStream_t)stream);
    HUB_GUARD_END
}

hub_status hub_solver_release(void) {
    HUB_GUARD_BEGIN
    clear_error();
    solver_release();
    return HUB_OK;
    HUB_GUARD_END
}

const char* hub_last_error(void) { return last_error(); }

}  // extern "C"
