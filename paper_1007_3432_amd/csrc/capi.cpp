// Exported C ABI of libhub (declarations and contracts in include/hub.h).
#include <cmath>
#include <cstdint>
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

const char* hub_last_error(void) { return last_error(); }

}  // extern "C"
