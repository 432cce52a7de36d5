// Host helpers shared by the C ABI translation units: error reporting,
// argument checks and the context (device + autotune cache).
#pragma once

#include <map>
#include <mutex>
#include <tuple>

#include "internal.hpp"

struct hisq_context {
    int device = 0;
    // Autotuned Dslash shapes keyed by (extents, link precision, field
    // precision, nrhs).
    using Key = std::tuple<int, int, int, int, int, int, int>;
    std::map<Key, hisq::DslashShape> shapes;
    std::mutex mu;

    static Key key(const hisq::Geom &g, int lp, int fp, int nrhs) {
        return Key(g.nx, g.ny, g.nz, g.nt, lp, fp, nrhs);
    }
    bool lookup(const hisq::Geom &g, int lp, int fp, int nrhs, hisq::DslashShape *s) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = shapes.find(key(g, lp, fp, nrhs));
        if (it == shapes.end())
            return false;
        *s = it->second;
        return true;
    }
    void store(const hisq::Geom &g, int lp, int fp, int nrhs, hisq::DslashShape s) {
        std::lock_guard<std::mutex> lk(mu);
        shapes[key(g, lp, fp, nrhs)] = s;
    }
};

namespace hisq {

hisq_status fail(hisq_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
hisq_status device_fail(hipError_t e, const char *where);
hisq_status check_lattice(const hisq_lattice *lat);
hisq_status check_prec(int prec);
hisq_status check_nrhs(int nrhs);
hisq_status check_ptr(const void *p, const char *name);
hisq_status set_device(hisq_context *ctx);
// Return the status of expr from the calling entry point unless it is HISQ_OK.
#define TRY(expr)                        \
    do {                                 \
        const hisq_status _s = (expr);   \
        if (_s != HISQ_OK)               \
            return _s;                   \
    } while (0)

DslashShape pick_shape(hisq_context *ctx, const Geom &g, int lp, int fp, int nrhs);

// M_e with the fused Re <in, out> (hisq_apply_m_dot and its variants): the
// checked arguments, the launch shape and the number of block partials.
struct ApplyMDot {
    Geom g;
    int lp, fp;
    double mass;
    const char *links;
    const void *in;
    void *out, *tmp;
    int nrhs;
    double *dot;
    DslashShape shape;
    size_t partials;  // doubles of block partials this call needs
};
size_t apply_m_dot_partials_max(const Geom &g, int nrhs);
hisq_status check_apply_m_dot(hisq_context *ctx, const hisq_lattice *lat, int link_prec, int field_prec, double mass,
                              const void *links, const void *in_even, void *out_even, void *tmp_odd, int nrhs,
                              double *dot_out, ApplyMDot *a);
hisq_status run_apply_m_dot(const ApplyMDot &a, double *partials, hipStream_t st);
DslashShape default_shape(const Geom &g, int lp, int fp, int nrhs);
// Looks up the device address of the allocation-free entry point's scratch
// array on `device` (once per device).
hisq_status noalloc_scratch_setup(int device);

}  // namespace hisq
