// Allocation-free M_e with the fused Re <p, M_e p>: hisq_apply_m_dot with its
// block partials in a file-scope device array instead of a caller workspace,
// for callers that cannot allocate device memory (code under graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// Each device that runs this entry point holds its own copy of `scratch`
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol); the device
// address of each device's copy is looked up once per device with
// hipGetSymbolAddress and used wherever the kernels need the buffer.
#include <mutex>

#include "api_util.hpp"

using namespace hisq;

namespace {

constexpr size_t kScratchDoubles = HISQ_NOALLOC_SCRATCH_BYTES / sizeof(double);
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be current.
hisq_status scratch_on_current(int device, double **out) {
    if (device < 0 || device >= kMaxDevices)
        return fail(HISQ_ERR_UNSUPPORTED, "device ordinal %d beyond the %d the scratch table holds", device,
                    kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return device_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p)
            return fail(HISQ_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[device] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[device];
    return HISQ_OK;
}

}  // namespace

namespace hisq {

// Set-up at context creation: the device address of `scratch` on `device`,
// with that device made current for the lookup and the caller's current
// device restored afterwards.
hisq_status noalloc_scratch_setup(int device) {
    int old = 0;
    hipError_t e = hipGetDevice(&old);
    if (e != hipSuccess)
        return device_fail(e, "hipGetDevice");
    if (old != device && (e = hipSetDevice(device)) != hipSuccess)
        return device_fail(e, "hipSetDevice");
    double *p = nullptr;
    const hisq_status s = scratch_on_current(device, &p);
    if (old != device && (e = hipSetDevice(old)) != hipSuccess)
        return device_fail(e, "hipSetDevice (restore)");
    return s;
}

}  // namespace hisq

extern "C" {

hisq_status hisq_apply_m_dot_noalloc(hisq_context *ctx, const hisq_lattice *lat, hisq_prec link_prec,
                                     hisq_prec field_prec, double mass, const void *links, const void *in_even,
                                     void *out_even, void *tmp_odd, int32_t nrhs, double *dot_out, void *stream) {
    ApplyMDot a;
    TRY(check_apply_m_dot(ctx, lat, link_prec, field_prec, mass, links, in_even, out_even, tmp_odd, nrhs, dot_out,
                          &a));
    if (a.partials > kScratchDoubles)
        return fail(HISQ_ERR_WORKSPACE,
                    "this call needs %zu bytes of block partials; the static scratch holds %zu "
                    "(HISQ_NOALLOC_SCRATCH_BYTES)",
                    a.partials * sizeof(double), (size_t)HISQ_NOALLOC_SCRATCH_BYTES);
    TRY(set_device(ctx));
    int device = 0;
    const hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess)
        return device_fail(e, "hipGetDevice");
    double *partials = nullptr;
    TRY(scratch_on_current(device, &partials));
    // every partial the finalize reads is written by this call's D_eo launch,
    // so nothing needs clearing
    return run_apply_m_dot(a, partials, static_cast<hipStream_t>(stream));
}

}  // extern "C"
