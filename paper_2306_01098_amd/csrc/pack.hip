// Conversion between the canonical complex128 layouts and the packed
// parity-split structure-of-arrays layouts (one-off per gauge field / source).
#include <mutex>

#include "internal.hpp"

// Raised by the pack kernel when a link does not fit a compressed format (one
// copy per device; host code uses the address hipGetSymbolAddress returns).
static __device__ int g_pack_bad;

namespace hisq {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_pack_mu;
int *g_pack_bad_ptr[kMaxDevices] = {};
}  // namespace

namespace {

// d[12..17] (row 2) against z conj(row 0 x row 1), all in FP64: returns the
// squared deviation; z = (1, 0) for reconstruct-12, and for W14 the
// least-squares factor z = <c, row 2> / <c, c>, c = conj(row 0 x row 1),
// returned in zr, zi (0 where c = 0).
__device__ __forceinline__ double row2_deviation(const double d[18], bool fit, double &zr, double &zi) {
    double c[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int j = (k + 1) % 3, l = (k + 2) % 3;
        const double ajr = d[2 * j], aji = d[2 * j + 1], alr = d[2 * l], ali = d[2 * l + 1];
        const double bjr = d[6 + 2 * j], bji = d[6 + 2 * j + 1], blr = d[6 + 2 * l], bli = d[6 + 2 * l + 1];
        c[2 * k] = ajr * blr - aji * bli - (alr * bjr - ali * bji);
        c[2 * k + 1] = -(ajr * bli + aji * blr - (alr * bji + ali * bjr));
    }
    zr = 1.0;
    zi = 0.0;
    if (fit) {
        double cc = 0.0, nr = 0.0, ni = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double cr = c[2 * k], ci = c[2 * k + 1], rr = d[12 + 2 * k], ri = d[12 + 2 * k + 1];
            cc += cr * cr + ci * ci;
            nr += cr * rr + ci * ri;  // conj(c) r
            ni += cr * ri - ci * rr;
        }
        zr = cc > 0.0 ? nr / cc : 0.0;
        zi = cc > 0.0 ? ni / cc : 0.0;
    }
    double dev = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double er = d[12 + 2 * k] - (zr * c[2 * k] - zi * c[2 * k + 1]);
        const double ei = d[12 + 2 * k + 1] - (zr * c[2 * k + 1] + zi * c[2 * k]);
        dev += er * er + ei * ei;
    }
    return dev;
}

// Stores matrix d (field f) in the format of LP.  The compressed formats
// (reconstruct-12; W14 Naik links) also check that the stored part rebuilds
// row 2 to tol times the Frobenius norm of the matrix, and set *bad otherwise
// (every offending thread stores 1: no ordering needed).
template <int LP>
__device__ __forceinline__ void store_matrix(char *blk, int vh, int i, const double d[18], int f, double tol,
                                             int *bad) {
    constexpr bool r12 = LP == HISQ_FP64R12 || LP == HISQ_FP32R12;
    constexpr bool w14 = LP == HISQ_FP64W14 || LP == HISQ_FP32W14;
    double zr = 1.0, zi = 0.0;
    if (r12 || (w14 && f == 1)) {
        double n2 = 0.0;
#pragma unroll
        for (int k = 0; k < 18; ++k)
            n2 += d[k] * d[k];
        const double dev = row2_deviation(d, w14, zr, zi);
        if (!(dev <= tol * tol * n2) && bad)
            *bad = 1;
    }
    if (w14 && f == 1) {  // rows 0 and 1, then z
        if (LP == HISQ_FP64W14) {
#pragma unroll
            for (int k = 0; k < 6; ++k)
                reinterpret_cast<double2 *>(blk + (size_t)vh * 16 * k)[i] = make_double2(d[2 * k], d[2 * k + 1]);
            reinterpret_cast<double2 *>(blk + (size_t)vh * 96)[i] = make_double2(zr, zi);
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                reinterpret_cast<float4 *>(blk + (size_t)vh * 16 * k)[i] =
                    make_float4((float)d[4 * k], (float)d[4 * k + 1], (float)d[4 * k + 2], (float)d[4 * k + 3]);
            reinterpret_cast<float2 *>(blk + (size_t)vh * 48)[i] = make_float2((float)zr, (float)zi);
        }
        return;
    }
    if (LP == HISQ_FP64R12) {  // rows 0 and 1 only
#pragma unroll
        for (int k = 0; k < 6; ++k)
            reinterpret_cast<double2 *>(blk + (size_t)vh * 16 * k)[i] = make_double2(d[2 * k], d[2 * k + 1]);
    } else if (LP == HISQ_FP32R12) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            reinterpret_cast<float4 *>(blk + (size_t)vh * 16 * k)[i] =
                make_float4((float)d[4 * k], (float)d[4 * k + 1], (float)d[4 * k + 2], (float)d[4 * k + 3]);
    } else if (LP == HISQ_FP64 || LP == HISQ_FP64W14) {
#pragma unroll
        for (int k = 0; k < 9; ++k)
            reinterpret_cast<double2 *>(blk + (size_t)vh * 16 * k)[i] = make_double2(d[2 * k], d[2 * k + 1]);
    } else if (LP == HISQ_FP32 || LP == HISQ_FP32W14) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            reinterpret_cast<float4 *>(blk + (size_t)vh * 16 * k)[i] =
                make_float4((float)d[4 * k], (float)d[4 * k + 1], (float)d[4 * k + 2], (float)d[4 * k + 3]);
        reinterpret_cast<float2 *>(blk + (size_t)vh * 64)[i] = make_float2((float)d[16], (float)d[17]);
    } else {
        // binary64 -> binary16 in one correctly rounded (nearest-even) step
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            H8 v;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                v.h[j] = (_Float16)d[8 * k + j];
            reinterpret_cast<uint4 *>(blk + (size_t)vh * 16 * k)[i] = v.u;
        }
        H2 t;
        t.h[0] = (_Float16)d[16];
        t.h[1] = (_Float16)d[17];
        reinterpret_cast<uint32_t *>(blk + (size_t)vh * 32)[i] = t.u;
    }
}

// One thread per (mu, lexicographic site): both X and W of that link.
template <int LP>
__global__ void __launch_bounds__(256) pack_links_kernel(Geom g, const double *fat, const double *naik,
                                                         char *packed, double tol, int *bad) {
    const int64_t V = 2 * (int64_t)g.vh;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 4 * V)
        return;
    const int mu = (int)(gid / V);
    const int64_t lex = gid - (int64_t)mu * V;
    int64_t rest = lex;
    const int x = (int)(rest % g.nx);
    rest /= g.nx;
    const int y = (int)(rest % g.ny);
    rest /= g.ny;
    const int z = (int)(rest % g.nz);
    const int t = (int)(rest / g.nz);
    const int p = (x + y + z + t) & 1;
    const int i = (int)(lex >> 1);
    for (int f = 0; f < 2; ++f) {
        const double *src = (f == 0 ? fat : naik) + gid * 18;
        double d[18];
#pragma unroll
        for (int k = 0; k < 18; ++k)
            d[k] = src[k];
        store_matrix<LP>(packed + link_block<LP>(f, p, mu, g.vh), g.vh, i, d, f, tol, bad);
    }
}

// Unpacking a reconstruct-12 link returns the rebuilt matrix (row 2 formed in
// the storage precision, as the Dslash forms it).
template <int LP>
__device__ __forceinline__ void load_matrix_f64(const char *blk, int vh, int i, double d[18], int f) {
    typename LinkIO<LP>::A m[18];
    LinkIO<LP>::load(blk, vh, i, m, f);
    if constexpr (LinkIO<LP>::rebuild)
        LinkIO<LP>::finish(m, f);
#pragma unroll
    for (int k = 0; k < 18; ++k)
        d[k] = (double)m[k];
}

template <int LP>
__global__ void __launch_bounds__(256) unpack_links_kernel(Geom g, const char *packed, double *fat,
                                                           double *naik) {
    const int64_t V = 2 * (int64_t)g.vh;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 4 * V)
        return;
    const int mu = (int)(gid / V);
    const int64_t lex = gid - (int64_t)mu * V;
    int64_t rest = lex;
    const int x = (int)(rest % g.nx);
    rest /= g.nx;
    const int y = (int)(rest % g.ny);
    rest /= g.ny;
    const int z = (int)(rest % g.nz);
    const int t = (int)(rest / g.nz);
    const int p = (x + y + z + t) & 1;
    const int i = (int)(lex >> 1);
    for (int f = 0; f < 2; ++f) {
        double d[18];
        load_matrix_f64<LP>(packed + link_block<LP>(f, p, mu, g.vh), g.vh, i, d, f);
        double *dst = (f == 0 ? fat : naik) + gid * 18;
#pragma unroll
        for (int k = 0; k < 18; ++k)
            dst[k] = d[k];
    }
}

template <int FP>
__global__ void __launch_bounds__(256) pack_field_kernel(Geom g, int nrhs, const double *src, void *dst) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)nrhs * g.vh)
        return;
    const int r = (int)(gid / g.vh);
    const int i = (int)(gid - (int64_t)r * g.vh);
    double d[6];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        d[k] = src[gid * 6 + k];
    if (FP == HISQ_FP64) {
        double2 *p = reinterpret_cast<double2 *>(dst) + (size_t)r * 3 * g.vh + i;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            p[(size_t)c * g.vh] = make_double2(d[2 * c], d[2 * c + 1]);
    } else if (FP == HISQ_FP32) {
        float2 *p = reinterpret_cast<float2 *>(dst);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            p[f32_index(g.vh, nrhs, r, c, i)] = make_float2((float)d[2 * c], (float)d[2 * c + 1]);
    } else {
        double n = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            n = fmax(n, fabs(d[k]));
        const float n32 = (float)n;
        F16NRecord rec;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            rec.s.h[k] = n32 > 0.f ? (_Float16)(d[k] / (double)n32) : (_Float16)0.f;
        rec.s.norm = n32;
        reinterpret_cast<uint4 *>(dst)[(size_t)r * g.vh + i] = rec.u;
    }
}

template <int FP>
__global__ void __launch_bounds__(256) unpack_field_kernel(Geom g, int nrhs, const void *src, double *dst) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)nrhs * g.vh)
        return;
    const int r = (int)(gid / g.vh);
    const int i = (int)(gid - (int64_t)r * g.vh);
    double d[6];
    if (FP == HISQ_FP64) {
        const double2 *p = reinterpret_cast<const double2 *>(src) + (size_t)r * 3 * g.vh + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double2 v = p[(size_t)c * g.vh];
            d[2 * c] = v.x;
            d[2 * c + 1] = v.y;
        }
    } else if (FP == HISQ_FP32) {
        const float2 *p = reinterpret_cast<const float2 *>(src);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float2 v = p[f32_index(g.vh, nrhs, r, c, i)];
            d[2 * c] = v.x;
            d[2 * c + 1] = v.y;
        }
    } else {
        F16NRecord rec;
        rec.u = reinterpret_cast<const uint4 *>(src)[(size_t)r * g.vh + i];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            d[k] = (double)rec.s.norm * (double)(float)rec.s.h[k];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k)
        dst[gid * 6 + k] = d[k];
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_pack_links(const Geom &g, int prec, const void *fat, const void *naik, void *packed,
                             hipStream_t st, int *bad) {
    const int64_t n = 8 * (int64_t)g.vh;
    const dim3 grid(blocks_for(n, 256));
    const double *f = static_cast<const double *>(fat);
    const double *w = static_cast<const double *>(naik);
    char *p = static_cast<char *>(packed);
    const bool check = prec == HISQ_FP64R12 || prec == HISQ_FP32R12 || prec == HISQ_FP64W14 || prec == HISQ_FP32W14;
    if (bad)
        *bad = 0;
    if (!check) {
        if (prec == HISQ_FP64)
            pack_links_kernel<HISQ_FP64><<<grid, 256, 0, st>>>(g, f, w, p, 0.0, nullptr);
        else if (prec == HISQ_FP32)
            pack_links_kernel<HISQ_FP32><<<grid, 256, 0, st>>>(g, f, w, p, 0.0, nullptr);
        else
            pack_links_kernel<HISQ_FP16N><<<grid, 256, 0, st>>>(g, f, w, p, 0.0, nullptr);
        return hipGetLastError();
    }
    // the compressed formats: the kernel raises the check's flag, read back
    // here; packs are serialized so that they do not share the flag
    std::lock_guard<std::mutex> lk(g_pack_mu);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    if (!g_pack_bad_ptr[dev]) {
        void *ptr = nullptr;
        if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_pack_bad))) != hipSuccess)
            return e;
        g_pack_bad_ptr[dev] = static_cast<int *>(ptr);
    }
    int *flag = g_pack_bad_ptr[dev];
    if ((e = launch_fill_u32(reinterpret_cast<unsigned *>(flag), 1, 0u, st)) != hipSuccess)
        return e;
    const double tol = prec == HISQ_FP64R12 || prec == HISQ_FP64W14 ? 1e-10 : 1e-5;
    if (prec == HISQ_FP64R12)
        pack_links_kernel<HISQ_FP64R12><<<grid, 256, 0, st>>>(g, f, w, p, tol, flag);
    else if (prec == HISQ_FP32R12)
        pack_links_kernel<HISQ_FP32R12><<<grid, 256, 0, st>>>(g, f, w, p, tol, flag);
    else if (prec == HISQ_FP64W14)
        pack_links_kernel<HISQ_FP64W14><<<grid, 256, 0, st>>>(g, f, w, p, tol, flag);
    else
        pack_links_kernel<HISQ_FP32W14><<<grid, 256, 0, st>>>(g, f, w, p, tol, flag);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    int h = 0;
    if ((e = hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, st)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess)
        return e;
    if (bad)
        *bad = h;
    return hipSuccess;
}

hipError_t launch_unpack_links(const Geom &g, int prec, const void *packed, void *fat, void *naik,
                               hipStream_t st) {
    const int64_t n = 8 * (int64_t)g.vh;
    const dim3 grid(blocks_for(n, 256));
    const char *p = static_cast<const char *>(packed);
    double *f = static_cast<double *>(fat);
    double *w = static_cast<double *>(naik);
    if (prec == HISQ_FP64)
        unpack_links_kernel<HISQ_FP64><<<grid, 256, 0, st>>>(g, p, f, w);
    else if (prec == HISQ_FP32)
        unpack_links_kernel<HISQ_FP32><<<grid, 256, 0, st>>>(g, p, f, w);
    else if (prec == HISQ_FP64R12)
        unpack_links_kernel<HISQ_FP64R12><<<grid, 256, 0, st>>>(g, p, f, w);
    else if (prec == HISQ_FP32R12)
        unpack_links_kernel<HISQ_FP32R12><<<grid, 256, 0, st>>>(g, p, f, w);
    else if (prec == HISQ_FP64W14)
        unpack_links_kernel<HISQ_FP64W14><<<grid, 256, 0, st>>>(g, p, f, w);
    else if (prec == HISQ_FP32W14)
        unpack_links_kernel<HISQ_FP32W14><<<grid, 256, 0, st>>>(g, p, f, w);
    else
        unpack_links_kernel<HISQ_FP16N><<<grid, 256, 0, st>>>(g, p, f, w);
    return hipGetLastError();
}

hipError_t launch_pack_field(const Geom &g, int prec, int nrhs, const void *src, void *dst, hipStream_t st) {
    const dim3 grid(blocks_for((int64_t)nrhs * g.vh, 256));
    const double *s = static_cast<const double *>(src);
    if (prec == HISQ_FP64)
        pack_field_kernel<HISQ_FP64><<<grid, 256, 0, st>>>(g, nrhs, s, dst);
    else if (prec == HISQ_FP32)
        pack_field_kernel<HISQ_FP32><<<grid, 256, 0, st>>>(g, nrhs, s, dst);
    else
        pack_field_kernel<HISQ_FP16N><<<grid, 256, 0, st>>>(g, nrhs, s, dst);
    return hipGetLastError();
}

hipError_t launch_unpack_field(const Geom &g, int prec, int nrhs, const void *src, void *dst, hipStream_t st) {
    const dim3 grid(blocks_for((int64_t)nrhs * g.vh, 256));
    double *d = static_cast<double *>(dst);
    if (prec == HISQ_FP64)
        unpack_field_kernel<HISQ_FP64><<<grid, 256, 0, st>>>(g, nrhs, src, d);
    else if (prec == HISQ_FP32)
        unpack_field_kernel<HISQ_FP32><<<grid, 256, 0, st>>>(g, nrhs, src, d);
    else
        unpack_field_kernel<HISQ_FP16N><<<grid, 256, 0, st>>>(g, nrhs, src, d);
    return hipGetLastError();
}

}  // namespace hisq
