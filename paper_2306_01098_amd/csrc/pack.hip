// Conversion between the canonical complex128 layouts and the packed
// parity-split structure-of-arrays layouts (one-off per gauge field / source).
#include "internal.hpp"

namespace hisq {

namespace {

template <int LP>
__device__ __forceinline__ void store_matrix(char *blk, int vh, int i, const double d[18]) {
    if (LP == HISQ_FP64R12) {  // rows 0 and 1 only
#pragma unroll
        for (int k = 0; k < 6; ++k)
            reinterpret_cast<double2 *>(blk + (size_t)vh * 16 * k)[i] = make_double2(d[2 * k], d[2 * k + 1]);
    } else if (LP == HISQ_FP32R12) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            reinterpret_cast<float4 *>(blk + (size_t)vh * 16 * k)[i] =
                make_float4((float)d[4 * k], (float)d[4 * k + 1], (float)d[4 * k + 2], (float)d[4 * k + 3]);
    } else if (LP == HISQ_FP64) {
#pragma unroll
        for (int k = 0; k < 9; ++k)
            reinterpret_cast<double2 *>(blk + (size_t)vh * 16 * k)[i] = make_double2(d[2 * k], d[2 * k + 1]);
    } else if (LP == HISQ_FP32) {
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
                                                         char *packed) {
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
    constexpr int MB = Prec<LP>::mat_bytes;
    for (int f = 0; f < 2; ++f) {
        const double *src = (f == 0 ? fat : naik) + gid * 18;
        double d[18];
#pragma unroll
        for (int k = 0; k < 18; ++k)
            d[k] = src[k];
        store_matrix<LP>(packed + link_block(f, p, mu, g.vh, MB), g.vh, i, d);
    }
}

// Unpacking a reconstruct-12 link returns the rebuilt matrix (row 2 formed in
// the storage precision, as the Dslash forms it).
template <int LP>
__device__ __forceinline__ void load_matrix_f64(const char *blk, int vh, int i, double d[18]) {
    typename LinkIO<LP>::A m[18];
    LinkIO<LP>::load(blk, vh, i, m);
    if constexpr (LinkIO<LP>::rebuild)
        rebuild_row2(m);
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
    constexpr int MB = Prec<LP>::mat_bytes;
    for (int f = 0; f < 2; ++f) {
        double d[18];
        load_matrix_f64<LP>(packed + link_block(f, p, mu, g.vh, MB), g.vh, i, d);
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
        float2 *p = reinterpret_cast<float2 *>(dst) + (size_t)r * 3 * g.vh + i;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            p[(size_t)c * g.vh] = make_float2((float)d[2 * c], (float)d[2 * c + 1]);
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
        const float2 *p = reinterpret_cast<const float2 *>(src) + (size_t)r * 3 * g.vh + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float2 v = p[(size_t)c * g.vh];
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
                             hipStream_t st) {
    const int64_t n = 8 * (int64_t)g.vh;
    const dim3 grid(blocks_for(n, 256));
    const double *f = static_cast<const double *>(fat);
    const double *w = static_cast<const double *>(naik);
    char *p = static_cast<char *>(packed);
    if (prec == HISQ_FP64)
        pack_links_kernel<HISQ_FP64><<<grid, 256, 0, st>>>(g, f, w, p);
    else if (prec == HISQ_FP32)
        pack_links_kernel<HISQ_FP32><<<grid, 256, 0, st>>>(g, f, w, p);
    else if (prec == HISQ_FP64R12)
        pack_links_kernel<HISQ_FP64R12><<<grid, 256, 0, st>>>(g, f, w, p);
    else if (prec == HISQ_FP32R12)
        pack_links_kernel<HISQ_FP32R12><<<grid, 256, 0, st>>>(g, f, w, p);
    else
        pack_links_kernel<HISQ_FP16N><<<grid, 256, 0, st>>>(g, f, w, p);
    return hipGetLastError();
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
