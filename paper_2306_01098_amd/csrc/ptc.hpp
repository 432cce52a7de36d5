// Parallel-transport convolution (PTC) network: shared definitions.
//
// Layer: out_c(x) = sum_{c'} sum_{p} w[c][c'][p] (T_p in_{c'})(x) with the
// nine paths p = 0 (identity), 1 + 2 mu (hop +mu: X_mu(x) in(x+mu)) and
// 2 + 2 mu (hop -mu: X_mu(x-mu)^+ in(x-mu)); time-boundary sign on wraps.
// Network 1 -> 8 -> 8 -> 1 channels, no bias, no nonlinearity, acting on the
// whole lattice; its input is an even-site field extended by zero.
#pragma once

#include "common.hpp"

namespace hisq {

constexpr int PTC_PATHS = 9;
constexpr int PTC_CH = 8;
constexpr int PTC_W1 = 0;                            // layer 1: [8][1][9]
constexpr int PTC_W2 = PTC_W1 + PTC_CH * 1 * PTC_PATHS;  // layer 2: [8][8][9]
constexpr int PTC_W3 = PTC_W2 + PTC_CH * PTC_CH * PTC_PATHS;  // layer 3: [1][8][9]
constexpr int PTC_NW = PTC_W3 + 1 * PTC_CH * PTC_PATHS;  // 720 complex weights
constexpr int PTC_BLOCK = 256;

// Whole-lattice FP32 fields of C channels: [c][parity][colour][site] float2,
// i.e. the packed FP32 half-field layout with right-hand-side index 2c + parity.
inline size_t ptc_field_bytes(const Geom &g, int channels) { return (size_t)channels * 2 * 3 * g.vh * 8; }

// skip (nullable): the launch does nothing while *skip != 0.
hipError_t ptc_embed(const Geom &g, const void *in_even, void *a0, hipStream_t st, const int *skip = nullptr);
hipError_t ptc_extract(const Geom &g, const void *a3, void *out_even, hipStream_t st, const int *skip = nullptr);
// Layer 3's output (cout = 1) is formed on the even sites only.
hipError_t ptc_layer_fwd(const Geom &g, int cin, int cout, const char *links, const float2 *w, const void *in,
                         void *out, hipStream_t st, const int *skip = nullptr);
hipError_t ptc_layer_bwd_in(const Geom &g, int cin, int cout, const char *links, const float2 *w,
                            const void *g_out, void *g_in, hipStream_t st);
hipError_t ptc_layer_bwd_w(const Geom &g, int cin, int cout, const char *links, const void *in, const void *g_out,
                           double *partials, double2 *grad, hipStream_t st);
int ptc_blocks(const Geom &g);
hipError_t ptc_xb(const Geom &g, const void *x64, const void *b32, double *partials, double *out, hipStream_t st);
hipError_t ptc_diff(const Geom &g, const void *a3, const void *x64, void *e, hipStream_t st);
hipError_t ptc_energy_grad(const Geom &g, const void *Ae, const double *eAe, const double *c, double inv_batch,
                           void *g3, double *loss_acc, hipStream_t st);
hipError_t ptc_adam(double2 *w_master, float2 *w_f32, const double2 *grad, double2 *m, double2 *v, int step,
                    double lr, double b1, double b2, double eps, hipStream_t st);
hipError_t ptc_fill_f64(double *p, size_t n, hipStream_t st);

}  // namespace hisq
