// Solver vector kernels (internal).
#pragma once

#include "common.h"

namespace wd {

constexpr int kGS = 8;            // basis vectors per orthogonalisation pass
constexpr int kRedThreads = 256;  // threads per reduction work-group
constexpr int kRedBlocks = 1024;  // reduction work-groups (fixed: deterministic sums)

struct VecList {
    const void *v[kGS];
    int n;
};

// host-side coefficients travel as kernel arguments (no host-to-device copy)
struct CoefList {
    double2 c[kGS];
};

// out[i] = <v_i, w> = v_i^H w for i < nv, out[nv].x = |w|^2; partial needs
// kRedBlocks * (kGS + 1) entries.  S = double2 (FP64) or float2 (FP32 storage).
template <typename S>
hipError_t mdot(const void *const *v, int nv, const void *w, long long N, double2 *partial, double2 *out,
                hipStream_t st);
// w -= sum_i coef[i] v_i; norm_out[0].x = |w_new|^2 when norm_out != null
template <typename S>
hipError_t axpy_multi(const void *const *v, int nv, const double2 *coef, void *w, long long N, double2 *partial,
                      double2 *norm_out, hipStream_t st);
// out = in * s * mult, s = sc[0].x or 1/sqrt(sc[0].x) (1 for null sc);
// SI == SO only (flat element order)
template <typename SI, typename SO>
hipError_t scale(const void *in, void *out, const double2 *sc, bool inv_sqrt, double mult, long long N,
                 hipStream_t st);
// r = b - w; norm_out[0].x = |r|^2
hipError_t residual(const double2 *b, const double2 *w, double2 *r, long long N, double2 *partial, double2 *norm_out,
                    hipStream_t st);
// x += sum_i coef[i] z_i (same precision: S = double2); coef is HOST memory
template <typename S>
hipError_t update(const void *const *z, int nz, const double2 *coef, double2 *x, long long N, hipStream_t st);
hipError_t norm2(const void *w, bool f32, long long N, double2 *partial, double2 *out, hipStream_t st);

// Same-precision flat operations above; the two cross-precision ones below
// follow the native layouts (component order differs between FP64 and FP32).
// dst (native FP32) = src (native FP64) * mult
hipError_t f64_to_f32(const void *src, void *dst, double mult, int V, hipStream_t st);
// x (native FP64) = sum_i coef[i] z_i, z_i native FP32 (x overwritten); coef HOST
hipError_t combine_f32_into_f64(const void *const *z, int nz, const double2 *coef, double2 *x, int V,
                                hipStream_t st);

// native FP32 field <-> native FP16S field (per-site scale), nrhs = 1
hipError_t f32_to_f16s(void *dst, const void *src, int V, hipStream_t st);
hipError_t f16s_to_f32(void *dst, const void *src, int V, hipStream_t st);

}  // namespace wd
