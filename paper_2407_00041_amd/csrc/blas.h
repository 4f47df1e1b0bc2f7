// Solver vector kernels (internal).
#pragma once

#include "common.h"

namespace wd {

constexpr int kGS = 32;           // basis vectors per FP64 update pass (a restart-30 step in one pass)
constexpr int kMdot = 8;          // basis vectors per FP64 inner-product pass (8 accumulators keep occupancy)
constexpr int kGSSite = 8;        // basis vectors per pass of the per-site (low-precision) kernels
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
struct ScaleList {
    double s[kGS];
};
// work-group chunks of the all-vector inner products: partial needs
// kMdotChunks * ceil(min(nv, kGS) / kMdot) * (kMdot + 1) entries
constexpr int kMdotChunks = kRedBlocks;

// out[i] = sum over groups of partial[g][i], i < gridDim.x; stride = columns per partial row
__global__ __launch_bounds__(kRedThreads) void k_colsum(const double2 *__restrict__ partial, int ngroups, int stride,
                                                        double2 *__restrict__ out);

// out[i] = <v_i, w> = v_i^H w for i < nv, out[nv].x = |w|^2, in one launch per
// kGS vectors (w read about once from HBM, see k_mdot_all); partial as
// documented at kMdotChunks.  S = double2 (FP64 storage).
template <typename S>
hipError_t mdot_all(const void *const *v, int nv, const void *w, long long N, double2 *partial, double2 *out,
                    hipStream_t st);
// w -= sum_i coef[i] cscale[i] v_i (coef on the device, cscale on the host or
// null for 1); norm_out[0].x = |w_new|^2 when norm_out != null.  partial needs
// kRedBlocks + kGS entries (norm partials, then the scaled coefficients of a pass)
template <typename S>
hipError_t axpy_multi(const void *const *v, int nv, const double2 *coef, const double *cscale, void *w, long long N,
                      double2 *partial, double2 *norm_out, hipStream_t st);
// out = in * s * mult, s = sc[0].x or 1/sqrt(sc[0].x) (1 for null sc);
// SI == SO == double2 (flat element order)
template <typename SI, typename SO>
hipError_t scale(const void *in, void *out, const double2 *sc, bool inv_sqrt, double mult, long long N,
                 hipStream_t st);
// r = b - w; norm_out[0].x = |r|^2
hipError_t residual(const double2 *b, const double2 *w, double2 *r, long long N, double2 *partial, double2 *norm_out,
                    hipStream_t st);
// x += sum_i coef[i] z_i (same precision: S = double2); coef is HOST memory
template <typename S>
hipError_t update(const void *const *z, int nz, const double2 *coef, double2 *x, long long N, hipStream_t st);

// Per-site operations on native fields of precision prec (WDIRAC_F64, _F32 or
// _F16S), nrhs = 1, FP64 accumulation; results re-encoded in the field's
// precision, in passes of kGSSite vectors.  partial needs kRedBlocks * (kGSSite + 1)
// entries.  hdr (nullable) is
// the device header of an inner cycle: hdr[0] = (completed steps, active
// flag), hdr[1].x = normalisation factor; with hdr[0].y == 0 the kernels of
// mdot and axpy do nothing.
// out[i] = v_i^H w (i < nv), out[nv].x = |w|^2
hipError_t site_mdot(int prec, const void *const *v, int nv, const void *w, int V, double2 *partial, double2 *out,
                     const double2 *hdr, hipStream_t st);
// w = f (w - sum_i coef[i] v_i), coef on the device, f = hdr[1].x (1 without
// hdr); norm_out[0].x = |w_new|^2 (before re-encoding) when non-null
hipError_t site_axpy(int prec, const void *const *v, int nv, const double2 *coef, void *w, int V, double2 *partial,
                     double2 *norm_out, const double2 *hdr, hipStream_t st);
// out (precision pout) = in (precision pin) * mult; pin == pout or pin = F64
hipError_t site_scale(int pin, int pout, const void *in, void *out, double mult, int V, hipStream_t st);
// x (native FP64) = sum_{i < n} coef[i] z_i with n = hdr[0].x <= nmax, z_i of
// precision prec, coef on the device (x overwritten; n = 0 gives x = 0)
hipError_t site_combine(int prec, const void *const *z, int nmax, const double2 *coef, const double2 *hdr, double2 *x,
                        int V, hipStream_t st);

}  // namespace wd
