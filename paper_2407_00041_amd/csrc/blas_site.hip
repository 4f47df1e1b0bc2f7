// Krylov vector kernels on native fields of any storage precision (FP64,
// FP32, FP16 with a per-site scale), one thread per lattice site: a site's
// 12 complex components are decoded with the stencil's own loaders, every sum
// is accumulated in FP64, and results are re-encoded with the stencil's
// stores (FP16S: a fresh per-site scale).  With these the inner GMRES of the
// mixed solver keeps its Krylov basis in the low-precision operator's layout,
// so the operator reads and writes basis vectors directly.
//
// The kernels can follow a device-side state header hdr of the inner cycle
// (hdr[0] = (completed steps, active flag), hdr[1].x = normalisation factor):
// they return at once for a right-hand side whose cycle has ended, and take
// their coefficients from device memory, so a whole cycle can be issued
// without host decisions (and captured as a graph).
//
// Reductions are deterministic: a fixed grid of kRedBlocks work-groups, each
// thread summing a fixed strided subset of sites, a fixed LDS tree per
// work-group, then k_colsum adding the per-group partials in order.
#include "blas.h"
#include "spinor_io.h"

namespace wd {

namespace {

template <int P> struct SiteIO {
    using T = typename Store<P>::T;
    static __device__ __forceinline__ void load(const void *f, int V, int s, double2 v[12]) {
        cx<T> a[12];
        Store<P>::load_spinor(f, V, s, a);
#pragma unroll
        for (int k = 0; k < 12; k++) v[k] = make_double2((double)a[k].r, (double)a[k].i);
    }
    static __device__ __forceinline__ void store(void *f, int V, int s, const double2 v[12]) {
        cx<T> a[12];
#pragma unroll
        for (int k = 0; k < 12; k++) a[k] = {(T)v[k].x, (T)v[k].y};
        Store<P>::store_spinor(f, V, s, a);
    }
};

template <int NV>
__device__ __forceinline__ void reduce_block(double2 (&v)[NV], double2 *lds) {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NV; i++) lds[i * kRedThreads + t] = v[i];
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int i = 0; i < NV; i++) {
                double2 a = lds[i * kRedThreads + t], b = lds[i * kRedThreads + t + s];
                lds[i * kRedThreads + t] = make_double2(a.x + b.x, a.y + b.y);
            }
        }
        __syncthreads();
    }
    if (t == 0) {
#pragma unroll
        for (int i = 0; i < NV; i++) v[i] = lds[i * kRedThreads];
    }
}

}  // namespace

// partial[blk][i] = sum over the group's sites of v_i^H w (i < n), [kGSSite] = |w|^2
template <int P>
__global__ __launch_bounds__(kRedThreads) void k_site_mdot(VecList vl, const void *__restrict__ w,
                                                            double2 *__restrict__ partial, const double2 *hdr, int V) {
    if (hdr && hdr[0].y == 0.0) return;
    __shared__ double2 lds[(kGSSite + 1) * kRedThreads];
    double2 acc[kGSSite + 1];
#pragma unroll
    for (int i = 0; i <= kGSSite; i++) acc[i] = make_double2(0, 0);
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < V; s += gridDim.x * blockDim.x) {
        double2 wv[12];
        SiteIO<P>::load(w, V, s, wv);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[kGSSite].x += wv[k].x * wv[k].x + wv[k].y * wv[k].y;
#pragma unroll
        for (int i = 0; i < kGSSite; i++) {
            if (i < vl.n) {
                double2 vv[12];
                SiteIO<P>::load(vl.v[i], V, s, vv);
#pragma unroll
                for (int k = 0; k < 12; k++) {
                    acc[i].x += vv[k].x * wv[k].x + vv[k].y * wv[k].y;
                    acc[i].y += vv[k].x * wv[k].y - vv[k].y * wv[k].x;
                }
            }
        }
    }
    reduce_block<kGSSite + 1>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i <= kGSSite; i++) partial[(size_t)blockIdx.x * (kGSSite + 1) + i] = acc[i];
    }
}

// w = f (w - sum_i coef[i] v_i), coefficients on the device; f = hdr[1].x when
// apply_f (last pass) and hdr are set, else 1.  partial[blk] = |w_new|^2 of the
// re-encoded values' source (before rounding) when partial != null.
template <int P>
__global__ __launch_bounds__(kRedThreads) void k_site_axpy(VecList vl, const double2 *__restrict__ coef,
                                                            void *__restrict__ w, double2 *__restrict__ partial,
                                                            const double2 *hdr, int apply_f, int V) {
    if (hdr && hdr[0].y == 0.0) return;
    __shared__ double2 lds[kRedThreads];
    const double f = (hdr && apply_f) ? hdr[1].x : 1.0;
    double2 nrm[1] = {make_double2(0, 0)};
    double2 c[kGSSite];
#pragma unroll
    for (int i = 0; i < kGSSite; i++) c[i] = i < vl.n ? coef[i] : make_double2(0, 0);
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < V; s += gridDim.x * blockDim.x) {
        double2 wv[12];
        SiteIO<P>::load(w, V, s, wv);
#pragma unroll
        for (int i = 0; i < kGSSite; i++) {
            if (i < vl.n) {
                double2 vv[12];
                SiteIO<P>::load(vl.v[i], V, s, vv);
#pragma unroll
                for (int k = 0; k < 12; k++) {
                    wv[k].x -= c[i].x * vv[k].x - c[i].y * vv[k].y;
                    wv[k].y -= c[i].x * vv[k].y + c[i].y * vv[k].x;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 12; k++) wv[k] = make_double2(wv[k].x * f, wv[k].y * f);
        SiteIO<P>::store(w, V, s, wv);
#pragma unroll
        for (int k = 0; k < 12; k++) nrm[0].x += wv[k].x * wv[k].x + wv[k].y * wv[k].y;
    }
    if (partial) {
        reduce_block<1>(nrm, lds);
        if (threadIdx.x == 0) partial[blockIdx.x] = nrm[0];
    }
}

// out (precision PO) = in (precision PI) * mult
template <int PI, int PO>
__global__ __launch_bounds__(kRedThreads) void k_site_scale(const void *__restrict__ in, void *__restrict__ out,
                                                             double mult, int V) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < V; s += gridDim.x * blockDim.x) {
        double2 v[12];
        SiteIO<PI>::load(in, V, s, v);
#pragma unroll
        for (int k = 0; k < 12; k++) v[k] = make_double2(v[k].x * mult, v[k].y * mult);
        SiteIO<PO>::store(out, V, s, v);
    }
}

// x (native FP64) = keep * x + sum_{i < n} coef[i] z_i, z_i of precision P,
// n = min(kGSSite, count - i0) with count = hdr[0].x (device coefficients)
template <int P>
__global__ __launch_bounds__(kRedThreads) void k_site_combine(VecList vl, const double2 *__restrict__ coef,
                                                               const double2 *hdr, int i0, double2 *__restrict__ x,
                                                               int V) {
    const int count = (int)hdr[0].x;
    const int n = count - i0 < kGSSite ? count - i0 : kGSSite;
    if (i0 > 0 && n <= 0) return;
    double2 c[kGSSite];
#pragma unroll
    for (int i = 0; i < kGSSite; i++) c[i] = i < n ? coef[i] : make_double2(0, 0);
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < V; s += gridDim.x * blockDim.x) {
        double2 xv[12];
        if (i0 > 0) {
            SiteIO<WDIRAC_F64>::load(x, V, s, xv);
        } else {
#pragma unroll
            for (int k = 0; k < 12; k++) xv[k] = make_double2(0, 0);
        }
#pragma unroll
        for (int i = 0; i < kGSSite; i++) {
            if (i < n) {
                double2 zv[12];
                SiteIO<P>::load(vl.v[i], V, s, zv);
#pragma unroll
                for (int k = 0; k < 12; k++) {
                    xv[k].x += c[i].x * zv[k].x - c[i].y * zv[k].y;
                    xv[k].y += c[i].x * zv[k].y + c[i].y * zv[k].x;
                }
            }
        }
        SiteIO<WDIRAC_F64>::store(x, V, s, xv);
    }
}

// ---------------------------------------------------------------------------

static int site_grid(int V) {
    const int g = (V + kRedThreads - 1) / kRedThreads;
    return g < kRedBlocks ? g : kRedBlocks;
}

template <int P>
static hipError_t site_mdot_p(const void *const *v, int nv, const void *w, int V, double2 *partial, double2 *out,
                              const double2 *hdr, hipStream_t st) {
    const int G = site_grid(V);
    for (int i0 = 0;; i0 += kGSSite) {
        VecList vl;
        vl.n = nv - i0 < kGSSite ? nv - i0 : kGSSite;
        if (vl.n < 0) vl.n = 0;
        for (int i = 0; i < kGSSite; i++) vl.v[i] = i < vl.n ? v[i0 + i] : w;
        hipLaunchKernelGGL(k_site_mdot<P>, dim3(G), dim3(kRedThreads), 0, st, vl, w, partial, hdr, V);
        if (vl.n > 0)
            hipLaunchKernelGGL(k_colsum, dim3(vl.n), dim3(kRedThreads), 0, st, partial, G, kGSSite + 1, out + i0);
        if (i0 + kGSSite >= nv) {
            hipLaunchKernelGGL(k_colsum, dim3(1), dim3(kRedThreads), 0, st, partial + kGSSite, G, kGSSite + 1, out + nv);
            break;
        }
    }
    return hipGetLastError();
}

template <int P>
static hipError_t site_axpy_p(const void *const *v, int nv, const double2 *coef, void *w, int V, double2 *partial,
                              double2 *norm_out, const double2 *hdr, hipStream_t st) {
    const int G = site_grid(V);
    for (int i0 = 0; i0 < nv; i0 += kGSSite) {
        VecList vl;
        vl.n = nv - i0 < kGSSite ? nv - i0 : kGSSite;
        for (int i = 0; i < kGSSite; i++) vl.v[i] = i < vl.n ? v[i0 + i] : w;
        const bool last = i0 + kGSSite >= nv;
        hipLaunchKernelGGL(k_site_axpy<P>, dim3(G), dim3(kRedThreads), 0, st, vl, coef + i0, w,
                           (last && norm_out) ? partial : (double2 *)nullptr, hdr, last ? 1 : 0, V);
        if (last && norm_out)
            hipLaunchKernelGGL(k_colsum, dim3(1), dim3(kRedThreads), 0, st, partial, G, 1, norm_out);
    }
    return hipGetLastError();
}

template <int P>
static hipError_t site_combine_p(const void *const *z, int nmax, const double2 *coef, const double2 *hdr, double2 *x,
                                 int V, hipStream_t st) {
    for (int i0 = 0;; i0 += kGSSite) {
        VecList vl;
        vl.n = nmax - i0 < kGSSite ? nmax - i0 : kGSSite;
        if (vl.n < 0) vl.n = 0;
        for (int i = 0; i < kGSSite; i++) vl.v[i] = i < vl.n ? z[i0 + i] : nullptr;
        hipLaunchKernelGGL(k_site_combine<P>, dim3(site_grid(V)), dim3(kRedThreads), 0, st, vl, coef + i0, hdr, i0,
                           x, V);
        if (i0 + kGSSite >= nmax) break;
    }
    return hipGetLastError();
}

hipError_t site_mdot(int prec, const void *const *v, int nv, const void *w, int V, double2 *partial, double2 *out,
                     const double2 *hdr, hipStream_t st) {
    switch (prec) {
    case WDIRAC_F64: return site_mdot_p<WDIRAC_F64>(v, nv, w, V, partial, out, hdr, st);
    case WDIRAC_F32: return site_mdot_p<WDIRAC_F32>(v, nv, w, V, partial, out, hdr, st);
    case WDIRAC_F16S: return site_mdot_p<WDIRAC_F16S>(v, nv, w, V, partial, out, hdr, st);
    }
    return hipErrorInvalidValue;
}

hipError_t site_axpy(int prec, const void *const *v, int nv, const double2 *coef, void *w, int V, double2 *partial,
                     double2 *norm_out, const double2 *hdr, hipStream_t st) {
    switch (prec) {
    case WDIRAC_F64: return site_axpy_p<WDIRAC_F64>(v, nv, coef, w, V, partial, norm_out, hdr, st);
    case WDIRAC_F32: return site_axpy_p<WDIRAC_F32>(v, nv, coef, w, V, partial, norm_out, hdr, st);
    case WDIRAC_F16S: return site_axpy_p<WDIRAC_F16S>(v, nv, coef, w, V, partial, norm_out, hdr, st);
    }
    return hipErrorInvalidValue;
}

hipError_t site_scale(int pin, int pout, const void *in, void *out, double mult, int V, hipStream_t st) {
    const dim3 g(site_grid(V)), b(kRedThreads);
#define WD_SITE_SCALE(PI, PO)                                                      \
    if (pin == PI && pout == PO) {                                                 \
        hipLaunchKernelGGL((k_site_scale<PI, PO>), g, b, 0, st, in, out, mult, V); \
        return hipGetLastError();                                                  \
    }
    WD_SITE_SCALE(WDIRAC_F64, WDIRAC_F64)
    WD_SITE_SCALE(WDIRAC_F64, WDIRAC_F32)
    WD_SITE_SCALE(WDIRAC_F64, WDIRAC_F16S)
    WD_SITE_SCALE(WDIRAC_F32, WDIRAC_F32)
    WD_SITE_SCALE(WDIRAC_F16S, WDIRAC_F16S)
#undef WD_SITE_SCALE
    return hipErrorInvalidValue;
}

hipError_t site_combine(int prec, const void *const *z, int nmax, const double2 *coef, const double2 *hdr, double2 *x,
                        int V, hipStream_t st) {
    switch (prec) {
    case WDIRAC_F64: return site_combine_p<WDIRAC_F64>(z, nmax, coef, hdr, x, V, st);
    case WDIRAC_F32: return site_combine_p<WDIRAC_F32>(z, nmax, coef, hdr, x, V, st);
    case WDIRAC_F16S: return site_combine_p<WDIRAC_F16S>(z, nmax, coef, hdr, x, V, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace wd
