// Krylov vector kernels on native fields of any storage precision (FP64,
// FP32, FP16 with a per-site scale), one thread per lattice site: a site's
// 12 complex components are decoded with the stencil's own loaders, every sum
// is accumulated in FP64, and results are re-encoded with the stencil's
// stores (FP16S: a fresh per-site scale).  With these the inner GMRES of the
// mixed solver keeps its Krylov basis in the low-precision operator's layout,
// so the operator reads and writes basis vectors directly.
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

// partial[blk][i] = sum over the group's sites of v_i^H w (i < n), [kGS] = |w|^2
template <int P>
__global__ __launch_bounds__(kRedThreads) void k_site_mdot(VecList vl, const void *__restrict__ w,
                                                            double2 *__restrict__ partial, int V) {
    __shared__ double2 lds[(kGS + 1) * kRedThreads];
    double2 acc[kGS + 1];
#pragma unroll
    for (int i = 0; i <= kGS; i++) acc[i] = make_double2(0, 0);
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < V; s += gridDim.x * blockDim.x) {
        double2 wv[12];
        SiteIO<P>::load(w, V, s, wv);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[kGS].x += wv[k].x * wv[k].x + wv[k].y * wv[k].y;
#pragma unroll
        for (int i = 0; i < kGS; i++) {
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
    reduce_block<kGS + 1>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i <= kGS; i++) partial[(size_t)blockIdx.x * (kGS + 1) + i] = acc[i];
    }
}

// w -= sum_i ml.m[i] coef[i] v_i (coef on the device, real multipliers by
// value); partial[blk] = |w_new|^2 when partial != null
template <int P>
__global__ __launch_bounds__(kRedThreads) void k_site_axpy(VecList vl, MultList ml, const double2 *__restrict__ coef,
                                                            void *__restrict__ w, double2 *__restrict__ partial, int V) {
    __shared__ double2 lds[kRedThreads];
    double2 nrm[1] = {make_double2(0, 0)};
    double2 c[kGS];
#pragma unroll
    for (int i = 0; i < kGS; i++) {
        const double2 a = i < vl.n ? coef[i] : make_double2(0, 0);
        c[i] = make_double2(a.x * ml.m[i], a.y * ml.m[i]);
    }
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < V; s += gridDim.x * blockDim.x) {
        double2 wv[12];
        SiteIO<P>::load(w, V, s, wv);
#pragma unroll
        for (int i = 0; i < kGS; i++) {
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

// x (native FP64) = keep * x + sum_i c_i z_i, z_i of precision P (coefficients by value)
template <int P>
__global__ __launch_bounds__(kRedThreads) void k_site_combine(VecList vl, CoefList cl, double2 *__restrict__ x,
                                                               int keep, int V) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < V; s += gridDim.x * blockDim.x) {
        double2 xv[12];
        if (keep) {
            SiteIO<WDIRAC_F64>::load(x, V, s, xv);
        } else {
#pragma unroll
            for (int k = 0; k < 12; k++) xv[k] = make_double2(0, 0);
        }
#pragma unroll
        for (int i = 0; i < kGS; i++) {
            if (i < vl.n) {
                double2 zv[12];
                SiteIO<P>::load(vl.v[i], V, s, zv);
                const double2 c = cl.c[i];
#pragma unroll
                for (int k = 0; k < 12; k++) {
                    xv[k].x += c.x * zv[k].x - c.y * zv[k].y;
                    xv[k].y += c.x * zv[k].y + c.y * zv[k].x;
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
                              hipStream_t st) {
    const int G = site_grid(V);
    for (int i0 = 0;; i0 += kGS) {
        VecList vl;
        vl.n = nv - i0 < kGS ? nv - i0 : kGS;
        if (vl.n < 0) vl.n = 0;
        for (int i = 0; i < kGS; i++) vl.v[i] = i < vl.n ? v[i0 + i] : w;
        hipLaunchKernelGGL(k_site_mdot<P>, dim3(G), dim3(kRedThreads), 0, st, vl, w, partial, V);
        if (vl.n > 0)
            hipLaunchKernelGGL(k_colsum, dim3(vl.n), dim3(kRedThreads), 0, st, partial, G, kGS + 1, out + i0);
        if (i0 + kGS >= nv) {
            hipLaunchKernelGGL(k_colsum, dim3(1), dim3(kRedThreads), 0, st, partial + kGS, G, kGS + 1, out + nv);
            break;
        }
    }
    return hipGetLastError();
}

template <int P>
static hipError_t site_axpy_p(const void *const *v, int nv, const double2 *coef, const double *mult, void *w, int V,
                              double2 *partial, double2 *norm_out, hipStream_t st) {
    const int G = site_grid(V);
    for (int i0 = 0; i0 < nv; i0 += kGS) {
        VecList vl;
        MultList ml;
        vl.n = nv - i0 < kGS ? nv - i0 : kGS;
        for (int i = 0; i < kGS; i++) {
            vl.v[i] = i < vl.n ? v[i0 + i] : w;
            ml.m[i] = (i < vl.n && mult) ? mult[i0 + i] : 1.0;
        }
        const bool last = i0 + kGS >= nv;
        hipLaunchKernelGGL(k_site_axpy<P>, dim3(G), dim3(kRedThreads), 0, st, vl, ml, coef + i0, w,
                           (last && norm_out) ? partial : (double2 *)nullptr, V);
        if (last && norm_out)
            hipLaunchKernelGGL(k_colsum, dim3(1), dim3(kRedThreads), 0, st, partial, G, 1, norm_out);
    }
    return hipGetLastError();
}

template <int P>
static hipError_t site_combine_p(const void *const *z, int nz, const double2 *coef, double2 *x, int V,
                                 hipStream_t st) {
    for (int i0 = 0;; i0 += kGS) {
        VecList vl;
        CoefList cl;
        vl.n = nz - i0 < kGS ? nz - i0 : kGS;
        if (vl.n < 0) vl.n = 0;
        for (int i = 0; i < kGS; i++) {
            vl.v[i] = i < vl.n ? z[i0 + i] : nullptr;
            cl.c[i] = i < vl.n ? coef[i0 + i] : make_double2(0, 0);
        }
        hipLaunchKernelGGL(k_site_combine<P>, dim3(site_grid(V)), dim3(kRedThreads), 0, st, vl, cl, x,
                           i0 > 0 ? 1 : 0, V);
        if (i0 + kGS >= nz) break;
    }
    return hipGetLastError();
}

hipError_t site_mdot(int prec, const void *const *v, int nv, const void *w, int V, double2 *partial, double2 *out,
                     hipStream_t st) {
    switch (prec) {
    case WDIRAC_F64: return site_mdot_p<WDIRAC_F64>(v, nv, w, V, partial, out, st);
    case WDIRAC_F32: return site_mdot_p<WDIRAC_F32>(v, nv, w, V, partial, out, st);
    case WDIRAC_F16S: return site_mdot_p<WDIRAC_F16S>(v, nv, w, V, partial, out, st);
    }
    return hipErrorInvalidValue;
}

hipError_t site_axpy(int prec, const void *const *v, int nv, const double2 *coef, const double *mult, void *w, int V,
                     double2 *partial, double2 *norm_out, hipStream_t st) {
    switch (prec) {
    case WDIRAC_F64: return site_axpy_p<WDIRAC_F64>(v, nv, coef, mult, w, V, partial, norm_out, st);
    case WDIRAC_F32: return site_axpy_p<WDIRAC_F32>(v, nv, coef, mult, w, V, partial, norm_out, st);
    case WDIRAC_F16S: return site_axpy_p<WDIRAC_F16S>(v, nv, coef, mult, w, V, partial, norm_out, st);
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

hipError_t site_combine(int prec, const void *const *z, int nz, const double2 *coef, double2 *x, int V,
                        hipStream_t st) {
    switch (prec) {
    case WDIRAC_F64: return site_combine_p<WDIRAC_F64>(z, nz, coef, x, V, st);
    case WDIRAC_F32: return site_combine_p<WDIRAC_F32>(z, nz, coef, x, V, st);
    case WDIRAC_F16S: return site_combine_p<WDIRAC_F16S>(z, nz, coef, x, V, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace wd
