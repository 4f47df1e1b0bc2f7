// Vector kernels of the outer FP64 Krylov solver (the non-operator work of
// Algorithm 2: inner products, norms, orthogonalisation updates, scaling and
// the solution update).
//
// A field is treated as a flat array of N = 12 V complex128 numbers (the
// native FP64 layout is a dense array, so the order does not matter for these
// operations); every sum is accumulated in FP64.  The low-precision inner
// solver uses the per-site kernels of blas_site.hip instead.
//
// Reductions are deterministic: a fixed grid of kRedBlocks work-groups, each
// thread summing a fixed strided subset, a fixed LDS tree per work-group,
// then one work-group per output summing the per-group partials in order.
// No floating-point atomics.
#include "blas.h"

namespace wd {

template <typename S> struct Elem;
template <> struct Elem<double2> {
    static __device__ __forceinline__ double2 ld(const double2 *p, long long i) { return p[i]; }
    static __device__ __forceinline__ void st(double2 *p, long long i, double2 v) { p[i] = v; }
};

__device__ __forceinline__ double2 cj_mul(double2 a, double2 b) {  // conj(a) b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// LDS tree reduction of NV complex values per thread; thread 0 gets the sums
template <int NV>
__device__ __forceinline__ void block_reduce(double2 (&v)[NV], double2 *lds) {
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

// Inner products of w with up to kGS basis vectors in ONE launch.  The grid
// is (vector group of kMdot, element chunk) work-groups, dealt so that the
// groups of one chunk are consecutive work-groups of the same XCD (the
// hardware hands work-groups to the 8 XCDs round-robin): after the first
// group, a chunk of w comes from that XCD's L2, so w crosses HBM about once
// whatever the number of vectors.  partial[(chunk * ngroups + group) *
// (kMdot + 1) + i] = sum conj(v_{kMdot group + i}) w over the chunk; column
// kMdot of group 0 holds sum |w|^2.
template <typename S, int NV>
__device__ __forceinline__ void mdot_chunk(const VecList &vl, int i0, const S *__restrict__ w, long long e0,
                                           long long stride, long long N, double2 (&acc)[kMdot + 1]) {
    for (long long e = e0; e < N; e += stride) {
        const double2 we = Elem<S>::ld(w, e);
        double2 vv[NV > 0 ? NV : 1];
#pragma unroll
        for (int i = 0; i < NV; i++) vv[i] = Elem<S>::ld(static_cast<const S *>(vl.v[i0 + i]), e);
        acc[kMdot].x += we.x * we.x + we.y * we.y;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const double2 p = cj_mul(vv[i], we);
            acc[i].x += p.x;
            acc[i].y += p.y;
        }
    }
}

// Inner products of w with up to kGS basis vectors in ONE launch.  The grid
// is (vector group of kMdot, element chunk) work-groups, dealt so that the
// groups of one chunk are consecutive work-groups of the same XCD (the
// hardware hands work-groups to the 8 XCDs round-robin): after the first
// group, a chunk of w comes from that XCD's L2, so w crosses HBM about once
// whatever the number of vectors.  partial[(chunk * ngroups + group) *
// (kMdot + 1) + i] = sum conj(v_{kMdot group + i}) w over the chunk; column
// kMdot holds sum |w|^2 (read from group 0).  Every group but the last has
// kMdot vectors, the last NL (a template parameter, so that each element's
// loads of all vectors are issued together, without a branch between them).
template <typename S, int NL>
__global__ __launch_bounds__(kRedThreads) void k_mdot_all(VecList vl, const S *__restrict__ w,
                                                           double2 *__restrict__ partial, long long N, int ngroups,
                                                           int nchunks) {
    __shared__ double2 lds[(kMdot + 1) * kRedThreads];
    const int b = blockIdx.x, xcd = b & 7, q = b >> 3;
    const int group = q % ngroups, chunk = (q / ngroups) * 8 + xcd;
    double2 acc[kMdot + 1];
#pragma unroll
    for (int i = 0; i <= kMdot; i++) acc[i] = make_double2(0, 0);
    const long long stride = (long long)nchunks * blockDim.x, e0 = (long long)chunk * blockDim.x + threadIdx.x;
    if (group < ngroups - 1)
        mdot_chunk<S, kMdot>(vl, group * kMdot, w, e0, stride, N, acc);
    else
        mdot_chunk<S, NL>(vl, group * kMdot, w, e0, stride, N, acc);
    block_reduce<kMdot + 1>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i <= kMdot; i++) partial[((size_t)chunk * ngroups + group) * (kMdot + 1) + i] = acc[i];
    }
}

// out[i] (i < nv) = sum over chunks of the inner-product partials of vector i, out[nv].x = |w|^2; one work-group
// per output, chunks summed in order
__global__ __launch_bounds__(kRedThreads) void k_colsum_groups(const double2 *__restrict__ partial, int nchunks,
                                                                int ngroups, int nv, double2 *__restrict__ out) {
    __shared__ double2 lds[kRedThreads];
    const int i = blockIdx.x;
    const int group = i < nv ? i / kMdot : 0, col = i < nv ? i % kMdot : kMdot;
    double2 a[1] = {make_double2(0, 0)};
    for (int c = threadIdx.x; c < nchunks; c += blockDim.x) {
        const double2 p = partial[((size_t)c * ngroups + group) * (kMdot + 1) + col];
        a[0].x += p.x;
        a[0].y += p.y;
    }
    block_reduce<1>(a, lds);
    if (threadIdx.x == 0) out[i] = a[0];
}

// out[i] = sum over groups of partial[g][i], i < ncols (one work-group per i);
// stride = number of columns per partial row
__global__ __launch_bounds__(kRedThreads) void k_colsum(const double2 *__restrict__ partial, int ngroups, int stride,
                                                        double2 *__restrict__ out) {
    __shared__ double2 lds[kRedThreads];
    double2 a[1] = {make_double2(0, 0)};
    for (int g = threadIdx.x; g < ngroups; g += blockDim.x) {
        double2 p = partial[(size_t)g * stride + blockIdx.x];
        a[0].x += p.x;
        a[0].y += p.y;
    }
    block_reduce<1>(a, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = a[0];
}

// cs[i] = coef[i] * sl.s[i], i < n (one work-group of kGS lanes)
__global__ void k_scale_coef(const double2 *__restrict__ coef, ScaleList sl, int n, double2 *__restrict__ cs) {
    const int i = threadIdx.x;
    if (i < n) cs[i] = make_double2(coef[i].x * sl.s[i], coef[i].y * sl.s[i]);
}

// w -= sum_i cs[i] v_i over NV vectors (a template parameter: the loads of all NV vectors of an element are issued
// together; the coefficients are read with uniform addresses, so they stay in scalar registers);
// partial[blk] = sum |w_new|^2 if partial
template <typename S, int NV>
__global__ __launch_bounds__(kRedThreads) void k_axpy_multi(VecList vl, const double2 *__restrict__ cs,
                                                             S *__restrict__ w, double2 *__restrict__ partial,
                                                             long long N) {
    __shared__ double2 lds[kRedThreads];
    double2 nrm[1] = {make_double2(0, 0)};
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        double2 we = Elem<S>::ld(w, e);
        double2 vv[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) vv[i] = Elem<S>::ld(static_cast<const S *>(vl.v[i]), e);
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const double2 c = cs[i];
            we.x -= c.x * vv[i].x - c.y * vv[i].y;
            we.y -= c.x * vv[i].y + c.y * vv[i].x;
        }
        Elem<S>::st(w, e, we);
        nrm[0].x += we.x * we.x + we.y * we.y;
    }
    if (partial) {
        block_reduce<1>(nrm, lds);
        if (threadIdx.x == 0) partial[blockIdx.x] = nrm[0];
    }
}

// out = in * s * mult, s = sc[0].x, 1/sqrt(sc[0].x) when inv_sqrt, or 1 when sc is null
template <typename SI, typename SO>
__global__ __launch_bounds__(kRedThreads) void k_scale(const SI *__restrict__ in, SO *__restrict__ out,
                                                        const double2 *__restrict__ sc, int inv_sqrt, double mult,
                                                        long long N) {
    const double s = (sc ? (inv_sqrt ? 1.0 / sqrt(sc[0].x) : sc[0].x) : 1.0) * mult;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        double2 a = Elem<SI>::ld(in, e);
        Elem<SO>::st(out, e, make_double2(a.x * s, a.y * s));
    }
}

// r = b - w, partial[blk] = sum |r|^2
__global__ __launch_bounds__(kRedThreads) void k_residual(const double2 *__restrict__ b, const double2 *__restrict__ w,
                                                           double2 *__restrict__ r, double2 *__restrict__ partial,
                                                           long long N) {
    __shared__ double2 lds[kRedThreads];
    double2 nrm[1] = {make_double2(0, 0)};
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        double2 a = b[e], c = w[e];
        double2 d = make_double2(a.x - c.x, a.y - c.y);
        r[e] = d;
        nrm[0].x += d.x * d.x + d.y * d.y;
    }
    block_reduce<1>(nrm, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = nrm[0];
}

// x += sum_i c_i z_i over NV vectors (x FP64, z of storage S; coefficients passed by value)
template <typename S, int NV>
__global__ __launch_bounds__(kRedThreads) void k_update(VecList vl, CoefList cl, double2 *__restrict__ x,
                                                         long long N) {
    const double2 *c = cl.c;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        double2 xe = x[e];
        double2 zz[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) zz[i] = Elem<S>::ld(static_cast<const S *>(vl.v[i]), e);
#pragma unroll
        for (int i = 0; i < NV; i++) {
            xe.x += c[i].x * zz[i].x - c[i].y * zz[i].y;
            xe.y += c[i].x * zz[i].y + c[i].y * zz[i].x;
        }
        x[e] = xe;
    }
}

// ---------------------------------------------------------------------------
// launchers

// one case per vector count of a pass, 1 .. kGS
#define WD_NV_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) \
    X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)
static_assert(kGS == 32, "WD_NV_CASES lists 1 .. kGS");

static int red_grid(long long N) {
    long long g = (N + kRedThreads - 1) / kRedThreads;
    return (int)(g < kRedBlocks ? g : kRedBlocks);
}

template <typename S>
hipError_t mdot_all(const void *const *v, int nv, const void *w, long long N, double2 *partial, double2 *out,
                    hipStream_t st) {
    const int nchunks = (red_grid(N) + 7) / 8 * 8;
    for (int i0 = 0; i0 < nv || i0 == 0; i0 += kGS) {
        VecList vl;
        vl.n = nv - i0 < kGS ? nv - i0 : kGS;
        if (vl.n < 0) vl.n = 0;
        for (int i = 0; i < kGS; i++) vl.v[i] = i < vl.n ? v[i0 + i] : w;
        const int ngroups = vl.n > 0 ? (vl.n + kMdot - 1) / kMdot : 1;
        const int nl = vl.n - (ngroups - 1) * kMdot;  // vectors of the last group (0 with none: |w|^2 only)
        const dim3 grid(nchunks * ngroups), blk(kRedThreads);
        const S *ws = static_cast<const S *>(w);
        switch (nl) {
#define WD_MDOT_CASE(n) \
    case n: hipLaunchKernelGGL((k_mdot_all<S, n>), grid, blk, 0, st, vl, ws, partial, N, ngroups, nchunks); break;
            WD_MDOT_CASE(0) WD_MDOT_CASE(1) WD_MDOT_CASE(2) WD_MDOT_CASE(3) WD_MDOT_CASE(4)
            WD_MDOT_CASE(5) WD_MDOT_CASE(6) WD_MDOT_CASE(7) WD_MDOT_CASE(8)
#undef WD_MDOT_CASE
        default: return hipErrorInvalidValue;
        }
        const bool last = i0 + kGS >= nv;
        // outputs of this launch: its vl.n products, plus |w|^2 after the last one
        hipLaunchKernelGGL(k_colsum_groups, dim3(vl.n + (last ? 1 : 0)), dim3(kRedThreads), 0, st, partial, nchunks,
                           ngroups, vl.n, out + i0);
        if (last) break;
    }
    return hipGetLastError();
}

template <typename S>
hipError_t axpy_multi(const void *const *v, int nv, const double2 *coef, const double *cscale, void *w, long long N,
                      double2 *partial, double2 *norm_out, hipStream_t st) {
    const int G = red_grid(N);
    for (int i0 = 0; i0 < nv; i0 += kGS) {
        VecList vl;
        ScaleList sl;
        vl.n = nv - i0 < kGS ? nv - i0 : kGS;
        for (int i = 0; i < kGS; i++) {
            vl.v[i] = i < vl.n ? v[i0 + i] : w;
            sl.s[i] = (i < vl.n && cscale) ? cscale[i0 + i] : 1.0;
        }
        const bool last = i0 + kGS >= nv;
        double2 *pt = (last && norm_out) ? partial : (double2 *)nullptr;
        S *ws = static_cast<S *>(w);
        // scaled coefficients after the first kRedBlocks entries of partial (the norm partials of this pass)
        double2 *cs = partial + kRedBlocks;
        hipLaunchKernelGGL(k_scale_coef, dim3(1), dim3(kGS), 0, st, coef + i0, sl, vl.n, cs);
        switch (vl.n) {
#define WD_AXPY_CASE(n) \
    case n: hipLaunchKernelGGL((k_axpy_multi<S, n>), dim3(G), dim3(kRedThreads), 0, st, vl, cs, ws, pt, N); break;
            WD_NV_CASES(WD_AXPY_CASE)
#undef WD_AXPY_CASE
        default: return hipErrorInvalidValue;
        }
        if (last && norm_out)
            hipLaunchKernelGGL(k_colsum, dim3(1), dim3(kRedThreads), 0, st, partial, G, 1, norm_out);
    }
    return hipGetLastError();
}

template <typename SI, typename SO>
hipError_t scale(const void *in, void *out, const double2 *sc, bool inv_sqrt, double mult, long long N,
                 hipStream_t st) {
    hipLaunchKernelGGL((k_scale<SI, SO>), dim3(red_grid(N)), dim3(kRedThreads), 0, st, static_cast<const SI *>(in),
                       static_cast<SO *>(out), sc, inv_sqrt ? 1 : 0, mult, N);
    return hipGetLastError();
}

hipError_t residual(const double2 *b, const double2 *w, double2 *r, long long N, double2 *partial, double2 *norm_out,
                    hipStream_t st) {
    const int G = red_grid(N);
    hipLaunchKernelGGL(k_residual, dim3(G), dim3(kRedThreads), 0, st, b, w, r, partial, N);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(kRedThreads), 0, st, partial, G, 1, norm_out);
    return hipGetLastError();
}

template <typename S>
hipError_t update(const void *const *z, int nz, const double2 *coef, double2 *x, long long N, hipStream_t st) {
    for (int i0 = 0; i0 < nz; i0 += kGS) {
        VecList vl;
        CoefList cl;
        vl.n = nz - i0 < kGS ? nz - i0 : kGS;
        for (int i = 0; i < kGS; i++) {
            vl.v[i] = i < vl.n ? z[i0 + i] : x;
            cl.c[i] = i < vl.n ? coef[i0 + i] : make_double2(0, 0);
        }
        switch (vl.n) {
#define WD_UPDATE_CASE(n) \
    case n: hipLaunchKernelGGL((k_update<S, n>), dim3(red_grid(N)), dim3(kRedThreads), 0, st, vl, cl, x, N); break;
            WD_NV_CASES(WD_UPDATE_CASE)
#undef WD_UPDATE_CASE
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

template hipError_t mdot_all<double2>(const void *const *, int, const void *, long long, double2 *, double2 *,
                                      hipStream_t);
template hipError_t axpy_multi<double2>(const void *const *, int, const double2 *, const double *, void *, long long,
                                        double2 *, double2 *, hipStream_t);
template hipError_t scale<double2, double2>(const void *, void *, const double2 *, bool, double, long long,
                                            hipStream_t);
template hipError_t update<double2>(const void *const *, int, const double2 *, double2 *, long long, hipStream_t);

}  // namespace wd
