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

// partial[blk][i] = sum conj(v_i) w over the group's elements (i < nv),
// partial[blk][kMdot] = sum |w|^2 (real part)
template <typename S>
__global__ __launch_bounds__(kRedThreads) void k_mdot(VecList vl, const S *__restrict__ w,
                                                       double2 *__restrict__ partial, long long N) {
    __shared__ double2 lds[(kMdot + 1) * kRedThreads];
    double2 acc[kMdot + 1];
#pragma unroll
    for (int i = 0; i <= kMdot; i++) acc[i] = make_double2(0, 0);
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        const double2 we = Elem<S>::ld(w, e);
        acc[kMdot].x += we.x * we.x + we.y * we.y;
#pragma unroll
        for (int i = 0; i < kMdot; i++) {
            if (i < vl.n) {
                const double2 vi = Elem<S>::ld(static_cast<const S *>(vl.v[i]), e);
                const double2 p = cj_mul(vi, we);
                acc[i].x += p.x;
                acc[i].y += p.y;
            }
        }
    }
    block_reduce<kMdot + 1>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i <= kMdot; i++) partial[(size_t)blockIdx.x * (kMdot + 1) + i] = acc[i];
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
template <typename S>
__global__ __launch_bounds__(kRedThreads) void k_mdot_all(VecList vl, const S *__restrict__ w,
                                                           double2 *__restrict__ partial, long long N, int ngroups,
                                                           int nchunks) {
    __shared__ double2 lds[(kMdot + 1) * kRedThreads];
    const int b = blockIdx.x, xcd = b & 7, q = b >> 3;
    const int group = q % ngroups, chunk = (q / ngroups) * 8 + xcd;
    const int i0 = group * kMdot;
    double2 acc[kMdot + 1];
#pragma unroll
    for (int i = 0; i <= kMdot; i++) acc[i] = make_double2(0, 0);
    const long long stride = (long long)nchunks * blockDim.x;
    for (long long e = (long long)chunk * blockDim.x + threadIdx.x; e < N; e += stride) {
        const double2 we = Elem<S>::ld(w, e);
        if (group == 0) acc[kMdot].x += we.x * we.x + we.y * we.y;
#pragma unroll
        for (int i = 0; i < kMdot; i++) {
            if (i0 + i < vl.n) {
                const double2 vi = Elem<S>::ld(static_cast<const S *>(vl.v[i0 + i]), e);
                const double2 p = cj_mul(vi, we);
                acc[i].x += p.x;
                acc[i].y += p.y;
            }
        }
    }
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

// w -= sum_i coef[i] v_i (i < nv); partial[blk] = sum |w_new|^2 if partial
template <typename S>
__global__ __launch_bounds__(kRedThreads) void k_axpy_multi(VecList vl, const double2 *__restrict__ coef,
                                                             ScaleList sl, S *__restrict__ w,
                                                             double2 *__restrict__ partial, long long N) {
    __shared__ double2 lds[kRedThreads];
    double2 c[kGS];
#pragma unroll
    for (int i = 0; i < kGS; i++) {
        const double2 ci = i < vl.n ? coef[i] : make_double2(0, 0);
        c[i] = make_double2(ci.x * sl.s[i], ci.y * sl.s[i]);
    }
    double2 nrm[1] = {make_double2(0, 0)};
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        double2 we = Elem<S>::ld(w, e);
#pragma unroll
        for (int i = 0; i < kGS; i++) {
            if (i < vl.n) {
                const double2 vi = Elem<S>::ld(static_cast<const S *>(vl.v[i]), e);
                we.x -= c[i].x * vi.x - c[i].y * vi.y;
                we.y -= c[i].x * vi.y + c[i].y * vi.x;
            }
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

// x += sum_i c_i z_i (x FP64, z of storage S; coefficients passed by value)
template <typename S>
__global__ __launch_bounds__(kRedThreads) void k_update(VecList vl, CoefList cl, double2 *__restrict__ x,
                                                         long long N) {
    const double2 *c = cl.c;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        double2 xe = x[e];
#pragma unroll
        for (int i = 0; i < kGS; i++) {
            if (i < vl.n) {
                const double2 zi = Elem<S>::ld(static_cast<const S *>(vl.v[i]), e);
                xe.x += c[i].x * zi.x - c[i].y * zi.y;
                xe.y += c[i].x * zi.y + c[i].y * zi.x;
            }
        }
        x[e] = xe;
    }
}

// ---------------------------------------------------------------------------
// launchers

static int red_grid(long long N) {
    long long g = (N + kRedThreads - 1) / kRedThreads;
    return (int)(g < kRedBlocks ? g : kRedBlocks);
}

template <typename S>
hipError_t mdot(const void *const *v, int nv, const void *w, long long N, double2 *partial, double2 *out,
                hipStream_t st) {
    // out[0..nv) = <v_i, w>, out[nv] = |w|^2 (real part), in passes of kMdot vectors
    const int G = red_grid(N);
    for (int i0 = 0; i0 < nv || i0 == 0; i0 += kMdot) {
        VecList vl;
        vl.n = nv - i0 < kMdot ? nv - i0 : kMdot;
        if (vl.n < 0) vl.n = 0;
        for (int i = 0; i < kGS; i++) vl.v[i] = i < vl.n ? v[i0 + i] : w;
        hipLaunchKernelGGL(k_mdot<S>, dim3(G), dim3(kRedThreads), 0, st, vl, static_cast<const S *>(w), partial, N);
        if (vl.n > 0)
            hipLaunchKernelGGL(k_colsum, dim3(vl.n), dim3(kRedThreads), 0, st, partial, G, kMdot + 1, out + i0);
        if (i0 + kMdot >= nv) {
            hipLaunchKernelGGL(k_colsum, dim3(1), dim3(kRedThreads), 0, st, partial + kMdot, G, kMdot + 1, out + nv);
            break;
        }
    }
    return hipGetLastError();
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
        hipLaunchKernelGGL(k_mdot_all<S>, dim3(nchunks * ngroups), dim3(kRedThreads), 0, st, vl,
                           static_cast<const S *>(w), partial, N, ngroups, nchunks);
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
        hipLaunchKernelGGL(k_axpy_multi<S>, dim3(G), dim3(kRedThreads), 0, st, vl, coef + i0, sl, static_cast<S *>(w),
                           (last && norm_out) ? partial : (double2 *)nullptr, N);
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
        hipLaunchKernelGGL(k_update<S>, dim3(red_grid(N)), dim3(kRedThreads), 0, st, vl, cl, x, N);
    }
    return hipGetLastError();
}

template hipError_t mdot<double2>(const void *const *, int, const void *, long long, double2 *, double2 *, hipStream_t);
template hipError_t mdot_all<double2>(const void *const *, int, const void *, long long, double2 *, double2 *,
                                      hipStream_t);
template hipError_t axpy_multi<double2>(const void *const *, int, const double2 *, const double *, void *, long long,
                                        double2 *, double2 *, hipStream_t);
template hipError_t scale<double2, double2>(const void *, void *, const double2 *, bool, double, long long,
                                            hipStream_t);
template hipError_t update<double2>(const void *const *, int, const double2 *, double2 *, long long, hipStream_t);

}  // namespace wd
