// Layout conversion kernels: canonical complex128 arrays <-> native
// structure-of-arrays layouts (the paper's componentwise storage, Eq. (4.1)
// of Sec. 4.5, here with one 16-byte vector per (block, site)), and the
// reduced-precision copies of the operator data.
//
// Each thread owns one site: it reads the site's contiguous canonical record
// (whole cache lines per wavefront) and writes each native component at
// consecutive sites across the wavefront.
#include <algorithm>
#include <cstring>

#include "spinor_io.h"

namespace wd {

// canonical spinor [V][12] c128 (one rhs) -> native
template <int P>
__global__ __launch_bounds__(256) void pack_kernel(void *__restrict__ nat, const double2 *__restrict__ can,
                                                   int V, size_t rhs_bytes) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const double2 *src = can + (size_t)blockIdx.y * 12 * V + (size_t)12 * s;
    char *dst = static_cast<char *>(nat) + (size_t)blockIdx.y * rhs_bytes;
    if (P == WDIRAC_F64) {
        double2 *o = reinterpret_cast<double2 *>(dst);
#pragma unroll
        for (int k = 0; k < 12; k++) o[(size_t)k * V + s] = src[k];
    } else if (P == WDIRAC_F32) {
        float4 *o = reinterpret_cast<float4 *>(dst);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            double2 a = src[2 * k], b = src[2 * k + 1];
            o[(size_t)k * V + s] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
        }
    } else {
        // F16S: scale = fp32(max |component|), q = fp16_rn(fp32(v) / scale)
        float v[24];
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            double2 a = src[k];
            v[2 * k] = (float)a.x;
            v[2 * k + 1] = (float)a.y;
            m = fmaxf(m, fmaxf(fabsf(v[2 * k]), fabsf(v[2 * k + 1])));
        }
        half8 *o = reinterpret_cast<half8 *>(dst);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            half8 q;
#pragma unroll
            for (int j = 0; j < 8; j++) q[j] = m > 0.f ? (_Float16)(v[8 * k + j] / m) : (_Float16)0.f;
            o[(size_t)k * V + s] = q;
        }
        reinterpret_cast<float *>(dst + (size_t)48 * V)[s] = m;
    }
}

template <int P>
__global__ __launch_bounds__(256) void unpack_kernel(double2 *__restrict__ can, const void *__restrict__ nat,
                                                     int V, size_t rhs_bytes) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    double2 *dst = can + (size_t)blockIdx.y * 12 * V + (size_t)12 * s;
    const char *src = static_cast<const char *>(nat) + (size_t)blockIdx.y * rhs_bytes;
    if (P == WDIRAC_F64) {
        const double2 *i = reinterpret_cast<const double2 *>(src);
#pragma unroll
        for (int k = 0; k < 12; k++) dst[k] = i[(size_t)k * V + s];
    } else if (P == WDIRAC_F32) {
        const float4 *i = reinterpret_cast<const float4 *>(src);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            float4 a = i[(size_t)k * V + s];
            dst[2 * k] = make_double2(a.x, a.y);
            dst[2 * k + 1] = make_double2(a.z, a.w);
        }
    } else {
        const half8 *i = reinterpret_cast<const half8 *>(src);
        float m = reinterpret_cast<const float *>(src + (size_t)48 * V)[s];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            half8 q = i[(size_t)k * V + s];
#pragma unroll
            for (int j = 0; j < 4; j++)
                dst[4 * k + j] = make_double2((double)(m * (float)q[2 * j]), (double)(m * (float)q[2 * j + 1]));
        }
    }
}

hipError_t pack_launch(void *nat, const double *can, int nrhs, int prec, int V, hipStream_t st) {
    dim3 grid((V + 255) / 256, nrhs);
    size_t rb = field_rhs_bytes(prec, V);
    const double2 *c = reinterpret_cast<const double2 *>(can);
    switch (prec) {
    case WDIRAC_F64: hipLaunchKernelGGL(pack_kernel<WDIRAC_F64>, grid, dim3(256), 0, st, nat, c, V, rb); break;
    case WDIRAC_F32: hipLaunchKernelGGL(pack_kernel<WDIRAC_F32>, grid, dim3(256), 0, st, nat, c, V, rb); break;
    case WDIRAC_F16S: hipLaunchKernelGGL(pack_kernel<WDIRAC_F16S>, grid, dim3(256), 0, st, nat, c, V, rb); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t unpack_launch(double *can, const void *nat, int nrhs, int prec, int V, hipStream_t st) {
    dim3 grid((V + 255) / 256, nrhs);
    size_t rb = field_rhs_bytes(prec, V);
    double2 *c = reinterpret_cast<double2 *>(can);
    switch (prec) {
    case WDIRAC_F64: hipLaunchKernelGGL(unpack_kernel<WDIRAC_F64>, grid, dim3(256), 0, st, c, nat, V, rb); break;
    case WDIRAC_F32: hipLaunchKernelGGL(unpack_kernel<WDIRAC_F32>, grid, dim3(256), 0, st, c, nat, V, rb); break;
    case WDIRAC_F16S: hipLaunchKernelGGL(unpack_kernel<WDIRAC_F16S>, grid, dim3(256), 0, st, c, nat, V, rb); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// operator data

// canonical links [V][4][3][3] c128 -> native FP64 site-tiled 4 x rows*3 double2
// entries per site (rows = 2 keeps the first two rows of every link)
__global__ __launch_bounds__(256) void links_to_native(double2 *__restrict__ nat, const double2 *__restrict__ can,
                                                       int V, int rows) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const int ne = 3 * rows;
    for (int mu = 0; mu < 4; mu++)
        for (int e = 0; e < ne; e++) nat[op_idx(mu * ne + e, 4 * ne, s)] = can[(size_t)36 * s + 9 * mu + e];
}

// largest deviation of a link from SU(3): max |U U^H - 1| and |det U - 1|,
// folded into *worst with an integer max on the bits of a non-negative double
__global__ __launch_bounds__(256) void su3_check(const double2 *__restrict__ can, int n,
                                                 unsigned long long *__restrict__ worst) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const double2 *u = can + (size_t)9 * l;
    double dev = 0.0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double re = 0, im = 0;
            for (int k = 0; k < 3; k++) {  // (U U^H)_ij = sum_k U_ik conj(U_jk)
                double2 a = u[3 * i + k], b = u[3 * j + k];
                re += a.x * b.x + a.y * b.y;
                im += a.y * b.x - a.x * b.y;
            }
            if (i == j) re -= 1.0;
            dev = fmax(dev, sqrt(re * re + im * im));
        }
    // det by the first row's cofactors
    auto mul = [](double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); };
    double2 c0 = mul(u[4], u[8]), c0b = mul(u[5], u[7]);
    double2 c1 = mul(u[5], u[6]), c1b = mul(u[3], u[8]);
    double2 c2 = mul(u[3], u[7]), c2b = mul(u[4], u[6]);
    double2 m0 = make_double2(c0.x - c0b.x, c0.y - c0b.y), m1 = make_double2(c1.x - c1b.x, c1.y - c1b.y),
            m2 = make_double2(c2.x - c2b.x, c2.y - c2b.y);
    double2 d0 = mul(u[0], m0), d1 = mul(u[1], m1), d2 = mul(u[2], m2);
    double dr = d0.x + d1.x + d2.x - 1.0, di = d0.y + d1.y + d2.y;
    dev = fmax(dev, sqrt(dr * dr + di * di));
    if (!(dev == dev)) dev = 1e300;  // NaN
    atomicMax(worst, (unsigned long long)__double_as_longlong(dev));
}

hipError_t su3_deviation(const double *links_can_dev, int V, double *out, hipStream_t st) {
    unsigned long long *w = nullptr;
    hipError_t e = hipMalloc(&w, sizeof(*w));
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(w, 0, sizeof(*w), st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(su3_check, dim3((4 * V + 255) / 256), dim3(256), 0, st,
                           reinterpret_cast<const double2 *>(links_can_dev), 4 * V, w);
        e = hipGetLastError();
    }
    unsigned long long h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, w, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(w);
    double d;
    memcpy(&d, &h, sizeof(d));
    *out = d;
    return e;
}

// *flag becomes 1 when any of the n doubles is a NaN or an infinity
__global__ __launch_bounds__(256) void nonfinite_check(const double *__restrict__ p, size_t n,
                                                       unsigned int *__restrict__ flag) {
    bool bad = false;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) bad = bad || !isfinite(p[i]);
    if (bad) atomicOr(flag, 1u);
}

hipError_t nonfinite_any(const double *dev, size_t n, bool *out, hipStream_t st) {
    unsigned int *f = nullptr;
    hipError_t e = hipMalloc(&f, sizeof(*f));
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(f, 0, sizeof(*f), st);
    if (e == hipSuccess) {
        const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
        hipLaunchKernelGGL(nonfinite_check, dim3((unsigned)std::max<size_t>(blocks, 1)), dim3(256), 0, st, dev, n, f);
        e = hipGetLastError();
    }
    unsigned int h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, f, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(f);
    *out = h != 0;
    return e;
}

// canonical unit clover [V][42] c128 -> native FP64 A(x) = (4+m0) I + csw C(x):
// site-tiled 2 blocks x 18 double2 entries, per block 3 vectors of diagonal
// reals then 15 strict-upper complex entries.
__global__ __launch_bounds__(256) void clover_to_native(double2 *__restrict__ nat, const double2 *__restrict__ can,
                                                        int V, double diag, double csw) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const double2 *c = can + (size_t)42 * s;
#pragma unroll
    for (int b = 0; b < 2; b++) {
#pragma unroll
        for (int e = 0; e < 3; e++)
            nat[op_idx(b * 18 + e, 36, s)] =
                make_double2(diag + csw * c[21 * b + 2 * e].x, diag + csw * c[21 * b + 2 * e + 1].x);
#pragma unroll
        for (int e = 0; e < 15; e++) {
            double2 u = c[21 * b + 6 + e];
            nat[op_idx(b * 18 + 3 + e, 36, s)] = make_double2(csw * u.x, csw * u.y);
        }
    }
}

// canonical unit clover [V][42] c128 -> compact native FP64 blocks of csw C(x):
// site-tiled 2 blocks x 14 double2 entries holding 28 reals per block: H = csw (C_00 - C_11)/2
// (h00, h11, h22, then h01, h02, h12 as re, im), A_01 = csw C_01 (9 complex,
// row-major), one zero pad.  Block-local index 3 s + c (s = spin within the
// block); the packed upper entries are in row-major pair order.
__global__ __launch_bounds__(256) void clover_to_native_compact(double2 *__restrict__ nat,
                                                                const double2 *__restrict__ can, int V, double csw) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const double2 *c = can + (size_t)42 * s;
    // index of the packed strict-upper entry (i, j), i < j < 6
    auto up = [](int i, int j) { return i * 5 - i * (i - 1) / 2 + (j - i - 1); };
#pragma unroll
    for (int b = 0; b < 2; b++) {
        const double2 *cb = c + 21 * b;
        double r[28];
        for (int k = 0; k < 3; k++) r[k] = 0.5 * csw * (cb[k].x - cb[3 + k].x);
        const int hp[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (int k = 0; k < 3; k++) {
            const double2 a = cb[6 + up(hp[k][0], hp[k][1])], d = cb[6 + up(3 + hp[k][0], 3 + hp[k][1])];
            r[3 + 2 * k] = 0.5 * csw * (a.x - d.x);
            r[4 + 2 * k] = 0.5 * csw * (a.y - d.y);
        }
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                const double2 m = cb[6 + up(i, 3 + j)];
                r[9 + 2 * (3 * i + j)] = csw * m.x;
                r[10 + 2 * (3 * i + j)] = csw * m.y;
            }
        r[27] = 0.0;
        for (int q = 0; q < 14; q++) nat[op_idx(b * 14 + q, 28, s)] = make_double2(r[2 * q], r[2 * q + 1]);
    }
}

// largest |C_00 + C_11| / max(1, max|C|) over sites and blocks (the compact
// clover's structure condition), folded into *worst like su3_check
__global__ __launch_bounds__(256) void clover_structure_check(const double2 *__restrict__ can, int V,
                                                              unsigned long long *__restrict__ worst) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const double2 *c = can + (size_t)42 * s;
    auto up = [](int i, int j) { return i * 5 - i * (i - 1) / 2 + (j - i - 1); };
    double dev = 0.0, big = 1.0;
    for (int k = 0; k < 42; k++) big = fmax(big, fmax(fabs(c[k].x), fabs(c[k].y)));
    for (int b = 0; b < 2; b++) {
        const double2 *cb = c + 21 * b;
        for (int k = 0; k < 3; k++) dev = fmax(dev, fabs(cb[k].x + cb[3 + k].x));
        const int hp[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (int k = 0; k < 3; k++) {
            const double2 a = cb[6 + up(hp[k][0], hp[k][1])], d = cb[6 + up(3 + hp[k][0], 3 + hp[k][1])];
            dev = fmax(dev, fmax(fabs(a.x + d.x), fabs(a.y + d.y)));
        }
    }
    dev /= big;
    if (!(dev == dev)) dev = 1e300;  // NaN
    atomicMax(worst, (unsigned long long)__double_as_longlong(dev));
}

hipError_t clover_structure_deviation(const double *clover_can_dev, int V, double *out, hipStream_t st) {
    unsigned long long *w = nullptr;
    hipError_t e = hipMalloc(&w, sizeof(*w));
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(w, 0, sizeof(*w), st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(clover_structure_check, dim3((V + 255) / 256), dim3(256), 0, st,
                           reinterpret_cast<const double2 *>(clover_can_dev), V, w);
        e = hipGetLastError();
    }
    unsigned long long h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, w, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(w);
    double d;
    memcpy(&d, &h, sizeof(d));
    *out = d;
    return e;
}

// compact FP64 clover (2 x 14 double2 entries) -> 2 x 7 float4 / 4 x half entries (same real order)
__global__ __launch_bounds__(256) void clover_narrow_compact(float4 *__restrict__ o32, half4 *__restrict__ o16,
                                                             const double2 *__restrict__ nat, int V) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
        for (int q = 0; q < 7; q++) {
            double2 a = nat[op_idx(b * 14 + 2 * q, 28, s)];
            double2 c = nat[op_idx(b * 14 + 2 * q + 1, 28, s)];
            if (o32) o32[op_idx(b * 7 + q, 14, s)] = make_float4((float)a.x, (float)a.y, (float)c.x, (float)c.y);
            if (o16) {
                half4 h;
                h[0] = (_Float16)a.x; h[1] = (_Float16)a.y; h[2] = (_Float16)c.x; h[3] = (_Float16)c.y;
                o16[op_idx(b * 7 + q, 14, s)] = h;
            }
        }
}

// native FP64 links (two stored rows, 24 entries) -> FP32 float4 / FP16 4 x half (12 entries)
__global__ __launch_bounds__(256) void links_narrow2(float4 *__restrict__ o32, half4 *__restrict__ o16,
                                                     const double2 *__restrict__ nat, int V) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    for (int q = 0; q < 12; q++) {  // (mu, pair) pairs of the [4][6] entries
        double2 a = nat[op_idx(2 * q, 24, s)], b = nat[op_idx(2 * q + 1, 24, s)];
        if (o32) o32[op_idx(q, 12, s)] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
        if (o16) {
            half4 h;
            h[0] = (_Float16)a.x; h[1] = (_Float16)a.y; h[2] = (_Float16)b.x; h[3] = (_Float16)b.y;
            o16[op_idx(q, 12, s)] = h;
        }
    }
}

// native FP64 links -> FP32 float2 / FP16 half2 (same site-tiled entry order, flat)
__global__ __launch_bounds__(256) void links_narrow(float2 *__restrict__ o32, half2v *__restrict__ o16,
                                                    const double2 *__restrict__ nat, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 a = nat[i];
    if (o32) o32[i] = make_float2((float)a.x, (float)a.y);
    if (o16) {
        half2v h;
        h[0] = (_Float16)a.x;
        h[1] = (_Float16)a.y;
        o16[i] = h;
    }
}

// native FP64 clover (2 x 18 double2 entries) -> 2 x 9 float4 / 4 x half entries
// (the block's 36 reals in the same order, four per vector)
__global__ __launch_bounds__(256) void clover_narrow(float4 *__restrict__ o32, half4 *__restrict__ o16,
                                                     const double2 *__restrict__ nat, int V) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
        for (int q = 0; q < 9; q++) {
            double2 a = nat[op_idx(b * 18 + 2 * q, 36, s)];
            double2 c = nat[op_idx(b * 18 + 2 * q + 1, 36, s)];
            if (o32) o32[op_idx(b * 9 + q, 18, s)] = make_float4((float)a.x, (float)a.y, (float)c.x, (float)c.y);
            if (o16) {
                half4 h;
                h[0] = (_Float16)a.x; h[1] = (_Float16)a.y; h[2] = (_Float16)c.x; h[3] = (_Float16)c.y;
                o16[op_idx(b * 9 + q, 18, s)] = h;
            }
        }
}

hipError_t operator_to_native(dirac_op *op, const double *links_can_dev, const double *clover_can_dev,
                              hipStream_t st) {
    int V = op->g.V;
    dim3 grid((V + 255) / 256);
    hipLaunchKernelGGL(links_to_native, grid, dim3(256), 0, st, (double2 *)op->links64,
                       (const double2 *)links_can_dev, V, op->link_rows);
    if (op->clover_compact)
        hipLaunchKernelGGL(clover_to_native_compact, grid, dim3(256), 0, st, (double2 *)op->clover64,
                           (const double2 *)clover_can_dev, V, op->csw);
    else
        hipLaunchKernelGGL(clover_to_native, grid, dim3(256), 0, st, (double2 *)op->clover64,
                           (const double2 *)clover_can_dev, V, 4.0 + op->m0, op->csw);
    if (op->links32 || op->links16) {
        if (op->link_rows == 2) {
            hipLaunchKernelGGL(links_narrow2, grid, dim3(256), 0, st, (float4 *)op->links32, (half4 *)op->links16,
                               (const double2 *)op->links64, V);
        } else {
            size_t n = (size_t)36 * op_sites(V);
            hipLaunchKernelGGL(links_narrow, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                               (float2 *)op->links32, (half2v *)op->links16, (const double2 *)op->links64, n);
        }
        if (op->clover_compact)
            hipLaunchKernelGGL(clover_narrow_compact, grid, dim3(256), 0, st, (float4 *)op->clover32,
                               (half4 *)op->clover16, (const double2 *)op->clover64, V);
        else
            hipLaunchKernelGGL(clover_narrow, grid, dim3(256), 0, st, (float4 *)op->clover32, (half4 *)op->clover16,
                               (const double2 *)op->clover64, V);
    }
    return hipGetLastError();
}

hipError_t clover_inverse_to_native(dirac_op *op, const double *inv_can_dev, hipStream_t st) {
    int V = op->g.V;
    dim3 grid((V + 255) / 256);
    hipLaunchKernelGGL(clover_to_native, grid, dim3(256), 0, st, (double2 *)op->cinv64, (const double2 *)inv_can_dev,
                       V, 0.0, 1.0);
    if (op->cinv32 || op->cinv16)
        hipLaunchKernelGGL(clover_narrow, grid, dim3(256), 0, st, (float4 *)op->cinv32, (half4 *)op->cinv16,
                           (const double2 *)op->cinv64, V);
    return hipGetLastError();
}

}  // namespace wd
