// Loads and stores of native-layout spinors, links and self-coupling matrices
// (layouts documented in wdirac.h and common.h).  Every access is one
// 16-, 8- or 4-byte vector per lane at consecutive sites, so a wavefront
// touches whole cache lines.
#pragma once

#include "common.h"

namespace wd {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

// Read-once data (the self-coupling matrices) may be loaded non-temporally so
// that it does not displace reusable neighbour spinors from the L2.
#ifndef WD_CLOVER_NT
#define WD_CLOVER_NT 1
#endif
template <typename V> __device__ __forceinline__ V ld_once(const V *p) {
    if (WD_CLOVER_NT) return __builtin_nontemporal_load(p);
    return *p;
}

// third row of an SU(3) matrix from the first two: conj(row0 x row1)
template <typename T> __device__ __forceinline__ void third_row(cx<T> U[9]) {
    const cx<T> a0 = U[0], a1 = U[1], a2 = U[2], b0 = U[3], b1 = U[4], b2 = U[5];
    const cx<T> c0 = cmul(a1, b2) - cmul(a2, b1);
    const cx<T> c1 = cmul(a2, b0) - cmul(a0, b2);
    const cx<T> c2 = cmul(a0, b1) - cmul(a1, b0);
    U[6] = {c0.r, -c0.i};
    U[7] = {c1.r, -c1.i};
    U[8] = {c2.r, -c2.i};
}

template <int P> struct Store;

// ---------------------------------------------------------------- FP64
template <> struct Store<WDIRAC_F64> {
    using T = double;
    static __device__ __forceinline__ void load_spinor(const void *base, int V, int s, cx<T> v[12]) {
        const double2 *p = static_cast<const double2 *>(base);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            double2 a = p[(size_t)k * V + s];
            v[k] = {a.x, a.y};
        }
    }
    // components [6 h, 6 h + 6) (chirality block h)
    static __device__ __forceinline__ void load_half(const void *base, int V, int s, int h, cx<T> v[6]) {
        const double2 *p = static_cast<const double2 *>(base) + (size_t)6 * h * V;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            double2 a = p[(size_t)k * V + s];
            v[k] = {a.x, a.y};
        }
    }
    static __device__ __forceinline__ void store_spinor(void *base, int V, int s, const cx<T> v[12]) {
        d2v *p = static_cast<d2v *>(base);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            d2v a = {v[k].r, v[k].i};
            __builtin_nontemporal_store(a, &p[(size_t)k * V + s]);
        }
    }
    static __device__ __forceinline__ void load_link(const void *base, int V, int mu, int s, cx<T> U[9],
                                                     int rows = 3) {
        const double2 *p = static_cast<const double2 *>(base);
        if (rows == 2) {
#pragma unroll
            for (int e = 0; e < 6; e++) {
                double2 a = p[op_idx(mu * 6 + e, 24, s)];
                U[e] = {a.x, a.y};
            }
            third_row(U);
            return;
        }
#pragma unroll
        for (int e = 0; e < 9; e++) {
            double2 a = p[op_idx(mu * 9 + e, 36, s)];
            U[e] = {a.x, a.y};
        }
    }
    // block b of A(x): 6 real diagonal entries and 15 complex strict-upper entries
    static __device__ __forceinline__ void load_clover(const void *base, int V, int b, int s, T d[6],
                                                       cx<T> u[15]) {
        const d2v *p = static_cast<const d2v *>(base);
#pragma unroll
        for (int e = 0; e < 3; e++) {
            d2v a = ld_once(&p[op_idx(b * 18 + e, 36, s)]);
            d[2 * e] = a.x;
            d[2 * e + 1] = a.y;
        }
#pragma unroll
        for (int e = 0; e < 15; e++) {
            d2v a = ld_once(&p[op_idx(b * 18 + 3 + e, 36, s)]);
            u[e] = {a.x, a.y};
        }
    }
    // compact block b: 28 reals (H diagonal, H upper re/im, A_01 re/im row-major, pad)
    static __device__ __forceinline__ void load_clover_compact(const void *base, int V, int b, int s, T r[28]) {
        const d2v *p = static_cast<const d2v *>(base);
#pragma unroll
        for (int q = 0; q < 14; q++) {
            d2v a = ld_once(&p[op_idx(b * 14 + q, 28, s)]);
            r[2 * q] = a.x;
            r[2 * q + 1] = a.y;
        }
    }
};

// ---------------------------------------------------------------- FP32
template <> struct Store<WDIRAC_F32> {
    using T = float;
    static __device__ __forceinline__ void load_spinor(const void *base, int V, int s, cx<T> v[12]) {
        const float4 *p = static_cast<const float4 *>(base);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            float4 a = p[(size_t)k * V + s];
            v[2 * k] = {a.x, a.y};
            v[2 * k + 1] = {a.z, a.w};
        }
    }
    static __device__ __forceinline__ void load_half(const void *base, int V, int s, int h, cx<T> v[6]) {
        const float4 *p = static_cast<const float4 *>(base) + (size_t)3 * h * V;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            float4 a = p[(size_t)k * V + s];
            v[2 * k] = {a.x, a.y};
            v[2 * k + 1] = {a.z, a.w};
        }
    }
    static __device__ __forceinline__ void store_spinor(void *base, int V, int s, const cx<T> v[12]) {
        f4v *p = static_cast<f4v *>(base);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            f4v a = {v[2 * k].r, v[2 * k].i, v[2 * k + 1].r, v[2 * k + 1].i};
            __builtin_nontemporal_store(a, &p[(size_t)k * V + s]);
        }
    }
    static __device__ __forceinline__ void load_link(const void *base, int V, int mu, int s, cx<T> U[9],
                                                     int rows = 3) {
        if (rows == 2) {
            const float4 *q = static_cast<const float4 *>(base);
#pragma unroll
            for (int e = 0; e < 3; e++) {
                float4 a = q[op_idx(mu * 3 + e, 12, s)];
                U[2 * e] = {a.x, a.y};
                U[2 * e + 1] = {a.z, a.w};
            }
            third_row(U);
            return;
        }
        const float2 *p = static_cast<const float2 *>(base);
#pragma unroll
        for (int e = 0; e < 9; e++) {
            float2 a = p[op_idx(mu * 9 + e, 36, s)];
            U[e] = {a.x, a.y};
        }
    }
    static __device__ __forceinline__ void load_clover(const void *base, int V, int b, int s, T d[6],
                                                       cx<T> u[15]) {
        const f4v *p = static_cast<const f4v *>(base);
        float r[36];
#pragma unroll
        for (int e = 0; e < 9; e++) {
            f4v a = ld_once(&p[op_idx(b * 9 + e, 18, s)]);
            r[4 * e] = a.x; r[4 * e + 1] = a.y; r[4 * e + 2] = a.z; r[4 * e + 3] = a.w;
        }
#pragma unroll
        for (int k = 0; k < 6; k++) d[k] = r[k];
#pragma unroll
        for (int k = 0; k < 15; k++) u[k] = {r[6 + 2 * k], r[7 + 2 * k]};
    }
    static __device__ __forceinline__ void load_clover_compact(const void *base, int V, int b, int s, T r[28]) {
        const f4v *p = static_cast<const f4v *>(base);
#pragma unroll
        for (int q = 0; q < 7; q++) {
            f4v a = ld_once(&p[op_idx(b * 7 + q, 14, s)]);
            r[4 * q] = a.x; r[4 * q + 1] = a.y; r[4 * q + 2] = a.z; r[4 * q + 3] = a.w;
        }
    }
};

// ---------------------------------------------------------------- FP16 + per-site scale
template <> struct Store<WDIRAC_F16S> {
    using T = float;
    static __device__ __forceinline__ const float *scales(const void *base, int V) {
        return reinterpret_cast<const float *>(static_cast<const char *>(base) + (size_t)48 * V);
    }
    static __device__ __forceinline__ void load_spinor(const void *base, int V, int s, cx<T> v[12]) {
        const half8 *p = static_cast<const half8 *>(base);
        float sc = scales(base, V)[s];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            half8 a = p[(size_t)k * V + s];
#pragma unroll
            for (int j = 0; j < 4; j++) v[4 * k + j] = {sc * (float)a[2 * j], sc * (float)a[2 * j + 1]};
        }
    }
    static __device__ __forceinline__ void load_half(const void *base, int V, int s, int h, cx<T> v[6]) {
        cx<T> w[12];
        load_spinor(base, V, s, w);
#pragma unroll
        for (int k = 0; k < 6; k++) v[k] = h ? w[6 + k] : w[k];
    }
    static __device__ __forceinline__ void store_spinor(void *base, int V, int s, const cx<T> v[12]) {
        half8 *p = static_cast<half8 *>(base);
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; k++) m = fmaxf(m, fmaxf(fabsf(v[k].r), fabsf(v[k].i)));
#pragma unroll
        for (int k = 0; k < 3; k++) {
            half8 a;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                a[2 * j] = m > 0.f ? (_Float16)(v[4 * k + j].r / m) : (_Float16)0.f;
                a[2 * j + 1] = m > 0.f ? (_Float16)(v[4 * k + j].i / m) : (_Float16)0.f;
            }
            __builtin_nontemporal_store(a, &p[(size_t)k * V + s]);
        }
        float *sp = reinterpret_cast<float *>(static_cast<char *>(base) + (size_t)48 * V);
        __builtin_nontemporal_store(m, &sp[s]);
    }
    static __device__ __forceinline__ void load_link(const void *base, int V, int mu, int s, cx<T> U[9],
                                                     int rows = 3) {
        if (rows == 2) {
            const half4 *q = static_cast<const half4 *>(base);
#pragma unroll
            for (int e = 0; e < 3; e++) {
                half4 a = q[op_idx(mu * 3 + e, 12, s)];
                U[2 * e] = {(float)a[0], (float)a[1]};
                U[2 * e + 1] = {(float)a[2], (float)a[3]};
            }
            third_row(U);
            return;
        }
        const half2v *p = static_cast<const half2v *>(base);
#pragma unroll
        for (int e = 0; e < 9; e++) {
            half2v a = p[op_idx(mu * 9 + e, 36, s)];
            U[e] = {(float)a[0], (float)a[1]};
        }
    }
    static __device__ __forceinline__ void load_clover(const void *base, int V, int b, int s, T d[6],
                                                       cx<T> u[15]) {
        const half4 *p = static_cast<const half4 *>(base);
        float r[36];
#pragma unroll
        for (int e = 0; e < 9; e++) {
            half4 a = ld_once(&p[op_idx(b * 9 + e, 18, s)]);
            r[4 * e] = (float)a[0]; r[4 * e + 1] = (float)a[1];
            r[4 * e + 2] = (float)a[2]; r[4 * e + 3] = (float)a[3];
        }
#pragma unroll
        for (int k = 0; k < 6; k++) d[k] = r[k];
#pragma unroll
        for (int k = 0; k < 15; k++) u[k] = {r[6 + 2 * k], r[7 + 2 * k]};
    }
    static __device__ __forceinline__ void load_clover_compact(const void *base, int V, int b, int s, T r[28]) {
        const half4 *p = static_cast<const half4 *>(base);
#pragma unroll
        for (int q = 0; q < 7; q++) {
            half4 a = ld_once(&p[op_idx(b * 7 + q, 14, s)]);
            r[4 * q] = (float)a[0]; r[4 * q + 1] = (float)a[1]; r[4 * q + 2] = (float)a[2]; r[4 * q + 3] = (float)a[3];
        }
    }
};

}  // namespace wd
