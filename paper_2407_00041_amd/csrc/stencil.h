// Per-site building blocks of the Wilson-clover stencil (Eq. (1.13)), shared
// by the full-lattice kernels and the even-odd kernels: spin projection to a
// half-spinor, the SU(3) product, reconstruction of the lower half, and the
// products with the 6x6 chirality blocks of the site-local term.
//
// Gamma basis: gamma_mu = [[0, B_mu], [B_mu^H, 0]], B_T = 1, B_Z = -i s3,
// B_Y = -i s2, B_X = -i s1, so the projector (I + s gamma_mu) maps
// (u, d) -> (h, s B_mu^H h) with h = u + s B_mu d.
#pragma once

#include "spinor_io.h"

namespace wd {

// h = f (u + S B_mu d)  (u = spins 0,1; d = spins 2,3)
template <int MU, int S, typename T>
__device__ __forceinline__ void project(const cx<T> p[12], cx<T> h[6], T f) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cx<T> d0 = p[6 + c], d1 = p[9 + c], b0, b1;
        if (MU == 0) { b0 = d0; b1 = d1; }
        else if (MU == 1) { b0 = times_mi(d0); b1 = times_i(d1); }
        else if (MU == 2) { b0 = mk<T>(-d1.r, -d1.i); b1 = d0; }
        else { b0 = times_mi(d1); b1 = times_mi(d0); }
        if (S > 0) { h[c] = f * (p[c] + b0); h[3 + c] = f * (p[3 + c] + b1); }
        else { h[c] = f * (p[c] - b0); h[3 + c] = f * (p[3 + c] - b1); }
    }
}

// h = u + S B_mu d (no factor)
template <int MU, int S, typename T>
__device__ __forceinline__ void project_unit(const cx<T> p[12], cx<T> h[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cx<T> d0 = p[6 + c], d1 = p[9 + c], b0, b1;
        if (MU == 0) { b0 = d0; b1 = d1; }
        else if (MU == 1) { b0 = times_mi(d0); b1 = times_i(d1); }
        else if (MU == 2) { b0 = mk<T>(-d1.r, -d1.i); b1 = d0; }
        else { b0 = times_mi(d1); b1 = times_mi(d0); }
        if (S > 0) { h[c] = p[c] + b0; h[3 + c] = p[3 + c] + b1; }
        else { h[c] = p[c] - b0; h[3 + c] = p[3 + c] - b1; }
    }
}

// upper += chi; lower += S B_mu^H chi
template <int MU, int S, typename T>
__device__ __forceinline__ void reconstruct(cx<T> acc[12], const cx<T> chi[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cx<T> c0 = chi[c], c1 = chi[3 + c], l0, l1;
        acc[c] = acc[c] + c0;
        acc[3 + c] = acc[3 + c] + c1;
        if (MU == 0) { l0 = c0; l1 = c1; }
        else if (MU == 1) { l0 = times_i(c0); l1 = times_mi(c1); }
        else if (MU == 2) { l0 = c1; l1 = mk<T>(-c0.r, -c0.i); }
        else { l0 = times_i(c1); l1 = times_i(c0); }
        if (S > 0) { acc[6 + c] = acc[6 + c] + l0; acc[9 + c] = acc[9 + c] + l1; }
        else { acc[6 + c] = acc[6 + c] - l0; acc[9 + c] = acc[9 + c] - l1; }
    }
}

// chi_s = U h_s (DAGU = false) or U^H h_s (DAGU = true), s = 0, 1
template <bool DAGU, typename T>
__device__ __forceinline__ void su3_mul(const cx<T> U[9], const cx<T> h[6], cx<T> chi[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; sp++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cx<T> acc = mk<T>(0, 0);
#pragma unroll
            for (int b = 0; b < 3; b++)
                acc = DAGU ? cjfma(acc, U[3 * b + a], h[3 * sp + b]) : cfma(acc, U[3 * a + b], h[3 * sp + b]);
            chi[3 * sp + a] = acc;
        }
}

// y = A_blk x for one 6x6 Hermitian chirality block (real diagonal d, strict
// upper u in row-major pair order)
template <typename T>
__device__ __forceinline__ void clover_block(const T d[6], const cx<T> u[15], const cx<T> x[6], cx<T> y[6]) {
#pragma unroll
    for (int i = 0; i < 6; i++) y[i] = d[i] * x[i];
    int k = 0;
#pragma unroll
    for (int i = 0; i < 6; i++)
#pragma unroll
        for (int j = i + 1; j < 6; j++, k++) {
            y[i] = cfma(y[i], u[k], x[j]);
            y[j] = cjfma(y[j], u[k], x[i]);
        }
}

// y = A_blk x for a compact chirality block: A_00 = dg + H, A_11 = dg - H, A_01
// (row-major), A_10 = A_01^H; r = (h00, h11, h22, h01, h02, h12 as re/im,
// A_01 as re/im, pad)
template <typename T>
__device__ __forceinline__ void clover_block_compact(T dg, const T r[28], const cx<T> x[6], cx<T> y[6]) {
    const cx<T> u01 = {r[3], r[4]}, u02 = {r[5], r[6]}, u12 = {r[7], r[8]};
#pragma unroll
    for (int c = 0; c < 3; c++) {
        y[c] = (dg + r[c]) * x[c];
        y[3 + c] = (dg - r[c]) * x[3 + c];
    }
    // off-diagonal entries of +H (spin 0) and -H (spin 1)
    cx<T> t0 = cmul(u01, x[1]), t1 = cjmul(u01, x[0]), t2 = cjmul(u02, x[0]);
    t0 = cfma(t0, u02, x[2]);
    t1 = cfma(t1, u12, x[2]);
    t2 = cjfma(t2, u12, x[1]);
    y[0] = y[0] + t0;
    y[1] = y[1] + t1;
    y[2] = y[2] + t2;
    cx<T> b0 = cmul(u01, x[4]), b1 = cjmul(u01, x[3]), b2 = cjmul(u02, x[3]);
    b0 = cfma(b0, u02, x[5]);
    b1 = cfma(b1, u12, x[5]);
    b2 = cjfma(b2, u12, x[4]);
    y[3] = y[3] - b0;
    y[4] = y[4] - b1;
    y[5] = y[5] - b2;
    // spin-off-diagonal block A_01 and its adjoint
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const cx<T> m = {r[9 + 2 * (3 * i + j)], r[10 + 2 * (3 * i + j)]};
            y[i] = cfma(y[i], m, x[3 + j]);
            y[3 + j] = cjfma(y[3 + j], m, x[i]);
        }
}

}  // namespace wd
