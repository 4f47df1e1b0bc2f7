// Clover term from the links, once at operator creation (Sec. 2.2: the
// self-coupling matrices do not change between applications).
//
//   Q_mu,nu(x) : sum of the four plaquettes around x in the mu-nu plane,
//                Eq. (1.12);
//   C(x)       : -(1/32) sum_{mu,nu} (gamma_mu gamma_nu) (x) (Q_mu,nu - Q_nu,mu),
//                Eq. (1.11).
// Q_nu,mu(x) is the same four plaquettes traversed the other way, i.e.
// Q_mu,nu(x)^H, and the (mu,nu) and (nu,mu) terms of the sum are equal, so
// C(x) = -(1/16) sum_{mu<nu} (gamma_mu gamma_nu) (x) (Q_mu,nu - Q_mu,nu^H).
// In the chiral basis gamma_mu gamma_nu = diag(B_mu B_nu^H, B_mu^H B_nu),
// which gives the two 6x6 chirality blocks that are stored.
//
// One thread per site, FP64, canonical AoS links in, canonical packed
// [V][42] out (entry order documented in wdirac.h).
#include "common.h"

namespace wd {

namespace {

struct M3 {
    cx<double> a[9];
};

__device__ __forceinline__ M3 load_u(const double2 *links, int site, int mu) {
    M3 m;
    const double2 *p = links + (size_t)(4 * site + mu) * 9;
#pragma unroll
    for (int e = 0; e < 9; e++) m.a[e] = {p[e].x, p[e].y};
    return m;
}

__device__ __forceinline__ M3 dag(const M3 &x) {
    M3 m;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) m.a[3 * i + j] = {x.a[3 * j + i].r, -x.a[3 * j + i].i};
    return m;
}

__device__ __forceinline__ M3 mul(const M3 &x, const M3 &y) {
    M3 m;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<double> s = mk<double>(0, 0);
#pragma unroll
            for (int k = 0; k < 3; k++) s = cfma(s, x.a[3 * i + k], y.a[3 * k + j]);
            m.a[3 * i + j] = s;
        }
    return m;
}

__device__ __forceinline__ int shift(const Geom &g, const int c[4], int mu, int step, int nu = 0, int step2 = 0) {
    int d[4] = {c[0], c[1], c[2], c[3]};
    d[mu] = (d[mu] + step + g.n[mu]) % g.n[mu];
    if (step2) d[nu] = (d[nu] + step2 + g.n[nu]) % g.n[nu];
    return ((d[0] * g.n[1] + d[1]) * g.n[2] + d[2]) * g.n[3] + d[3];
}

// 2x2 spin matrices B_mu (gamma_mu = [[0, B], [B^H, 0]])
__device__ __forceinline__ void bmat(int mu, cx<double> B[4]) {
    for (int k = 0; k < 4; k++) B[k] = mk<double>(0, 0);
    if (mu == 0) { B[0] = mk<double>(1, 0); B[3] = mk<double>(1, 0); }
    if (mu == 1) { B[0] = mk<double>(0, -1); B[3] = mk<double>(0, 1); }
    if (mu == 2) { B[1] = mk<double>(-1, 0); B[2] = mk<double>(1, 0); }
    if (mu == 3) { B[1] = mk<double>(0, -1); B[2] = mk<double>(0, -1); }
}

}  // namespace

__global__ __launch_bounds__(128) void clover_build_kernel(double2 *__restrict__ out, const double2 *__restrict__ links,
                                                           Geom g) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    int c[4];
    {
        int r = s;
        c[3] = r % g.n[3]; r /= g.n[3];
        c[2] = r % g.n[2]; r /= g.n[2];
        c[1] = r % g.n[1];
        c[0] = r / g.n[1];
    }
    // accumulate the two 6x6 blocks
    cx<double> blk[2][36];
    for (int b = 0; b < 2; b++)
        for (int k = 0; k < 36; k++) blk[b][k] = mk<double>(0, 0);

    for (int mu = 0; mu < 4; mu++)
        for (int nu = mu + 1; nu < 4; nu++) {
            const int xpm = shift(g, c, mu, +1), xpn = shift(g, c, nu, +1);
            const int xmm = shift(g, c, mu, -1), xmn = shift(g, c, nu, -1);
            const int xmm_pn = shift(g, c, mu, -1, nu, +1), xmm_mn = shift(g, c, mu, -1, nu, -1);
            const int xmn_pm = shift(g, c, nu, -1, mu, +1);
            M3 q = mul(mul(load_u(links, s, mu), load_u(links, xpm, nu)),
                       mul(dag(load_u(links, xpn, mu)), dag(load_u(links, s, nu))));
            M3 t = mul(mul(load_u(links, s, nu), dag(load_u(links, xmm_pn, mu))),
                       mul(dag(load_u(links, xmm, nu)), load_u(links, xmm, mu)));
            for (int e = 0; e < 9; e++) q.a[e] = q.a[e] + t.a[e];
            t = mul(mul(dag(load_u(links, xmm, mu)), dag(load_u(links, xmm_mn, nu))),
                    mul(load_u(links, xmm_mn, mu), load_u(links, xmn, nu)));
            for (int e = 0; e < 9; e++) q.a[e] = q.a[e] + t.a[e];
            t = mul(mul(dag(load_u(links, xmn, nu)), load_u(links, xmn, mu)),
                    mul(load_u(links, xmn_pm, nu), dag(load_u(links, s, mu))));
            for (int e = 0; e < 9; e++) q.a[e] = q.a[e] + t.a[e];
            // F = Q - Q^H
            M3 F;
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++)
                    F.a[3 * i + j] = {q.a[3 * i + j].r - q.a[3 * j + i].r, q.a[3 * i + j].i + q.a[3 * j + i].i};
            // spin factors: block + = B_mu B_nu^H, block - = B_mu^H B_nu
            cx<double> Bm[4], Bn[4], P[2][4];
            bmat(mu, Bm);
            bmat(nu, Bn);
            for (int i = 0; i < 2; i++)
                for (int j = 0; j < 2; j++) {
                    cx<double> sp = mk<double>(0, 0), sm = mk<double>(0, 0);
                    for (int k = 0; k < 2; k++) {
                        sp = cfma(sp, Bm[2 * i + k], mk<double>(Bn[2 * j + k].r, -Bn[2 * j + k].i));
                        sm = cfma(sm, mk<double>(Bm[2 * k + i].r, -Bm[2 * k + i].i), Bn[2 * k + j]);
                    }
                    P[0][2 * i + j] = sp;
                    P[1][2 * i + j] = sm;
                }
            for (int b = 0; b < 2; b++)
                for (int si = 0; si < 2; si++)
                    for (int sj = 0; sj < 2; sj++) {
                        cx<double> f = (-1.0 / 16.0) * P[b][2 * si + sj];
                        for (int a = 0; a < 3; a++)
                            for (int bb = 0; bb < 3; bb++)
                                blk[b][6 * (3 * si + a) + 3 * sj + bb] =
                                    cfma(blk[b][6 * (3 * si + a) + 3 * sj + bb], f, F.a[3 * a + bb]);
                    }
        }
    double2 *o = out + (size_t)42 * s;
    for (int b = 0; b < 2; b++) {
        for (int i = 0; i < 6; i++) o[21 * b + i] = make_double2(blk[b][7 * i].r, blk[b][7 * i].i);
        int k = 6;
        for (int i = 0; i < 6; i++)
            for (int j = i + 1; j < 6; j++, k++) o[21 * b + k] = make_double2(blk[b][6 * i + j].r, blk[b][6 * i + j].i);
    }
}

hipError_t clover_build_launch(double *out, const double *links, const Geom &g, hipStream_t st) {
    hipLaunchKernelGGL(clover_build_kernel, dim3((g.V + 127) / 128), dim3(128), 0, st,
                       reinterpret_cast<double2 *>(out), reinterpret_cast<const double2 *>(links), g);
    return hipGetLastError();
}

}  // namespace wd
