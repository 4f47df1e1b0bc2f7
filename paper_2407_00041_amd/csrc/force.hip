// Link derivative ("force") of L = Re sum_r <eta_r, D(U) x_r>, FP64.
//
// G_rho(y) = dL/dRe U_rho(y) + i dL/dIm U_rho(y) collects two kinds of terms.
//
// Hopping (Eq. (1.13)): U_rho(y) multiplies x(y+rho) in the forward hop of
// site y and its adjoint multiplies x(y) in the backward hop of site y+rho:
//   G += -1/2 sum_s eta(y)_s q_s^H,   q = (I - gamma_rho) x(y+rho)
//   G += -1/2 sum_s p_s eta(y+rho)_s^H, p = (I + gamma_rho) x(y)
// (times -1 for a link crossing the anti-periodic T boundary).  With
// gamma = [[0, B], [B^H, 0]], q = (h, -B^H h) for h = u - B d, and
// p = (k, B^H k) for k = u + B d, so both sums reduce to half-spinor outer
// products:  sum_s eta_s q_s^H = sum_j (eta_u - B eta_d)_j h_j^H and
// sum_s p_s eta'_s^H = sum_j k_j (eta'_u + B eta'_d)_j^H.
//
// Clover (Eqs. (1.11)-(1.12)): with Q_nu,mu = Q_mu,nu^H the clover part of L
// is sum_x sum_{mu<nu} (-c_sw/16) Re tr(Q_mu,nu(x) M_mu,nu(x)) with
// M = K - K^H, K_{ba}(x) = sum_{al,be} (gamma_mu gamma_nu)_{al,be} x_{be b}
// conj(eta_{al a}) summed over right-hand sides; M_nu,mu = -M_mu,nu since
// distinct gammas anticommute.  U_rho(y) lies on two plaquettes of each plane
// (rho, nu): the one above (corners y, y+rho, y+rho+nu, y+nu; the link
// un-daggered) and the one below (corners y-nu, y-nu+rho, y+rho, y; the link
// daggered).  Cutting each of the four corner loops of Eq. (1.12) open at the
// link gives, with kappa = -c_sw/16,
//   above: G += kappa [S M(y) + M(y+rho) S + U_nu(y+rho) M(y+rho+nu) W
//                     + U_nu(y+rho) U_rho(y+nu)^H M(y+nu) U_nu(y)^H]^H,
//          S = U_nu(y+rho) W, W = U_rho(y+nu)^H U_nu(y)^H
//   below: G += kappa [U_nu(a)^H M(a) U_rho(a) U_nu(b) + U_nu(a)^H U_rho(a)
//                     M(b) U_nu(b) + R M(y+rho) + M(y) R],
//          a = y-nu, b = y-nu+rho, R = U_nu(a)^H U_rho(a) U_nu(b)
// (for P = A U B the derivative of Re tr(P M) is (B M A)^H, for
// P = A U^H B it is B M A).
//
// Two passes: force_insert_kernel forms M_mu,nu(x) for the six planes once
// per site (anti-Hermitian, 9 reals each), force_link_kernel then gathers
// them with the links around each plaquette, read from the operator's
// site-tiled FP64 copy of the links.  One work-group covers 64 sites; its
// wave w computes the links of direction w, so every branch on the direction
// is wave-uniform, and the work-group's 64 x 4 link matrices are written out
// through LDS in contiguous order.
//
// Output: P_TA(G U^H) = (M - M^H)/2 - tr(M - M^H)/6 (the su(3) projection),
// or G itself (raw), canonical [V][4][3][3] complex128.
#include "common.h"

namespace wd {

namespace {

using C = cx<double>;

constexpr int kPlanes = 6;        // (T,Z) (T,Y) (T,X) (Z,Y) (Z,X) (Y,X)
constexpr int kInsertVec = 5;     // double2 per plane and site
constexpr int kLinkSites = 64;    // sites per work-group of force_link_kernel
constexpr int kLdsPitch = 37;     // double2 per site in the LDS staging (36 + 1)

struct M3 {
    C a[9];
};

__device__ __forceinline__ C cz() { return mk<double>(0, 0); }
__device__ __forceinline__ C neg(C v) { return {-v.r, -v.i}; }
__device__ __forceinline__ C mul_i(C v) { return {-v.i, v.r}; }
__device__ __forceinline__ C mul_mi(C v) { return {v.i, -v.r}; }
// acc + conj(a) * b
__device__ __forceinline__ C cjfma(C acc, C a, C b) {
    acc.r = fma(a.r, b.r, acc.r);
    acc.r = fma(a.i, b.i, acc.r);
    acc.i = fma(a.r, b.i, acc.i);
    acc.i = fma(-a.i, b.r, acc.i);
    return acc;
}

__device__ __forceinline__ M3 mmul(const M3 &x, const M3 &y) {
    M3 m;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            C s = cmul(x.a[3 * i], y.a[j]);
            s = cfma(s, x.a[3 * i + 1], y.a[3 + j]);
            m.a[3 * i + j] = cfma(s, x.a[3 * i + 2], y.a[6 + j]);
        }
    return m;
}

// links site-tiled, U[((site / 64) * 36 + 9 mu + e) * 64 + site % 64] (e = 3 row
// + column): the lanes of a wave, at consecutive sites, read contiguous memory,
// and a link's nine entries lie 1 KB apart from one per-lane address
constexpr int kLinkTile = 64;
__device__ __forceinline__ const double2 *link_ptr(const double2 *U, int site, int mu) {
    return U + ((size_t)(site / kLinkTile) * 36 + 9 * mu) * kLinkTile + site % kLinkTile;
}

__device__ __forceinline__ M3 link(const double2 *U, int site, int mu) {
    M3 m;
    const double2 *p = link_ptr(U, site, mu);
#pragma unroll
    for (int e = 0; e < 9; e++) {
        const double2 v = p[e * kLinkTile];
        m.a[e] = {v.x, v.y};
    }
    return m;
}

__device__ __forceinline__ M3 link_dag(const double2 *U, int site, int mu) {
    M3 m;
    const double2 *p = link_ptr(U, site, mu);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const double2 v = p[(3 * i + j) * kLinkTile];
            m.a[3 * j + i] = {v.x, -v.y};
        }
    return m;
}

// Half-spinor products with the 2x2 blocks of gamma_mu = [[0, B], [B^H, 0]]:
// B_T = 1, B_Z = diag(-i, i), B_Y = [[0, -1], [1, 0]], B_X = [[0, -i], [-i, 0]].
template <int MU> __device__ __forceinline__ void bmul(C v0, C v1, C &w0, C &w1) {
    if constexpr (MU == 0) { w0 = v0; w1 = v1; }
    else if constexpr (MU == 1) { w0 = mul_mi(v0); w1 = mul_i(v1); }
    else if constexpr (MU == 2) { w0 = neg(v1); w1 = v0; }
    else { w0 = mul_mi(v1); w1 = mul_mi(v0); }
}
template <int MU> __device__ __forceinline__ void bhmul(C v0, C v1, C &w0, C &w1) {
    if constexpr (MU == 0) { w0 = v0; w1 = v1; }
    else if constexpr (MU == 1) { w0 = mul_i(v0); w1 = mul_mi(v1); }
    else if constexpr (MU == 2) { w0 = v1; w1 = neg(v0); }
    else { w0 = mul_i(v1); w1 = mul_i(v0); }
}

__device__ __forceinline__ C ld(const double2 *f, int V, int k, int s) {
    const double2 a = f[(size_t)k * V + s];
    return {a.x, a.y};
}

// ---------------------------------------------------------------------------
// pass 1: M_mu,nu(s) for the six planes, summed over right-hand sides.  A lane
// loads one chiral block of its site's eta and x (6 components each) at a time
// and folds that block's part of every plane's K into the plane's 9 reals of
// M = K - K^H (linear in K), so the spinors are read once, not once per plane,
// and only one block of them is live.
//
// m[9] = (Im M_00, Im M_11, Im M_22, M_01, M_02, M_12) as (i, i, i, re, im, re, im, re, im)
template <int MU, int NU, int BLK>
__device__ __forceinline__ void insert_plane_acc(double (&m)[9], const C (&e)[6], const C (&xv)[6]) {
    // K = sum_blk sum_be x_{blk,be} (x) conj(zeta_{blk,be}) with zeta = P_blk^H eta_blk for the chiral blocks
    // P_0 = B_mu B_nu^H and P_1 = B_mu^H B_nu of gamma_mu gamma_nu, i.e. zeta_0 = B_nu (B_mu^H eta_0) and
    // zeta_1 = B_nu^H (B_mu eta_1).
    C z[2][3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        C t0, t1;
        if constexpr (BLK == 0) {
            bhmul<MU>(e[a], e[3 + a], t0, t1);
            bmul<NU>(t0, t1, z[0][a], z[1][a]);
        } else {
            bmul<MU>(e[a], e[3 + a], t0, t1);
            bhmul<NU>(t0, t1, z[0][a], z[1][a]);
        }
    }
    M3 K;
#pragma unroll
    for (int q = 0; q < 9; q++) K.a[q] = cz();
#pragma unroll
    for (int be = 0; be < 2; be++)
#pragma unroll
        for (int b = 0; b < 3; b++)
#pragma unroll
            for (int a = 0; a < 3; a++) K.a[3 * b + a] = cjfma(K.a[3 * b + a], z[be][a], xv[3 * be + b]);
    // M = K - K^H: imaginary diagonal and upper triangle
    m[0] += 2.0 * K.a[0].i;
    m[1] += 2.0 * K.a[4].i;
    m[2] += 2.0 * K.a[8].i;
    m[3] += K.a[1].r - K.a[3].r;
    m[4] += K.a[1].i + K.a[3].i;
    m[5] += K.a[2].r - K.a[6].r;
    m[6] += K.a[2].i + K.a[6].i;
    m[7] += K.a[5].r - K.a[7].r;
    m[8] += K.a[5].i + K.a[7].i;
}

template <int BLK>
__device__ __forceinline__ void insert_block(double (&m)[kPlanes][9], const double2 *__restrict__ eta,
                                             const double2 *__restrict__ x, int V, int s) {
    C e[6], xv[6];
#pragma unroll
    for (int k = 0; k < 6; k++) {
        e[k] = ld(eta, V, 6 * BLK + k, s);
        xv[k] = ld(x, V, 6 * BLK + k, s);
    }
    insert_plane_acc<0, 1, BLK>(m[0], e, xv);
    insert_plane_acc<0, 2, BLK>(m[1], e, xv);
    insert_plane_acc<0, 3, BLK>(m[2], e, xv);
    insert_plane_acc<1, 2, BLK>(m[3], e, xv);
    insert_plane_acc<1, 3, BLK>(m[4], e, xv);
    insert_plane_acc<2, 3, BLK>(m[5], e, xv);
}

__device__ __forceinline__ void store_insert(double2 *__restrict__ out, int V, int plane, int s, const double (&m)[9]) {
    double2 *o = out + (size_t)plane * kInsertVec * V + s;
    o[0] = make_double2(m[0], m[1]);
    o[(size_t)V] = make_double2(m[2], m[3]);
    o[(size_t)2 * V] = make_double2(m[4], m[5]);
    o[(size_t)3 * V] = make_double2(m[6], m[7]);
    o[(size_t)4 * V] = make_double2(m[8], 0.0);
}

// An insertion matrix as stored: anti-Hermitian, so its diagonal is imaginary
// (d = Im M_kk) and its lower triangle is minus the conjugate of the upper
// (u = M_01, M_02, M_12).  Products with it skip the zero real parts of the
// diagonal and rebuild the lower triangle from the upper.
struct AH {
    double d[3];
    C u[3];
};

__device__ __forceinline__ AH load_ah(const double2 *__restrict__ M, int V, int plane, int s) {
    const double2 *p = M + (size_t)plane * kInsertVec * V + s;
    const double2 a = p[0], b = p[(size_t)V], c = p[(size_t)2 * V], d = p[(size_t)3 * V], e = p[(size_t)4 * V];
    AH m;
    m.d[0] = a.x;
    m.d[1] = a.y;
    m.d[2] = b.x;
    m.u[0] = {b.y, c.x};
    m.u[1] = {c.y, d.x};
    m.u[2] = {d.y, e.x};
    return m;
}

// index of M_jk (j < k) in AH::u
__device__ __forceinline__ constexpr int ah_u(int j, int k) { return j == 0 ? k - 1 : 2; }

// acc - conj(a) * b
__device__ __forceinline__ C cjfms(C acc, C a, C b) {
    acc.r = fma(-a.r, b.r, acc.r);
    acc.r = fma(-a.i, b.i, acc.r);
    acc.i = fma(-a.r, b.i, acc.i);
    acc.i = fma(a.i, b.r, acc.i);
    return acc;
}
// acc - a * conj(b)
__device__ __forceinline__ C cfms_cj(C acc, C a, C b) {
    acc.r = fma(-a.r, b.r, acc.r);
    acc.r = fma(-a.i, b.i, acc.r);
    acc.i = fma(-a.i, b.r, acc.i);
    acc.i = fma(a.r, b.i, acc.i);
    return acc;
}
// acc + i d b
__device__ __forceinline__ C cfma_i(C acc, double d, C b) {
    acc.r = fma(-d, b.i, acc.r);
    acc.i = fma(d, b.r, acc.i);
    return acc;
}

// acc += M y
__device__ __forceinline__ void ah_mul_acc(M3 &acc, const AH &m, const M3 &y) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            C s = acc.a[3 * i + j];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                if (k == i) s = cfma_i(s, m.d[i], y.a[3 * k + j]);
                else if (k > i) s = cfma(s, m.u[ah_u(i, k)], y.a[3 * k + j]);
                else s = cjfms(s, m.u[ah_u(k, i)], y.a[3 * k + j]);
            }
            acc.a[3 * i + j] = s;
        }
}
// acc += x M
__device__ __forceinline__ void mul_ah_acc(M3 &acc, const M3 &x, const AH &m) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            C s = acc.a[3 * i + j];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                if (k == j) s = cfma_i(s, m.d[j], x.a[3 * i + k]);
                else if (k < j) s = cfma(s, x.a[3 * i + k], m.u[ah_u(k, j)]);
                else s = cfms_cj(s, x.a[3 * i + k], m.u[ah_u(j, k)]);
            }
            acc.a[3 * i + j] = s;
        }
}
__device__ __forceinline__ M3 ah_mul(const AH &m, const M3 &y) {
    M3 r;
#pragma unroll
    for (int q = 0; q < 9; q++) r.a[q] = cz();
    ah_mul_acc(r, m, y);
    return r;
}

// ---------------------------------------------------------------------------
// pass 2 helpers
struct Site {
    int c[4];
};

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ int index_of(const Geom &g, const Site &p, int mu1, int d1, int mu2, int d2) {
    int s = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        int v = p.c[k];
        if (k == mu1) v = wrap(v + d1, g.n[k]);
        if (k == mu2) v = wrap(v + d2, g.n[k]);
        s += v * g.stride[k];
    }
    return s;
}

__device__ __forceinline__ int plane_of(int mu, int nu) {
    // mu < nu
    return mu == 0 ? nu - 1 : (mu == 1 ? nu + 1 : 5);
}

template <int RHO>
__device__ M3 link_force(const double2 *__restrict__ U, const double2 *__restrict__ Mins,
                         const double2 *__restrict__ eta, const double2 *__restrict__ x, int nrhs, const Geom &g,
                         int apbc, int with_clover, double csw, int y, const Site &p) {
    const int V = g.V;
    M3 G;
#pragma unroll
    for (int e = 0; e < 9; e++) G.a[e] = cz();

    // hopping
    {
        const int yp = index_of(g, p, RHO, 1, -1, 0);
        const size_t rs = (size_t)12 * V;
        for (int r = 0; r < nrhs; r++) {
            const double2 *er = eta + r * rs, *xr = x + r * rs;
            // sum_j (eta_u - B eta_d)(y)_j h_j^H,  h = x_u - B x_d at y + rho
#pragma unroll
            for (int t = 0; t < 2; t++) {
                C A[2][3], H[2][3];
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    C b0, b1;
                    if (t == 0) {
                        bmul<RHO>(ld(er, V, 6 + a, y), ld(er, V, 9 + a, y), b0, b1);
                        A[0][a] = ld(er, V, a, y) - b0;
                        A[1][a] = ld(er, V, 3 + a, y) - b1;
                        bmul<RHO>(ld(xr, V, 6 + a, yp), ld(xr, V, 9 + a, yp), b0, b1);
                        H[0][a] = ld(xr, V, a, yp) - b0;
                        H[1][a] = ld(xr, V, 3 + a, yp) - b1;
                    } else {
                        // sum_j k_j (eta'_u + B eta'_d)_j^H, k = x_u + B x_d at y, eta' = eta(y + rho)
                        bmul<RHO>(ld(xr, V, 6 + a, y), ld(xr, V, 9 + a, y), b0, b1);
                        A[0][a] = ld(xr, V, a, y) + b0;
                        A[1][a] = ld(xr, V, 3 + a, y) + b1;
                        bmul<RHO>(ld(er, V, 6 + a, yp), ld(er, V, 9 + a, yp), b0, b1);
                        H[0][a] = ld(er, V, a, yp) + b0;
                        H[1][a] = ld(er, V, 3 + a, yp) + b1;
                    }
                }
#pragma unroll
                for (int j = 0; j < 2; j++)
#pragma unroll
                    for (int a = 0; a < 3; a++)
#pragma unroll
                        for (int b = 0; b < 3; b++) G.a[3 * a + b] = cjfma(G.a[3 * a + b], H[j][b], A[j][a]);
            }
        }
        const double sgn = (apbc && RHO == 0 && p.c[0] == g.n[0] - 1) ? -1.0 : 1.0;
#pragma unroll
        for (int e = 0; e < 9; e++) G.a[e] = (-0.5 * sgn) * G.a[e];
    }

    if (!with_clover) return G;
    const double kappa = -csw / 16.0;
    for (int nu = 0; nu < 4; nu++) {
        if (nu == RHO) continue;
        const int plane = RHO < nu ? plane_of(RHO, nu) : plane_of(nu, RHO);
        const double kap = RHO < nu ? kappa : -kappa;
        const int yr = index_of(g, p, RHO, 1, -1, 0);
        const int yn = index_of(g, p, nu, 1, -1, 0);
        const int yrn = index_of(g, p, RHO, 1, nu, 1);
        const int ya = index_of(g, p, nu, -1, -1, 0);
        const int yb = index_of(g, p, nu, -1, RHO, 1);
        // plaquette above: T = M(y+rho) S + U_nu(y+rho) X, S = U_nu(y+rho) W,
        // X = U_rho(y+nu)^H M(y+nu) U_nu(y)^H + W M(y) + M(y+rho+nu) W
        {
            const M3 W = mmul(link_dag(U, yn, RHO), link_dag(U, y, nu));
            M3 X = mmul(link_dag(U, yn, RHO), ah_mul(load_ah(Mins, V, plane, yn), link_dag(U, y, nu)));
            mul_ah_acc(X, W, load_ah(Mins, V, plane, y));
            ah_mul_acc(X, load_ah(Mins, V, plane, yrn), W);
            const M3 A = link(U, yr, nu);
            const M3 S = mmul(A, W);
            M3 T = mmul(A, X);
            ah_mul_acc(T, load_ah(Mins, V, plane, yr), S);
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    const C t = T.a[3 * j + i];
                    G.a[3 * i + j].r = fma(kap, t.r, G.a[3 * i + j].r);
                    G.a[3 * i + j].i = fma(-kap, t.i, G.a[3 * i + j].i);
                }
        }
        // plaquette below: T = U_nu(a)^H Z + R M(y+rho) + M(y) R, R = U_nu(a)^H U_rho(a) U_nu(b),
        // Z = (M(a) U_rho(a) + U_rho(a) M(b)) U_nu(b)
        {
            M3 Z = ah_mul(load_ah(Mins, V, plane, ya), link(U, ya, RHO));
            mul_ah_acc(Z, link(U, ya, RHO), load_ah(Mins, V, plane, yb));
            Z = mmul(Z, link(U, yb, nu));
            const M3 E = mmul(link(U, ya, RHO), link(U, yb, nu));
            const M3 a = link_dag(U, ya, nu);
            M3 T = mmul(a, Z);
            const M3 R = mmul(a, E);
            mul_ah_acc(T, R, load_ah(Mins, V, plane, yr));
            ah_mul_acc(T, load_ah(Mins, V, plane, y), R);
#pragma unroll
            for (int e = 0; e < 9; e++) {
                G.a[e].r = fma(kap, T.a[e].r, G.a[e].r);
                G.a[e].i = fma(kap, T.a[e].i, G.a[e].i);
            }
        }
    }
    return G;
}

}  // namespace

__global__ __launch_bounds__(256) void force_insert_kernel(double2 *__restrict__ out, const double2 *__restrict__ eta,
                                                           const double2 *__restrict__ x, int nrhs, int V) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    double m[kPlanes][9];
#pragma unroll
    for (int q = 0; q < kPlanes; q++)
#pragma unroll
        for (int k = 0; k < 9; k++) m[q][k] = 0.0;
    const size_t rs = (size_t)12 * V;
    for (int r = 0; r < nrhs; r++) {
        insert_block<0>(m, eta + r * rs, x + r * rs, V, s);
        insert_block<1>(m, eta + r * rs, x + r * rs, V, s);
    }
#pragma unroll
    for (int q = 0; q < kPlanes; q++) store_insert(out, V, q, s, m[q]);
}

__global__ __launch_bounds__(256, 2) void force_link_kernel(double2 *__restrict__ out, const double2 *__restrict__ U,
                                                         const double2 *__restrict__ Mins,
                                                         const double2 *__restrict__ eta,
                                                         const double2 *__restrict__ x, int nrhs, Geom g, int apbc,
                                                         int with_clover, double csw, int raw, int eighth) {
    __shared__ double2 stage[kLinkSites * kLdsPitch];
    const int lane = threadIdx.x & 63, rho = threadIdx.x >> 6;
    // XCD-aware tiles (work-groups go round-robin to the 8 XCDs): XCD k takes the k-th eighth of every T-slice
    // (eighth = sites, a multiple of kLinkSites), and all XCDs advance through the slices together, so a tile's
    // X, Y and most Z neighbours are its own XCD's recent tiles (its L2) and its T neighbours were read by the
    // same XCD one slice earlier or are read one slice later
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int tpe = eighth / kLinkSites;
    const int t = j / tpe;
    const int slice = g.stride[0];
    const int lo = xcd * eighth + (j - t * tpe) * kLinkSites;  // the tile's first site within its T-slice
    const int hi = min((xcd + 1) * eighth, slice);             // end of this XCD's eighth
    const int base = t * slice + lo;
    const int y = base + lane;
    if (lo + lane < hi) {
        Site p;
        int r = y;
        p.c[3] = r % g.n[3]; r /= g.n[3];
        p.c[2] = r % g.n[2]; r /= g.n[2];
        p.c[1] = r % g.n[1];
        p.c[0] = r / g.n[1];
        M3 G;
        switch (rho) {
        case 0: G = link_force<0>(U, Mins, eta, x, nrhs, g, apbc, with_clover, csw, y, p); break;
        case 1: G = link_force<1>(U, Mins, eta, x, nrhs, g, apbc, with_clover, csw, y, p); break;
        case 2: G = link_force<2>(U, Mins, eta, x, nrhs, g, apbc, with_clover, csw, y, p); break;
        default: G = link_force<3>(U, Mins, eta, x, nrhs, g, apbc, with_clover, csw, y, p); break;
        }
        double2 *o = stage + lane * kLdsPitch + rho * 9;
        if (raw) {
#pragma unroll
            for (int e = 0; e < 9; e++) o[e] = make_double2(G.a[e].r, G.a[e].i);
        } else {
            const M3 F = mmul(G, link_dag(U, y, rho));
            const double tr = (2.0 / 6.0) * (F.a[0].i + F.a[4].i + F.a[8].i);  // Im tr(M - M^H) / 6
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    double fr = 0.5 * (F.a[3 * i + j].r - F.a[3 * j + i].r);
                    double fi = 0.5 * (F.a[3 * i + j].i + F.a[3 * j + i].i);
                    if (i == j) fi -= tr;
                    o[3 * i + j] = make_double2(fr, fi);
                }
        }
    }
    __syncthreads();
    const int nsite = min(kLinkSites, hi - lo);  // <= 0 for the empty tiles past a short slice's end
    double2 *dst = out + (size_t)base * 36;
    for (int t = threadIdx.x; t < nsite * 36; t += blockDim.x) dst[t] = stage[(t / 36) * kLdsPitch + t % 36];
}

// canonical [V][4][3][3] complex links -> the force kernel's site tiles (zeros past V in the last tile)
__global__ __launch_bounds__(256) void force_layout_kernel(double2 *__restrict__ dst, const double2 *__restrict__ src,
                                                           int V) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int ntile = (V + kLinkTile - 1) / kLinkTile;
    if (t >= (long long)ntile * 36 * kLinkTile) return;
    const int l = (int)(t % kLinkTile), q = (int)(t / kLinkTile % 36), tile = (int)(t / (36 * kLinkTile));
    const int s = tile * kLinkTile + l;
    dst[t] = s < V ? src[(size_t)s * 36 + q] : make_double2(0.0, 0.0);
}

size_t force_links_bytes(int V) { return (size_t)(V + kLinkTile - 1) / kLinkTile * kLinkTile * 36 * sizeof(double2); }

hipError_t force_links_layout(double *dst, const double *canon, int V, hipStream_t st) {
    const long long n = (long long)(V + kLinkTile - 1) / kLinkTile * kLinkTile * 36;
    hipLaunchKernelGGL(force_layout_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<double2 *>(dst), reinterpret_cast<const double2 *>(canon), V);
    return hipGetLastError();
}

}  // namespace wd

using namespace wd;

static int force_has_clover(const dirac_op *op) { return (op->clover_from_links && op->csw != 0.0) ? 1 : 0; }

extern "C" size_t dirac_force_workspace_bytes(const dirac_op *op) {
    if (!op || !force_has_clover(op)) return 0;
    return (size_t)kPlanes * kInsertVec * sizeof(double2) * op->g.V;
}

extern "C" int dirac_force(const dirac_op *op, double *dU, const double *eta, const double *x, int nrhs, int raw,
                           void *work, size_t work_bytes, void *stream) {
    if (!op || !dU || !eta || !x) return fail(WDIRAC_EINVAL, "null argument");
    if (nrhs < 1) return fail(WDIRAC_EINVAL, "nrhs must be >= 1");
    const int with_clover = force_has_clover(op);
    const size_t need = dirac_force_workspace_bytes(op);
    if (need && (!work || work_bytes < need))
        return fail(WDIRAC_EINVAL, "force workspace smaller than dirac_force_workspace_bytes");
    hipStream_t st = (hipStream_t)stream;
    const int V = op->g.V;
    const auto *e2 = reinterpret_cast<const double2 *>(eta);
    const auto *x2 = reinterpret_cast<const double2 *>(x);
    auto *M = reinterpret_cast<double2 *>(work);
    if (with_clover) {
        hipLaunchKernelGGL(force_insert_kernel, dim3((V + 255) / 256), dim3(256), 0, st, M, e2, x2, nrhs, V);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("force insert launch: ") + hipGetErrorString(e));
    }
    const int slice = op->g.stride[0];
    const int eighth = ((slice + 7) / 8 + kLinkSites - 1) / kLinkSites * kLinkSites;
    hipLaunchKernelGGL(force_link_kernel, dim3(op->g.n[0] * 8 * (eighth / kLinkSites)), dim3(4 * kLinkSites), 0, st,
                       reinterpret_cast<double2 *>(dU), reinterpret_cast<const double2 *>(op->links_force),
                       (const double2 *)M, e2, x2, nrhs, op->g, (op->flags & WDIRAC_ANTIPERIODIC_T) ? 1 : 0,
                       with_clover, op->csw, raw ? 1 : 0, eighth);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("force launch: ") + hipGetErrorString(e));
    return WDIRAC_OK;
}
