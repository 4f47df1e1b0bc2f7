// Link derivative ("force") of L = Re sum_r <eta_r, D(U) x_r>, FP64.
//
// G_rho(y) = dL/dRe U_rho(y) + i dL/dIm U_rho(y) collects two kinds of terms.
//
// Hopping (Eq. (1.13)): U_rho(y) multiplies x(y+rho) in the forward hop of
// site y and its adjoint multiplies x(y) in the backward hop of site y+rho:
//   G += -1/2 sum_s eta(y)_s q_s^H,   q = (I - gamma_rho) x(y+rho)
//   G += -1/2 sum_s p_s eta(y+rho)_s^H, p = (I + gamma_rho) x(y)
// (times -1 for a link crossing the anti-periodic T boundary).
//
// Clover (Eqs. (1.11)-(1.12)): with Q_nu,mu = Q_mu,nu^H the clover part of L
// is sum_x sum_{mu<nu} (-c_sw/16) Re tr(Q_mu,nu(x) M_mu,nu(x)) with
// M = K - K^H, K_{ba}(x) = sum_{al,be} (gamma_mu gamma_nu)_{al,be} x_{be b}
// conj(eta_{al a}); Re tr(Q_nu,mu M_nu,mu) = Re tr(Q_mu,nu M_mu,nu), so every
// plane nu != rho can be taken in the orientation (rho, nu).  Each leaf of
// Eq. (1.12) is the counter-clockwise plaquette loop starting at its base
// corner, and U_rho(y) lies on two plaquettes of each plane: the one above
// (corners y, y+rho, y+rho+nu, y+nu; the link un-daggered) and the one below
// (corners y-nu, y-nu+rho, y+rho, y; the link daggered).  Cutting each of the
// four corner loops open at the link gives, with kappa = -c_sw/16,
//   above: G += kappa [S M(y) + M(y+rho) S + U_nu(y+rho) M(y+rho+nu) W
//                     + U_nu(y+rho) U_rho(y+nu)^H M(y+nu) U_nu(y)^H]^H,
//          S = U_nu(y+rho) U_rho(y+nu)^H U_nu(y)^H, W = U_rho(y+nu)^H U_nu(y)^H
//   below: G += kappa [U_nu(a)^H M(a) U_rho(a) U_nu(b) + U_nu(a)^H U_rho(a)
//                     M(b) U_nu(b) + R M(y+rho) + M(y) R],
//          a = y-nu, b = y-nu+rho, R = U_nu(a)^H U_rho(a) U_nu(b)
// (for P = A U B the derivative of Re tr(P M) is (B M A)^H, for
// P = A U^H B it is B M A).
//
// Output: P_TA(G U^H) = (M - M^H)/2 - tr(M - M^H)/6 (the su(3) projection),
// or G itself (raw), canonical [V][4][3][3] complex128.
#include "common.h"

namespace wd {

namespace {

using C = cx<double>;

struct M3 {
    C a[9];
};

__device__ __forceinline__ M3 mzero() {
    M3 m;
#pragma unroll
    for (int e = 0; e < 9; e++) m.a[e] = mk<double>(0, 0);
    return m;
}

__device__ __forceinline__ M3 mmul(const M3 &x, const M3 &y) {
    M3 m;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            C s = mk<double>(0, 0);
#pragma unroll
            for (int k = 0; k < 3; k++) s = cfma(s, x.a[3 * i + k], y.a[3 * k + j]);
            m.a[3 * i + j] = s;
        }
    return m;
}

__device__ __forceinline__ M3 mdag(const M3 &x) {
    M3 m;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) m.a[3 * i + j] = {x.a[3 * j + i].r, -x.a[3 * j + i].i};
    return m;
}

__device__ __forceinline__ void madd(M3 &acc, const M3 &x, double s) {
#pragma unroll
    for (int e = 0; e < 9; e++) acc.a[e] = acc.a[e] + s * x.a[e];
}

__device__ __forceinline__ M3 link(const double2 *U, int site, int mu) {
    M3 m;
    const double2 *p = U + (size_t)(4 * site + mu) * 9;
#pragma unroll
    for (int e = 0; e < 9; e++) m.a[e] = {p[e].x, p[e].y};
    return m;
}

__device__ __forceinline__ int step(const Geom &g, int site, int mu, int d) {
    int c[4];
    int r = site;
    c[3] = r % g.n[3]; r /= g.n[3];
    c[2] = r % g.n[2]; r /= g.n[2];
    c[1] = r % g.n[1];
    c[0] = r / g.n[1];
    c[mu] = (c[mu] + d + g.n[mu]) % g.n[mu];
    return ((c[0] * g.n[1] + c[1]) * g.n[2] + c[2]) * g.n[3] + c[3];
}

// B_mu of gamma_mu = [[0, B], [B^H, 0]] (row-major 2x2)
__device__ __forceinline__ void bspin(int mu, C B[4]) {
    for (int k = 0; k < 4; k++) B[k] = mk<double>(0, 0);
    if (mu == 0) { B[0] = mk<double>(1, 0); B[3] = mk<double>(1, 0); }
    else if (mu == 1) { B[0] = mk<double>(0, -1); B[3] = mk<double>(0, 1); }
    else if (mu == 2) { B[1] = mk<double>(-1, 0); B[2] = mk<double>(1, 0); }
    else { B[1] = mk<double>(0, -1); B[2] = mk<double>(0, -1); }
}

__device__ __forceinline__ void load12(const double2 *f, int V, int s, C v[12]) {
#pragma unroll
    for (int k = 0; k < 12; k++) {
        double2 a = f[(size_t)k * V + s];
        v[k] = {a.x, a.y};
    }
}

// M(x) = K - K^H for the plane (rho, nu), summed over right-hand sides
__device__ M3 mcorner(const double2 *eta, const double2 *x, size_t rhs_stride, int nrhs, int V, int s,
                      const C P[2][4]) {
    M3 K = mzero();
    for (int r = 0; r < nrhs; r++) {
        C e[12], p[12];
        load12(eta + r * rhs_stride, V, s, e);
        load12(x + r * rhs_stride, V, s, p);
        for (int blk = 0; blk < 2; blk++)
            for (int al = 0; al < 2; al++)
                for (int be = 0; be < 2; be++) {
                    const C g = P[blk][2 * al + be];
                    if (g.r == 0.0 && g.i == 0.0) continue;
                    for (int b = 0; b < 3; b++)
                        for (int a = 0; a < 3; a++) {
                            // K_{ba} += g x_{be b} conj(eta_{al a})
                            C t = cjmul(e[6 * blk + 3 * al + a], p[6 * blk + 3 * be + b]);
                            K.a[3 * b + a] = cfma(K.a[3 * b + a], g, t);
                        }
                }
    }
    M3 M;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            M.a[3 * i + j] = {K.a[3 * i + j].r - K.a[3 * j + i].r, K.a[3 * i + j].i + K.a[3 * j + i].i};
    return M;
}

}  // namespace

__global__ __launch_bounds__(128) void force_kernel(double2 *__restrict__ out, const double2 *__restrict__ U,
                                                    const double2 *__restrict__ eta, const double2 *__restrict__ x,
                                                    int nrhs, Geom g, int apbc, int with_clover, double csw, int raw) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= 4 * g.V) return;
    const int y = tid >> 2, rho = tid & 3;
    const int V = g.V;
    const size_t rs = (size_t)12 * V;  // complex numbers per right-hand side
    M3 G = mzero();

    // hopping
    {
        const int yp = step(g, y, rho, +1);
        int c0 = y / g.stride[0];
        const double sgn = (apbc && rho == 0 && c0 == g.n[0] - 1) ? -1.0 : 1.0;
        C B[4];
        bspin(rho, B);
        for (int r = 0; r < nrhs; r++) {
            C ey[12], eyp[12], xy[12], xyp[12];
            load12(eta + r * rs, V, y, ey);
            load12(eta + r * rs, V, yp, eyp);
            load12(x + r * rs, V, y, xy);
            load12(x + r * rs, V, yp, xyp);
            // q = (I - gamma) x(y+rho) = (h, -B^H h), h = u - B d
            // p = (I + gamma) x(y)     = (k,  B^H k), k = u + B d
            C q[12], pp[12];
            for (int c = 0; c < 3; c++) {
                C d0 = xyp[6 + c], d1 = xyp[9 + c];
                C bd0 = cmul(B[0], d0) + cmul(B[1], d1), bd1 = cmul(B[2], d0) + cmul(B[3], d1);
                C h0 = xyp[c] - bd0, h1 = xyp[3 + c] - bd1;
                q[c] = h0;
                q[3 + c] = h1;
                // B^H h: (B^H)_{ij} = conj(B_{ji})
                q[6 + c] = -1.0 * (cjmul(B[0], h0) + cjmul(B[2], h1));
                q[9 + c] = -1.0 * (cjmul(B[1], h0) + cjmul(B[3], h1));
                C e0 = xy[6 + c], e1 = xy[9 + c];
                C be0 = cmul(B[0], e0) + cmul(B[1], e1), be1 = cmul(B[2], e0) + cmul(B[3], e1);
                C k0 = xy[c] + be0, k1 = xy[3 + c] + be1;
                pp[c] = k0;
                pp[3 + c] = k1;
                pp[6 + c] = cjmul(B[0], k0) + cjmul(B[2], k1);
                pp[9 + c] = cjmul(B[1], k0) + cjmul(B[3], k1);
            }
            for (int s = 0; s < 4; s++)
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) {
                        // eta(y)_s q_s^H and p_s eta(y+rho)_s^H
                        C t1 = cjmul(q[3 * s + b], ey[3 * s + a]);
                        C t2 = cjmul(eyp[3 * s + b], pp[3 * s + a]);
                        G.a[3 * a + b] = G.a[3 * a + b] + (-0.5 * sgn) * (t1 + t2);
                    }
        }
    }

    // clover leaves
    if (with_clover) {
        const double kappa = -csw / 16.0;
        C Br[4];
        bspin(rho, Br);
        const M3 Ur = link(U, y, rho);
        for (int nu = 0; nu < 4; nu++) {
            if (nu == rho) continue;
            // spin blocks of gamma_rho gamma_nu: upper B_rho B_nu^H, lower B_rho^H B_nu
            C Bn[4], P[2][4];
            bspin(nu, Bn);
            for (int i = 0; i < 2; i++)
                for (int j = 0; j < 2; j++) {
                    C su = mk<double>(0, 0), sl = mk<double>(0, 0);
                    for (int k = 0; k < 2; k++) {
                        su = cfma(su, Br[2 * i + k], mk<double>(Bn[2 * j + k].r, -Bn[2 * j + k].i));
                        sl = cfma(sl, mk<double>(Br[2 * k + i].r, -Br[2 * k + i].i), Bn[2 * k + j]);
                    }
                    P[0][2 * i + j] = su;
                    P[1][2 * i + j] = sl;
                }
            const int yr = step(g, y, rho, +1);          // y + rho
            const int yn = step(g, y, nu, +1);           // y + nu
            const int yrn = step(g, yr, nu, +1);         // y + rho + nu
            const int ya = step(g, y, nu, -1);           // y - nu
            const int yb = step(g, ya, rho, +1);         // y - nu + rho
            // plaquette above
            {
                const M3 Unb = link(U, yr, nu);                      // U_nu(y+rho)
                const M3 Urd = mdag(link(U, yn, rho));               // U_rho(y+nu)^H
                const M3 Una = mdag(link(U, y, nu));                 // U_nu(y)^H
                const M3 Wd = mmul(Urd, Una);
                const M3 S = mmul(Unb, Wd);
                M3 T = mmul(S, mcorner(eta, x, rs, nrhs, V, y, P));
                madd(T, mmul(mcorner(eta, x, rs, nrhs, V, yr, P), S), 1.0);
                madd(T, mmul(mmul(Unb, mcorner(eta, x, rs, nrhs, V, yrn, P)), Wd), 1.0);
                madd(T, mmul(mmul(mmul(Unb, Urd), mcorner(eta, x, rs, nrhs, V, yn, P)), Una), 1.0);
                madd(G, mdag(T), kappa);
            }
            // plaquette below
            {
                const M3 Unad = mdag(link(U, ya, nu));               // U_nu(a)^H
                const M3 Ura = link(U, ya, rho);                     // U_rho(a)
                const M3 Unb = link(U, yb, nu);                      // U_nu(b)
                const M3 R = mmul(mmul(Unad, Ura), Unb);
                M3 T = mmul(mmul(Unad, mcorner(eta, x, rs, nrhs, V, ya, P)), mmul(Ura, Unb));
                madd(T, mmul(mmul(mmul(Unad, Ura), mcorner(eta, x, rs, nrhs, V, yb, P)), Unb), 1.0);
                madd(T, mmul(R, mcorner(eta, x, rs, nrhs, V, yr, P)), 1.0);
                madd(T, mmul(mcorner(eta, x, rs, nrhs, V, y, P), R), 1.0);
                madd(G, T, kappa);
            }
        }
        (void)Ur;
    }

    double2 *o = out + (size_t)(4 * y + rho) * 9;
    if (raw) {
#pragma unroll
        for (int e = 0; e < 9; e++) o[e] = make_double2(G.a[e].r, G.a[e].i);
        return;
    }
    const M3 M = mmul(G, mdag(link(U, y, rho)));
    C tr = mk<double>(0, 0);
    for (int i = 0; i < 3; i++) tr = tr + mk<double>(0, 2.0 * M.a[4 * i].i);  // tr(M - M^H)
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            C f = 0.5 * (M.a[3 * i + j] - mk<double>(M.a[3 * j + i].r, -M.a[3 * j + i].i));
            if (i == j) f = f - (1.0 / 6.0) * tr;
            o[3 * i + j] = make_double2(f.r, f.i);
        }
}

}  // namespace wd

using namespace wd;

extern "C" int dirac_force(const dirac_op *op, double *dU, const double *eta, const double *x, int nrhs, int raw,
                           void *stream) {
    if (!op || !dU || !eta || !x) return fail(WDIRAC_EINVAL, "null argument");
    if (nrhs < 1) return fail(WDIRAC_EINVAL, "nrhs must be >= 1");
    const int with_clover = (op->clover_from_links && op->csw != 0.0) ? 1 : 0;
    const int n = 4 * op->g.V;
    hipLaunchKernelGGL(force_kernel, dim3((n + 127) / 128), dim3(128), 0, (hipStream_t)stream,
                       reinterpret_cast<double2 *>(dU), reinterpret_cast<const double2 *>(op->links_canon),
                       reinterpret_cast<const double2 *>(eta), reinterpret_cast<const double2 *>(x), nrhs, op->g,
                       (op->flags & WDIRAC_ANTIPERIODIC_T) ? 1 : 0, with_clover, op->csw, raw ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("force launch: ") + hipGetErrorString(e));
    return WDIRAC_OK;
}
