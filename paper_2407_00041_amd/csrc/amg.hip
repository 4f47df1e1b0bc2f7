// Two-level aggregation multigrid: the AMG preconditioner Sec. 1.3 outlines
// (a coarse operator D_c acting like D on the near kernel with D's
// nearest-neighbour structure, restriction R and prolongation P, the subspace
// correction z <- z + P D_c^{-1} R r together with the smoother, and a setup
// that approximates right eigenvectors of small eigenvalues), made definite
// as follows:
//   * aggregates are a_T x a_Z x a_Y x a_X blocks of sites, one coarse site
//     each (lexicographic block coordinates);
//   * P is block-diagonal over (aggregate, chirality): the N test vectors
//     restricted to the aggregate's sites and to spins 0,1 (or 2,3) are
//     orthonormalised in order, R = P^H, D_c = P^H D P;
//   * M r = e + SAP(r - D e) with e = P D_c^{-1} P^H r, D_c^{-1} by GMRES on
//     the coarse lattice to a relative tolerance;
//   * setup: SAP inverse iteration on the caller's (random) test vectors, then
//     two-level inverse iteration v <- M v / |M v|, rebuilding P and D_c after
//     every pass.
//
// Storage: P (FP64, or FP32 with amg_params.prec) aggregate-major and component-major inside a column,
// [Vc][N][12][na] complex, so consecutive lanes (consecutive local sites) read
// consecutive entries and a chirality block of a column is one contiguous run; D_c as [Vc][5][2N][2N] complex, the block of
// a coarse site with itself and with its +T, +Z, +Y, +X neighbours (row-major,
// rows = output unknowns s*N + k).  The block to the -mu neighbour is not
// stored: gamma_5-hermiticity of D and the chirality split of P give
// D_c[a, a - mu] = G5 D_c[a - mu, a]^H G5 (G5 = +1 on s = 0, -1 on s = 1), hop
// by hop, so the coarse apply reads the neighbour's forward block transposed.
// Coarse vectors: [Vc][2][N] complex.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <vector>

#include "amg.h"
#include "blas.h"
#include "dslash.h"
#include "stencil.h"

namespace wd {

namespace {

using zc = std::complex<double>;

#define AMG_TRY(expr)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(WDIRAC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t a256(size_t n) { return (n + 255) / 256 * 256; }

// ---------------------------------------------------------------------------
// geometry helpers

__device__ __forceinline__ void site_coords(const Geom &g, int s, int c[4]) {
    c[3] = s % g.n[3];
    int r = s / g.n[3];
    c[2] = r % g.n[2];
    r /= g.n[2];
    c[1] = r % g.n[1];
    c[0] = r / g.n[1];
}

// aggregate and local index (local x fastest) of site coordinates
__device__ __forceinline__ void agg_of(const AmgGeom &ag, const int c[4], int &a, int &j) {
    a = 0;
    j = 0;
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        a = a * ag.nc[mu] + c[mu] / ag.a[mu];
        j = j * ag.a[mu] + c[mu] % ag.a[mu];
    }
}

// site coordinates of local index j of aggregate a
__device__ __forceinline__ void coords_of(const AmgGeom &ag, int a, int j, int c[4]) {
    int ca[4], lj[4];
#pragma unroll
    for (int mu = 3; mu >= 0; mu--) {
        ca[mu] = a % ag.nc[mu];
        a /= ag.nc[mu];
        lj[mu] = j % ag.a[mu];
        j /= ag.a[mu];
    }
#pragma unroll
    for (int mu = 0; mu < 4; mu++) c[mu] = ca[mu] * ag.a[mu] + lj[mu];
}

__device__ __forceinline__ int site_index(const Geom &g, const int c[4]) {
    return ((c[0] * g.n[1] + c[1]) * g.n[2] + c[2]) * g.n[3] + c[3];
}

// start of column k of aggregate a in P: entry (component e, local site j) at + e * na + j
__device__ __forceinline__ size_t pcol(const AmgGeom &ag, int a, int k) {
    return (size_t)(a * ag.N + k) * 12 * ag.na;
}

// deterministic work-group sum of M complex values (every thread gets the totals); lds holds [4][M]
template <int M> __device__ __forceinline__ void wg_sum(double2 v[M], double2 *lds) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int m = 0; m < M; m++) {
            v[m].x += __shfl_xor(v[m].x, o, 64);
            v[m].y += __shfl_xor(v[m].y, o, 64);
        }
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int m = 0; m < M; m++) lds[w * M + m] = v[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < M; m++) {
        double2 t = make_double2(0.0, 0.0);
        for (int q = 0; q < nw; q++) {
            t.x += lds[q * M + m].x;
            t.y += lds[q * M + m].y;
        }
        v[m] = t;
    }
    __syncthreads();
}

// acc += conj(a) b
__device__ __forceinline__ void cj_acc(double2 &acc, double2 a, double2 b) {
    acc.x += a.x * b.x + a.y * b.y;
    acc.y += a.x * b.y - a.y * b.x;
}

// entries of P in storage S (double2: FP64, float2: FP32, round to nearest), arithmetic always in FP64
__device__ __forceinline__ double2 pld(const double2 *p) { return *p; }
__device__ __forceinline__ double2 pld(const float2 *p) {
    const float2 v = *p;
    return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ void pst(double2 *p, double2 v) { *p = v; }
__device__ __forceinline__ void pst(float2 *p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }

// ---------------------------------------------------------------------------
// kernels

// dir 0: P[a][k][j] = test_k(site);  dir 1: out_k(site) = P[a][k][j]   (native FP64 fields)
template <typename S>
__global__ __launch_bounds__(kAmgThreads) void k_gather(double2 *fields, S *P, Geom g, AmgGeom ag, int dir) {
    const int s = blockIdx.x * kAmgThreads + threadIdx.x;
    if (s >= g.V) return;
    const int k = blockIdx.y;
    int c[4], a, j;
    site_coords(g, s, c);
    agg_of(ag, c, a, j);
    double2 *f = fields + (size_t)k * 12 * g.V;
    S *q = P + pcol(ag, a, k) + j;
#pragma unroll
    for (int e = 0; e < 12; e++) {
        if (dir == 0) pst(q + (size_t)e * ag.na, f[(size_t)e * g.V + s]);
        else f[(size_t)e * g.V + s] = pld(q + (size_t)e * ag.na);
    }
}

// Gram-Schmidt (classical, two passes) of the N columns of one (aggregate, chirality) in order; flag |= 1 when a
// column is dependent on the previous ones (remaining norm <= 1e-12 of its original norm)
template <typename S>
__global__ __launch_bounds__(kAmgThreads) void k_block_gs(S *P, AmgGeom ag, int *flag) {
    __shared__ double2 red[4 * kAmgChunk];
    __shared__ double2 h[kAmgMaxTv];
    const int a = blockIdx.x, sp = blockIdx.y;
    const int L = 6 * ag.na;
    // the chirality's 6 components of all na sites are one contiguous run of the column
    auto at = [&](int k, int e) { return P + pcol(ag, a, k) + (size_t)6 * sp * ag.na + e; };
    auto el = [&](int k, int e) { return pld(at(k, e)); };
    for (int k = 0; k < ag.N; k++) {
        double2 n0[1] = {make_double2(0.0, 0.0)};
        for (int e = threadIdx.x; e < L; e += kAmgThreads) {
            const double2 w = el(k, e);
            n0[0].x += w.x * w.x + w.y * w.y;
        }
        wg_sum<1>(n0, red);
        for (int pass = 0; pass < 2 && k > 0; pass++) {
            for (int j0 = 0; j0 < k; j0 += kAmgChunk) {
                const int nj = min(kAmgChunk, k - j0);
                double2 acc[kAmgChunk];
#pragma unroll
                for (int q = 0; q < kAmgChunk; q++) acc[q] = make_double2(0.0, 0.0);
                for (int e = threadIdx.x; e < L; e += kAmgThreads) {
                    const double2 w = el(k, e);
#pragma unroll
                    for (int q = 0; q < kAmgChunk; q++)
                        if (q < nj) cj_acc(acc[q], el(j0 + q, e), w);
                }
                wg_sum<kAmgChunk>(acc, red);
                if (threadIdx.x == 0) {
#pragma unroll
                    for (int q = 0; q < kAmgChunk; q++)
                        if (q < nj) h[j0 + q] = acc[q];
                }
            }
            __syncthreads();
            for (int e = threadIdx.x; e < L; e += kAmgThreads) {
                double2 w = el(k, e);
                for (int q = 0; q < k; q++) {
                    const double2 v = el(q, e), c = h[q];
                    w.x -= c.x * v.x - c.y * v.y;
                    w.y -= c.x * v.y + c.y * v.x;
                }
                pst(at(k, e), w);
            }
            __syncthreads();
        }
        double2 nk[1] = {make_double2(0.0, 0.0)};
        for (int e = threadIdx.x; e < L; e += kAmgThreads) {
            const double2 w = el(k, e);
            nk[0].x += w.x * w.x + w.y * w.y;
        }
        wg_sum<1>(nk, red);
        const bool dep = !(nk[0].x > 1e-24 * n0[0].x);
        if (dep && threadIdx.x == 0) atomicOr(flag, 1);
        const double inv = dep ? 0.0 : 1.0 / sqrt(nk[0].x);
        for (int e = threadIdx.x; e < L; e += kAmgThreads) {
            const double2 w = el(k, e);
            pst(at(k, e), make_double2(w.x * inv, w.y * inv));
        }
        __syncthreads();
    }
}

// column (sp, l) of aggregate `src` at the site with coordinates c (zero off its chirality), into p[12]
template <typename S>
__device__ __forceinline__ void column_at(const S *P, const AmgGeom &ag, int src, int l, int sp,
                                          const int c[4], cx<double> p[12]) {
    int a, j;
    agg_of(ag, c, a, j);
#pragma unroll
    for (int e = 0; e < 12; e++) p[e] = mk<double>(0.0, 0.0);
    if (a != src) return;
    const S *q = P + pcol(ag, a, l) + (size_t)6 * sp * ag.na + j;
#pragma unroll
    for (int e = 0; e < 6; e++) {
        const double2 u = pld(q + (size_t)e * ag.na);
        const cx<double> v = mk<double>(u.x, u.y);
        if (sp == 0) p[e] = v;
        else p[6 + e] = v;
    }
}

// acc += H_{+mu}(x) p(x + mu) (FWD) or H_{-mu}(x) p(x - mu); s = x, sn = the neighbour, f = -1/2 (+1/2 across
// the anti-periodic T boundary)
template <int MU, bool FWD>
__device__ __forceinline__ void hop_into(const OpData &d, int V, int s, int sn, double f, const cx<double> p[12],
                                         cx<double> acc[12]) {
    cx<double> U[9], h[6], chi[6];
    if (FWD) {
        Store<WDIRAC_F64>::load_link(d.links, V, MU, s, U, d.rows);
        project<MU, -1>(p, h, f);
        su3_mul<false>(U, h, chi);
        reconstruct<MU, -1>(acc, chi);
    } else {
        Store<WDIRAC_F64>::load_link(d.links, V, MU, sn, U, d.rows);
        project<MU, +1>(p, h, f);
        su3_mul<true>(U, h, chi);
        reconstruct<MU, +1>(acc, chi);
    }
}

template <bool FWD>
__device__ __forceinline__ void hop_dir(int mu, const OpData &d, int V, int s, int sn, double f,
                                        const cx<double> p[12], cx<double> acc[12]) {
    switch (mu) {
    case 0: hop_into<0, FWD>(d, V, s, sn, f, p, acc); break;
    case 1: hop_into<1, FWD>(d, V, s, sn, f, p, acc); break;
    case 2: hop_into<2, FWD>(d, V, s, sn, f, p, acc); break;
    default: hop_into<3, FWD>(d, V, s, sn, f, p, acc); break;
    }
}

// A(x) p for the FP64 site-local term (packed or compact clover blocks)
__device__ __forceinline__ void site_term(const OpData &d, int V, int s, const cx<double> p[12], cx<double> y[12]) {
#pragma unroll
    for (int b = 0; b < 2; b++) {
        if (d.clover_compact) {
            double r[28];
            Store<WDIRAC_F64>::load_clover_compact(d.clover, V, b, s, r);
            clover_block_compact(d.diag, r, &p[6 * b], &y[6 * b]);
        } else {
            double dd[6];
            cx<double> uu[15];
            Store<WDIRAC_F64>::load_clover(d.clover, V, b, s, dd, uu);
            clover_block(dd, uu, &p[6 * b], &y[6 * b]);
        }
    }
}

// D_c = P^H D P, block by block: one work-group per coarse site a.  Block 0 gathers every term of D whose source
// and target sites lie in a (site-local term and the hops inside a, including those that wrap around a
// direction with one aggregate); block 1 + mu the forward hops from a's sites on its +mu face into a + mu
// (zero when one aggregate spans mu).
template <typename S>
__global__ __launch_bounds__(kAmgThreads) void k_coarse_build(const S *P, double2 *Dc, OpData d, Geom g,
                                                              AmgGeom ag, int apbc) {
    __shared__ double2 red[4 * 2 * kAmgChunk];
    const int a = blockIdx.x;
    const int N = ag.N, n2 = 2 * N;
    int ca[4];
    {
        int r = a;
        for (int mu = 3; mu >= 0; mu--) {
            ca[mu] = r % ag.nc[mu];
            r /= ag.nc[mu];
        }
    }
    for (int blk = 0; blk < 5; blk++) {
        const int mu = blk - 1;
        double2 *out = Dc + (size_t)(a * 5 + blk) * n2 * n2;
        if (blk > 0 && ag.nc[mu] == 1) {
            for (int e = threadIdx.x; e < n2 * n2; e += kAmgThreads) out[e] = make_double2(0.0, 0.0);
            continue;
        }
        int src = a;
        if (blk > 0) {
            int cb[4] = {ca[0], ca[1], ca[2], ca[3]};
            cb[mu] = (cb[mu] + 1) % ag.nc[mu];
            src = ((cb[0] * ag.nc[1] + cb[1]) * ag.nc[2] + cb[2]) * ag.nc[3] + cb[3];
        }
        for (int col = 0; col < n2; col++) {
            const int sp = col / N, l = col % N;
            for (int k0 = 0; k0 < N; k0 += kAmgChunk) {
                const int nk = min(kAmgChunk, N - k0);
                double2 acc[2 * kAmgChunk];
#pragma unroll
                for (int q = 0; q < 2 * kAmgChunk; q++) acc[q] = make_double2(0.0, 0.0);
                for (int j = threadIdx.x; j < ag.na; j += kAmgThreads) {
                    int c[4];
                    coords_of(ag, a, j, c);
                    const int s = site_index(g, c);
                    cx<double> y[12], p[12];
#pragma unroll
                    for (int e = 0; e < 12; e++) y[e] = mk<double>(0.0, 0.0);
                    bool any = false;
                    if (blk == 0) {
                        column_at(P, ag, src, l, sp, c, p);
                        site_term(d, g.V, s, p, y);
                        any = true;
                        for (int nu = 0; nu < 4; nu++) {
                            for (int dir = 0; dir < 2; dir++) {
                                int cn[4] = {c[0], c[1], c[2], c[3]};
                                const bool wraps = dir == 0 ? c[nu] == g.n[nu] - 1 : c[nu] == 0;
                                cn[nu] = dir == 0 ? (wraps ? 0 : c[nu] + 1) : (wraps ? g.n[nu] - 1 : c[nu] - 1);
                                int an, jn;
                                agg_of(ag, cn, an, jn);
                                if (an != a) continue;
                                column_at(P, ag, src, l, sp, cn, p);
                                const double f = (nu == 0 && apbc && wraps) ? 0.5 : -0.5;
                                const int sn = site_index(g, cn);
                                if (dir == 0) hop_dir<true>(nu, d, g.V, s, sn, f, p, y);
                                else hop_dir<false>(nu, d, g.V, s, sn, f, p, y);
                            }
                        }
                    } else if (c[mu] % ag.a[mu] == ag.a[mu] - 1) {
                        int cn[4] = {c[0], c[1], c[2], c[3]};
                        const bool wraps = c[mu] == g.n[mu] - 1;
                        cn[mu] = wraps ? 0 : c[mu] + 1;
                        column_at(P, ag, src, l, sp, cn, p);
                        const double f = (mu == 0 && apbc && wraps) ? 0.5 : -0.5;
                        hop_dir<true>(mu, d, g.V, s, site_index(g, cn), f, p, y);
                        any = true;
                    }
                    if (!any) continue;
#pragma unroll
                    for (int q = 0; q < kAmgChunk; q++) {
                        if (q >= nk) break;
                        const S *pk = P + pcol(ag, a, k0 + q) + j;
#pragma unroll
                        for (int e = 0; e < 6; e++) {
                            cj_acc(acc[2 * q], pld(pk + (size_t)e * ag.na), make_double2(y[e].r, y[e].i));
                            cj_acc(acc[2 * q + 1], pld(pk + (size_t)(6 + e) * ag.na),
                                   make_double2(y[6 + e].r, y[6 + e].i));
                        }
                    }
                }
                wg_sum<2 * kAmgChunk>(acc, red);
                if (threadIdx.x == 0) {
#pragma unroll
                    for (int q = 0; q < kAmgChunk; q++)
                        if (q < nk) {
                            out[(size_t)(k0 + q) * n2 + col] = acc[2 * q];
                            out[(size_t)(N + k0 + q) * n2 + col] = acc[2 * q + 1];
                        }
                }
            }
        }
    }
}

// c[a][s][k] = scale * sum over a's sites and s's components of conj(P) f; one work-group per (a, rhs).  The
// work-group's eight 32-lane groups take one test vector each (passes of eight), every lane a strided subset of
// the aggregate's sites (consecutive lanes read consecutive entries of P's component-major column); each group
// reduces over its lanes in a fixed order.
template <typename S>
__global__ __launch_bounds__(kAmgThreads) void k_restrict(const S *P, const double2 *f, double2 *c, Geom g,
                                                          AmgGeom ag, double scale) {
    const int a = blockIdx.x;
    const int kq = threadIdx.x >> 5, lane = threadIdx.x & 31;
    f += (size_t)blockIdx.y * 12 * g.V;
    c += (size_t)blockIdx.y * ag.Vc * 2 * ag.N;
    for (int k0 = 0; k0 < ag.N; k0 += kAmgThreads / 32) {
        const int k = k0 + kq;
        double2 acc0 = make_double2(0.0, 0.0), acc1 = make_double2(0.0, 0.0);
        if (k < ag.N)
            for (int j = lane; j < ag.na; j += 32) {
                int cc[4];
                coords_of(ag, a, j, cc);
                const int s = site_index(g, cc);
                const S *pk = P + pcol(ag, a, k) + j;
#pragma unroll
                for (int e = 0; e < 6; e++) {
                    cj_acc(acc0, pld(pk + (size_t)e * ag.na), f[(size_t)e * g.V + s]);
                    cj_acc(acc1, pld(pk + (size_t)(6 + e) * ag.na), f[(size_t)(6 + e) * g.V + s]);
                }
            }
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) {
            acc0.x += __shfl_xor(acc0.x, o, 32);
            acc0.y += __shfl_xor(acc0.y, o, 32);
            acc1.x += __shfl_xor(acc1.x, o, 32);
            acc1.y += __shfl_xor(acc1.y, o, 32);
        }
        if (lane == 0 && k < ag.N) {
            c[((size_t)a * 2 + 0) * ag.N + k] = make_double2(scale * acc0.x, scale * acc0.y);
            c[((size_t)a * 2 + 1) * ag.N + k] = make_double2(scale * acc1.x, scale * acc1.y);
        }
    }
}

// f(x) = sum_k P_k(x) c[a(x)][s][k] on the components of s; one thread per site, blockIdx.y = rhs
template <typename S>
__global__ __launch_bounds__(kAmgThreads) void k_prolong(const S *P, const double2 *c, double2 *f, Geom g,
                                                         AmgGeom ag) {
    const int s = blockIdx.x * kAmgThreads + threadIdx.x;
    if (s >= g.V) return;
    f += (size_t)blockIdx.y * 12 * g.V;
    c += (size_t)blockIdx.y * ag.Vc * 2 * ag.N;
    int cc[4], a, j;
    site_coords(g, s, cc);
    agg_of(ag, cc, a, j);
    double2 o[12];
#pragma unroll
    for (int e = 0; e < 12; e++) o[e] = make_double2(0.0, 0.0);
    const double2 *ca = c + (size_t)a * 2 * ag.N;
    for (int k = 0; k < ag.N; k++) {
        const S *pk = P + pcol(ag, a, k) + j;
        const double2 c0 = ca[k], c1 = ca[ag.N + k];
#pragma unroll
        for (int e = 0; e < 6; e++) {
            const double2 p0 = pld(pk + (size_t)e * ag.na), p1 = pld(pk + (size_t)(6 + e) * ag.na);
            o[e].x += p0.x * c0.x - p0.y * c0.y;
            o[e].y += p0.x * c0.y + p0.y * c0.x;
            o[6 + e].x += p1.x * c1.x - p1.y * c1.y;
            o[6 + e].y += p1.x * c1.y + p1.y * c1.x;
        }
    }
#pragma unroll
    for (int e = 0; e < 12; e++) f[(size_t)e * g.V + s] = o[e];
}

// y = D_c x on the coarse lattice: one wavefront per (coarse site, rhs), lane i = output unknown i < 2N.  Self
// and forward blocks are read by rows; the backward blocks are the neighbours' forward blocks read by columns,
// conjugated, with the G5 signs.
__global__ __launch_bounds__(64) void k_coarse_apply(const double2 *Dc, const double2 *x, double2 *y, AmgGeom ag) {
    __shared__ double2 xs[9][2 * kAmgMaxTv];
    const int a = blockIdx.x, i = threadIdx.x;
    const int N = ag.N, n2 = 2 * N;
    x += (size_t)blockIdx.y * ag.Vc * n2;
    y += (size_t)blockIdx.y * ag.Vc * n2;
    int ca[4];
    {
        int r = a;
        for (int mu = 3; mu >= 0; mu--) {
            ca[mu] = r % ag.nc[mu];
            r /= ag.nc[mu];
        }
    }
    int nb[9];
    nb[0] = a;
    for (int mu = 0; mu < 4; mu++) {
        int cf[4] = {ca[0], ca[1], ca[2], ca[3]}, cb[4] = {ca[0], ca[1], ca[2], ca[3]};
        cf[mu] = (ca[mu] + 1) % ag.nc[mu];
        cb[mu] = (ca[mu] + ag.nc[mu] - 1) % ag.nc[mu];
        nb[1 + mu] = ((cf[0] * ag.nc[1] + cf[1]) * ag.nc[2] + cf[2]) * ag.nc[3] + cf[3];
        nb[5 + mu] = ((cb[0] * ag.nc[1] + cb[1]) * ag.nc[2] + cb[2]) * ag.nc[3] + cb[3];
    }
    if (i < n2)
        for (int q = 0; q < 9; q++) xs[q][i] = x[(size_t)nb[q] * n2 + i];
    __syncthreads();
    if (i >= n2) return;
    double2 acc = make_double2(0.0, 0.0);
    for (int blk = 0; blk < 5; blk++) {
        const double2 *row = Dc + ((size_t)(a * 5 + blk) * n2 + i) * n2;
        for (int jj = 0; jj < n2; jj++) {
            const double2 m = row[jj], v = xs[blk][jj];
            acc.x += m.x * v.x - m.y * v.y;
            acc.y += m.x * v.y + m.y * v.x;
        }
    }
    const double gi = i < N ? 1.0 : -1.0;
    for (int mu = 0; mu < 4; mu++) {
        const double2 *F = Dc + (size_t)(nb[5 + mu] * 5 + 1 + mu) * n2 * n2;
        double2 t = make_double2(0.0, 0.0);
        for (int jj = 0; jj < n2; jj++) {
            const double2 m = F[(size_t)jj * n2 + i], v = xs[5 + mu][jj];
            const double gj = jj < N ? 1.0 : -1.0;
            // conj(m) * (gj v)
            t.x += gj * (m.x * v.x + m.y * v.y);
            t.y += gj * (m.x * v.y - m.y * v.x);
        }
        acc.x += gi * t.x;
        acc.y += gi * t.y;
    }
    y[(size_t)a * n2 + i] = acc;
}

// out = s a - b (native FP64 fields, N complex elements)
__global__ __launch_bounds__(256) void k_scaled_sub(const double2 *a, const double2 *b, double2 *out, double s,
                                                    long long N) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        const double2 u = a[e], v = b[e];
        out[e] = make_double2(s * u.x - v.x, s * u.y - v.y);
    }
}

int grid_of(long long n, int threads, int cap = 4096) {
    long long g = (n + threads - 1) / threads;
    return (int)std::max<long long>(1, std::min<long long>(g, cap));
}

// ---------------------------------------------------------------------------
// host side

int check_params(const dirac_op *op, const amg_params *p, AmgGeom &ag, SapGeom &sg) {
    if (!op || !p) return fail(WDIRAC_EINVAL, "null operator or AMG parameters");
    if (!op->links64) return fail(WDIRAC_EUNSUPPORTED, "the AMG needs the FP64 operator");
    if (p->ntv < 1 || p->ntv > kAmgMaxTv) return fail(WDIRAC_EINVAL, "ntv must be in [1, 32]");
    if (p->init_iters < 0 || p->setup_iters < 0) return fail(WDIRAC_EINVAL, "setup iteration counts must be >= 0");
    if (p->coarse_restart < 1 || p->coarse_restart > 1000) return fail(WDIRAC_EINVAL, "coarse_restart in [1, 1000]");
    if (p->coarse_maxit < 1) return fail(WDIRAC_EINVAL, "coarse_maxit must be >= 1");
    if (!(p->coarse_tol > 0.0) || !(p->coarse_tol < 1.0)) return fail(WDIRAC_EINVAL, "coarse_tol must be in (0, 1)");
    if (p->prec != WDIRAC_F64 && p->prec != WDIRAC_F32)
        return fail(WDIRAC_EINVAL, "AMG prec (storage of P) must be WDIRAC_F64 or WDIRAC_F32");
    long long na = 1, vc = 1;
    for (int mu = 0; mu < 4; mu++) {
        const int A = p->agg[mu], L = op->g.n[mu];
        if (A < 1 || L % A) return fail(WDIRAC_EINVAL, "aggregate extents must divide the lattice extents");
        ag.a[mu] = A;
        ag.nc[mu] = L / A;
        na *= A;
        vc *= L / A;
    }
    if (6 * na < p->ntv) return fail(WDIRAC_EINVAL, "ntv exceeds 6 x the sites of an aggregate");
    ag.na = (int)na;
    ag.Vc = (int)vc;
    ag.N = p->ntv;
    ag.cstr[3] = 1;
    ag.cstr[2] = ag.nc[3];
    ag.cstr[1] = ag.nc[3] * ag.nc[2];
    ag.cstr[0] = ag.nc[3] * ag.nc[2] * ag.nc[1];
    return sap_geometry(op, &p->smoother, sg);
}

long long coarse_len(const AmgGeom &ag) { return (long long)ag.Vc * 2 * ag.N; }  // complex entries

size_t partial_entries_amg() { return (size_t)kMdotChunks * ((kGS + kMdot - 1) / kMdot) * (kMdot + 1); }

// Hessenberg least-squares state of one GMRES cycle (Givens rotations)
struct Givens {
    int m = 0;
    std::vector<zc> H, sn, g;
    std::vector<double> cs;
    void reset(int m_, double beta) {
        m = m_;
        H.assign((size_t)(m + 1) * m, zc(0));
        sn.assign(m, zc(0));
        cs.assign(m, 0.0);
        g.assign(m + 1, zc(0));
        g[0] = beta;
    }
    zc &h(int i, int k) { return H[(size_t)k * (m + 1) + i]; }
    double add(int j, const std::vector<zc> &col) {
        for (int i = 0; i <= j + 1; i++) h(i, j) = col[i];
        for (int i = 0; i < j; i++) {
            const zc a = h(i, j), b = h(i + 1, j);
            h(i, j) = cs[i] * a + sn[i] * b;
            h(i + 1, j) = -std::conj(sn[i]) * a + cs[i] * b;
        }
        const zc a = h(j, j), b = h(j + 1, j);
        const double r = std::sqrt(std::norm(a) + std::norm(b));
        if (r == 0.0) {
            cs[j] = 1.0;
            sn[j] = 0.0;
        } else if (std::abs(a) == 0.0) {
            cs[j] = 0.0;
            sn[j] = std::conj(b) / std::abs(b);
        } else {
            cs[j] = std::abs(a) / r;
            sn[j] = (a / std::abs(a)) * std::conj(b) / r;
        }
        h(j, j) = cs[j] * a + sn[j] * b;
        h(j + 1, j) = 0.0;
        const zc gj = g[j];
        g[j] = cs[j] * gj;
        g[j + 1] = -std::conj(sn[j]) * gj;
        return std::abs(g[j + 1]);
    }
    std::vector<zc> solve(int n) {
        std::vector<zc> y(n);
        for (int i = n - 1; i >= 0; i--) {
            zc s = g[i];
            for (int k = i + 1; k < n; k++) s -= h(i, k) * y[k];
            y[i] = s / h(i, i);
        }
        return y;
    }
};

int fetch_scalars(const dirac_amg *A, const double2 *src, int n, std::vector<zc> &out, hipStream_t st) {
    if ((size_t)n > A->pinned_n) return fail(WDIRAC_EINVAL, "internal: AMG staging buffer too small");
    AMG_TRY(hipMemcpyAsync(A->pinned, src, n * sizeof(double2), hipMemcpyDeviceToHost, st));
    AMG_TRY(hipStreamSynchronize(st));
    out.resize(n);
    for (int i = 0; i < n; i++) out[i] = zc(A->pinned[i].x, A->pinned[i].y);
    return WDIRAC_OK;
}

hipError_t coarse_apply_launch(const dirac_amg *A, double2 *y, const double2 *x, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_coarse_apply, dim3(A->ag.Vc, nrhs), dim3(64), 0, st, A->Dc, x, y, A->ag);
    return hipGetLastError();
}

// x = D_c^{-1} b by GMRES(coarse_restart) from x = 0 to |b - D_c x| <= coarse_tol |b| (Givens estimate), or
// coarse_maxit applications of D_c.  x must not alias b or the workspace.
int coarse_gmres(const dirac_amg *A, double2 *x, const double2 *b, long long *iters, hipStream_t st) {
    dirac_amg *M = const_cast<dirac_amg *>(A);
    const long long n = coarse_len(A->ag);
    const int m = A->p.coarse_restart;
    const size_t vb = a256((size_t)n * sizeof(double2));
    auto vec = [&](int i) { return reinterpret_cast<double2 *>(reinterpret_cast<char *>(A->cb) + vb * i); };
    std::vector<const void *> vl(m + 1);
    for (int i = 0; i <= m; i++) vl[i] = vec(i);
    double2 *hcol = A->scal, *nrm = A->scal + m + 2;
    AMG_TRY(hipMemsetAsync(x, 0, n * sizeof(double2), st));
    // |b|
    AMG_TRY(mdot_all<double2>(vl.data(), 0, b, n, A->partial, nrm, st));
    std::vector<zc> got;
    int rc = fetch_scalars(A, nrm, 1, got, st);
    if (rc) return rc;
    const double bnorm = std::sqrt(std::max(got[0].real(), 0.0));
    long long applies = 0;
    if (!(bnorm > 0.0) || !std::isfinite(bnorm)) {
        if (iters) *iters = 0;
        return std::isfinite(bnorm) ? WDIRAC_OK : fail(WDIRAC_EINVAL, "coarse right-hand side not finite");
    }
    const double target = A->p.coarse_tol * bnorm;
    double beta = bnorm;
    AMG_TRY((scale<double2, double2>(b, vec(0), nullptr, false, 1.0 / beta, n, st)));
    Givens gv;
    bool done = false;
    while (!done) {
        gv.reset(m, beta);
        int ncols = 0;
        for (int j = 0; j < m; j++) {
            AMG_TRY(coarse_apply_launch(A, vec(j + 1), vec(j), 1, st));
            applies++;
            AMG_TRY(mdot_all<double2>(vl.data(), j + 1, vec(j + 1), n, A->partial, hcol, st));
            AMG_TRY(axpy_multi<double2>(vl.data(), j + 1, hcol, nullptr, vec(j + 1), n, A->partial, hcol + j + 1,
                                        st));
            rc = fetch_scalars(A, hcol, j + 2, got, st);
            if (rc) return rc;
            const double hn = std::sqrt(std::max(got[j + 1].real(), 0.0));
            got[j + 1] = hn;
            const double res = gv.add(j, got);
            ncols = j + 1;
            if (!std::isfinite(res)) return fail(WDIRAC_EINVAL, "coarse GMRES met a NaN or Inf");
            if (res <= target || applies >= A->p.coarse_maxit || hn <= 1e-300) {
                done = res <= target || applies >= A->p.coarse_maxit;
                break;
            }
            AMG_TRY((scale<double2, double2>(vec(j + 1), vec(j + 1), nullptr, false, 1.0 / hn, n, st)));
        }
        const std::vector<zc> y = gv.solve(ncols);
        std::vector<double2> coef(ncols);
        for (int i = 0; i < ncols; i++) coef[i] = make_double2(y[i].real(), y[i].imag());
        AMG_TRY(update<double2>(vl.data(), ncols, coef.data(), x, n, st));
        if (done) break;
        // restart: r = b - D_c x into vec(0)
        AMG_TRY(coarse_apply_launch(A, vec(1), x, 1, st));
        applies++;
        AMG_TRY(residual(b, vec(1), vec(0), n, A->partial, nrm, st));
        rc = fetch_scalars(A, nrm, 1, got, st);
        if (rc) return rc;
        beta = std::sqrt(std::max(got[0].real(), 0.0));
        if (beta <= target || applies >= A->p.coarse_maxit) break;
        AMG_TRY((scale<double2, double2>(vec(0), vec(0), nullptr, false, 1.0 / beta, n, st)));
    }
    M->coarse_iters += applies;
    M->coarse_solves++;
    if (iters) *iters = applies;
    return WDIRAC_OK;
}

bool p32(const dirac_amg *A) { return A->p.prec == WDIRAC_F32; }
const float2 *P32(const dirac_amg *A) { return static_cast<const float2 *>(A->P); }
const double2 *P64(const dirac_amg *A) { return static_cast<const double2 *>(A->P); }

hipError_t restrict_launch(const dirac_amg *A, double2 *c, const double2 *f, int nrhs, double scale_, hipStream_t st) {
    const dim3 grid(A->ag.Vc, nrhs), blk(kAmgThreads);
    if (p32(A)) hipLaunchKernelGGL(k_restrict<float2>, grid, blk, 0, st, P32(A), f, c, A->op->g, A->ag, scale_);
    else hipLaunchKernelGGL(k_restrict<double2>, grid, blk, 0, st, P64(A), f, c, A->op->g, A->ag, scale_);
    return hipGetLastError();
}

hipError_t prolong_launch(const dirac_amg *A, double2 *f, const double2 *c, int nrhs, hipStream_t st) {
    const dim3 grid((A->op->g.V + kAmgThreads - 1) / kAmgThreads, nrhs), blk(kAmgThreads);
    if (p32(A)) hipLaunchKernelGGL(k_prolong<float2>, grid, blk, 0, st, P32(A), c, f, A->op->g, A->ag);
    else hipLaunchKernelGGL(k_prolong<double2>, grid, blk, 0, st, P64(A), c, f, A->op->g, A->ag);
    return hipGetLastError();
}

// native FP64 fields <-> P (dir 0: fields into P, dir 1: P into fields)
hipError_t gather_launch(const dirac_amg *A, double2 *fields, int dir, hipStream_t st) {
    const Geom &g = A->op->g;
    const dim3 grid((g.V + kAmgThreads - 1) / kAmgThreads, A->ag.N), blk(kAmgThreads);
    if (p32(A))
        hipLaunchKernelGGL(k_gather<float2>, grid, blk, 0, st, fields, static_cast<float2 *>(A->P), g, A->ag, dir);
    else
        hipLaunchKernelGGL(k_gather<double2>, grid, blk, 0, st, fields, static_cast<double2 *>(A->P), g, A->ag, dir);
    return hipGetLastError();
}

// P and D_c from the current test vectors
int build(dirac_amg *A, hipStream_t st) {
    const Geom &g = A->op->g;
    AMG_TRY(hipMemsetAsync(A->flag, 0, sizeof(int), st));
    AMG_TRY(gather_launch(A, A->test, 0, st));
    if (p32(A))
        hipLaunchKernelGGL(k_block_gs<float2>, dim3(A->ag.Vc, 2), dim3(kAmgThreads), 0, st,
                           static_cast<float2 *>(A->P), A->ag, A->flag);
    else
        hipLaunchKernelGGL(k_block_gs<double2>, dim3(A->ag.Vc, 2), dim3(kAmgThreads), 0, st,
                           static_cast<double2 *>(A->P), A->ag, A->flag);
    AMG_TRY(hipGetLastError());
    int flag = 0;
    AMG_TRY(hipMemcpyAsync(&flag, A->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    AMG_TRY(hipStreamSynchronize(st));
    if (flag) return fail(WDIRAC_EINVAL, "test vectors are linearly dependent on some aggregate");
    const int apbc = (A->op->flags & WDIRAC_ANTIPERIODIC_T) ? 1 : 0;
    if (p32(A))
        hipLaunchKernelGGL(k_coarse_build<float2>, dim3(A->ag.Vc), dim3(kAmgThreads), 0, st, P32(A), A->Dc,
                           A->op->data(WDIRAC_F64), g, A->ag, apbc);
    else
        hipLaunchKernelGGL(k_coarse_build<double2>, dim3(A->ag.Vc), dim3(kAmgThreads), 0, st, P64(A), A->Dc,
                           A->op->data(WDIRAC_F64), g, A->ag, apbc);
    AMG_TRY(hipGetLastError());
    return WDIRAC_OK;
}

// v <- v / |v| (one native FP64 field)
int normalise(dirac_amg *A, double2 *v, hipStream_t st) {
    const long long n = 12LL * A->op->g.V;
    const void *vl[1] = {v};
    AMG_TRY(mdot_all<double2>(vl, 0, v, n, A->partial, A->scal, st));
    AMG_TRY((scale<double2, double2>(v, v, A->scal, true, 1.0, n, st)));
    return WDIRAC_OK;
}

int setup(dirac_amg *A, hipStream_t st) {
    const Geom &g = A->op->g;
    const size_t fb = (size_t)12 * g.V;  // complex entries per field
    for (int it = 0; it < A->p.init_iters; it++)
        for (int k = 0; k < A->ag.N; k++) {
            AMG_TRY(sap_apply(A->op, A->p.smoother, A->sg, A->f1, A->test + k * fb, 1, A->fsap, 1.0, st));
            AMG_TRY(hipMemcpyAsync(A->test + k * fb, A->f1, fb * sizeof(double2), hipMemcpyDeviceToDevice, st));
            int rc = normalise(A, A->test + k * fb, st);
            if (rc) return rc;
        }
    int rc = build(A, st);
    if (rc) return rc;
    if (log_level() >= 2)
        std::fprintf(stderr, "[wdirac] amg setup: %d smoother passes over %d test vectors, P and D_c built\n",
                     A->p.init_iters, A->ag.N);
    for (int it = 0; it < A->p.setup_iters; it++) {
        // every test vector through the current two-level method, then one rebuild
        for (int k = 0; k < A->ag.N; k++) {
            rc = amg_precond_one(A, A->f3, A->test + k * fb, 1.0, st);
            if (rc) return rc;
            AMG_TRY(hipMemcpyAsync(A->test + k * fb, A->f3, fb * sizeof(double2), hipMemcpyDeviceToDevice, st));
            rc = normalise(A, A->test + k * fb, st);
            if (rc) return rc;
        }
        rc = build(A, st);
        if (rc) return rc;
        if (log_level() >= 2)
            std::fprintf(stderr, "[wdirac] amg setup: two-level pass %d done (%lld coarse solves, %lld D_c applies)\n",
                         it + 1, A->coarse_solves, A->coarse_iters);
    }
    return WDIRAC_OK;
}

int check_amg(const dirac_amg *A) {
    if (!A || !A->op || !A->P) return fail(WDIRAC_EINVAL, "null AMG handle");
    return WDIRAC_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
    return x < y + nb && y < x + na;
}

}  // namespace

int amg_precond_one(const dirac_amg *A, double2 *x, const double2 *r, double rscale, hipStream_t st) {
    const dirac_op *op = A->op;
    const long long nf = 12LL * op->g.V;
    // coarse-grid correction e = P D_c^{-1} P^H (rscale r), written to x
    AMG_TRY(restrict_launch(A, A->crhs, r, 1, rscale, st));
    int rc = coarse_gmres(A, A->csol, A->crhs, nullptr, st);
    if (rc) return rc;
    AMG_TRY(prolong_launch(A, x, A->csol, 1, st));
    // post-smoothing: x += SAP(rscale r - D e)
    const dirac_batch b1 = {A->f1, x, 1};
    AMG_TRY(dslash_launch_batches(&b1, 1, WDIRAC_F64, false, op->data(WDIRAC_F64), op->g,
                                  (op->flags & WDIRAC_ANTIPERIODIC_T) ? 1 : 0, false, st));
    hipLaunchKernelGGL(k_scaled_sub, dim3(grid_of(nf, 256)), dim3(256), 0, st, r, A->f1, A->f1, rscale, nf);
    AMG_TRY(hipGetLastError());
    AMG_TRY(sap_apply(op, A->p.smoother, A->sg, A->f2, A->f1, 1, A->fsap, 1.0, st));
    const void *zl[1] = {A->f2};
    const double2 one = make_double2(1.0, 0.0);
    AMG_TRY(update<double2>(zl, 1, &one, x, nf, st));
    return WDIRAC_OK;
}

}  // namespace wd

using namespace wd;

extern "C" {

int dirac_amg_create(dirac_amg **out, const dirac_op *op, const amg_params *p, const double *testvecs, void *stream) {
    if (!out) return fail(WDIRAC_EINVAL, "null output handle");
    *out = nullptr;
    AmgGeom ag{};
    SapGeom sg{};
    int rc = check_params(op, p, ag, sg);
    if (rc) return rc;
    if (!testvecs) return fail(WDIRAC_EINVAL, "null test vectors");
    if (reinterpret_cast<uintptr_t>(testvecs) & 15) return fail(WDIRAC_EINVAL, "test vectors must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    const Geom &g = op->g;
    const size_t field = a256((size_t)12 * g.V * sizeof(double2));
    const size_t cvec = a256((size_t)coarse_len(ag) * sizeof(double2));
    const size_t nT = a256((size_t)ag.N * field);
    const size_t nP = a256((size_t)ag.N * 12 * g.V * (p->prec == WDIRAC_F32 ? sizeof(float2) : sizeof(double2)));
    const size_t nDc = a256((size_t)ag.Vc * 5 * 4 * ag.N * ag.N * sizeof(double2));
    const size_t nsap = a256(sap_workspace(op, &p->smoother, 1));
    const size_t nscal = a256((p->coarse_restart + 4) * sizeof(double2));
    const size_t npart = a256(partial_entries_amg() * sizeof(double2));
    const size_t total = nT /*test*/ + nP /*P*/ + nDc + (size_t)(p->coarse_restart + 1) * cvec + 2 * cvec +
                         3 * field + nsap + nscal + npart + 256;
    auto *A = new dirac_amg;
    A->op = op;
    A->device = op->device;
    A->p = *p;
    A->ag = ag;
    A->sg = sg;
    if (hipSetDevice(op->device) != hipSuccess || hipMalloc(&A->mem, total) != hipSuccess) {
        (void)hipGetLastError();
        delete A;
        return fail(WDIRAC_ENOMEM, "AMG device allocation failed");
    }
    char *q = static_cast<char *>(A->mem);
    auto take = [&](size_t n) {
        char *r = q;
        q += n;
        return r;
    };
    A->test = reinterpret_cast<double2 *>(take(nT));
    A->P = take(nP);
    A->Dc = reinterpret_cast<double2 *>(take(nDc));
    A->cb = reinterpret_cast<double2 *>(take((size_t)(p->coarse_restart + 1) * cvec));
    A->crhs = reinterpret_cast<double2 *>(take(cvec));
    A->csol = reinterpret_cast<double2 *>(take(cvec));
    A->f1 = reinterpret_cast<double2 *>(take(field));
    A->f2 = reinterpret_cast<double2 *>(take(field));
    A->f3 = reinterpret_cast<double2 *>(take(field));
    A->fsap = nsap ? reinterpret_cast<double2 *>(take(nsap)) : nullptr;
    A->scal = reinterpret_cast<double2 *>(take(nscal));
    A->partial = reinterpret_cast<double2 *>(take(npart));
    A->flag = reinterpret_cast<int *>(take(256));
    A->pinned_n = (size_t)p->coarse_restart + 4;
    if (hipHostMalloc((void **)&A->pinned, A->pinned_n * sizeof(double2), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(A->mem);
        delete A;
        return fail(WDIRAC_ENOMEM, "AMG pinned staging allocation failed");
    }
    auto cleanup = [&](int code) {
        (void)hipStreamSynchronize(st);
        (void)hipHostFree(A->pinned);
        (void)hipFree(A->mem);
        delete A;
        return code;
    };
    const size_t fb = (size_t)12 * g.V * sizeof(double2);
    for (int k = 0; k < ag.N; k++) {
        if (hipMemcpyAsync(reinterpret_cast<char *>(A->test) + k * fb, reinterpret_cast<const char *>(testvecs) + k * fb,
                           fb, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return cleanup(fail(WDIRAC_EHIP, "copy of the test vectors failed"));
    }
    rc = setup(A, st);
    if (rc) return cleanup(rc);
    if (hipStreamSynchronize(st) != hipSuccess) return cleanup(fail(WDIRAC_EHIP, "AMG setup failed"));
    *out = A;
    return WDIRAC_OK;
}

int dirac_amg_destroy(dirac_amg *amg) {
    if (!amg) return WDIRAC_OK;
    (void)hipSetDevice(amg->device);
    (void)hipDeviceSynchronize();
    (void)hipHostFree(amg->pinned);
    (void)hipFree(amg->mem);
    delete amg;
    return WDIRAC_OK;
}

int dirac_amg_sizes(const dirac_amg *amg, int coarse_dims[4], int *unknowns_per_site, long long *coarse_stats) {
    int rc = check_amg(amg);
    if (rc) return rc;
    if (coarse_dims)
        for (int mu = 0; mu < 4; mu++) coarse_dims[mu] = amg->ag.nc[mu];
    if (unknowns_per_site) *unknowns_per_site = 2 * amg->ag.N;
    if (coarse_stats) {
        coarse_stats[0] = amg->coarse_solves;
        coarse_stats[1] = amg->coarse_iters;
    }
    return WDIRAC_OK;
}

int dirac_amg_restrict(const dirac_amg *amg, double *coarse, const double *fine, int nrhs, void *stream) {
    int rc = check_amg(amg);
    if (rc) return rc;
    if (!coarse || !fine || nrhs < 1) return fail(WDIRAC_EINVAL, "null field or nrhs < 1");
    hipError_t e = restrict_launch(amg, reinterpret_cast<double2 *>(coarse), reinterpret_cast<const double2 *>(fine),
                                   nrhs, 1.0, (hipStream_t)stream);
    if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("restriction: ") + hipGetErrorString(e));
    return WDIRAC_OK;
}

int dirac_amg_prolong(const dirac_amg *amg, double *fine, const double *coarse, int nrhs, void *stream) {
    int rc = check_amg(amg);
    if (rc) return rc;
    if (!coarse || !fine || nrhs < 1) return fail(WDIRAC_EINVAL, "null field or nrhs < 1");
    hipError_t e = prolong_launch(amg, reinterpret_cast<double2 *>(fine), reinterpret_cast<const double2 *>(coarse),
                                  nrhs, (hipStream_t)stream);
    if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("prolongation: ") + hipGetErrorString(e));
    return WDIRAC_OK;
}

int dirac_amg_coarse_apply(const dirac_amg *amg, double *out, const double *in, int nrhs, void *stream) {
    int rc = check_amg(amg);
    if (rc) return rc;
    if (!out || !in || nrhs < 1) return fail(WDIRAC_EINVAL, "null coarse vector or nrhs < 1");
    const size_t n = (size_t)coarse_len(amg->ag) * nrhs * sizeof(double2);
    if (overlaps(out, n, in, n)) return fail(WDIRAC_EINVAL, "out overlaps in");
    hipError_t e = coarse_apply_launch(amg, reinterpret_cast<double2 *>(out), reinterpret_cast<const double2 *>(in),
                                       nrhs, (hipStream_t)stream);
    if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("coarse apply: ") + hipGetErrorString(e));
    return WDIRAC_OK;
}

int dirac_amg_coarse_solve(const dirac_amg *amg, double *x, const double *b, long long *iters, void *stream) {
    int rc = check_amg(amg);
    if (rc) return rc;
    if (!x || !b) return fail(WDIRAC_EINVAL, "null coarse vector");
    const size_t n = (size_t)coarse_len(amg->ag) * sizeof(double2);
    if (overlaps(x, n, b, n)) return fail(WDIRAC_EINVAL, "x overlaps b");
    return coarse_gmres(amg, reinterpret_cast<double2 *>(x), reinterpret_cast<const double2 *>(b), iters,
                        (hipStream_t)stream);
}

int dirac_amg_precond(const dirac_amg *amg, double *z, const double *r, int nrhs, void *stream) {
    int rc = check_amg(amg);
    if (rc) return rc;
    if (!z || !r || nrhs < 1) return fail(WDIRAC_EINVAL, "null field or nrhs < 1");
    const size_t fb = (size_t)12 * amg->op->g.V * sizeof(double2);
    if (overlaps(z, fb * nrhs, r, fb * nrhs)) return fail(WDIRAC_EINVAL, "z overlaps r");
    for (int k = 0; k < nrhs; k++) {
        rc = amg_precond_one(amg, reinterpret_cast<double2 *>(reinterpret_cast<char *>(z) + k * fb),
                             reinterpret_cast<const double2 *>(reinterpret_cast<const char *>(r) + k * fb), 1.0,
                             (hipStream_t)stream);
        if (rc) return rc;
    }
    return WDIRAC_OK;
}

int dirac_amg_export(const dirac_amg *amg, int what, double *out, void *stream) {
    int rc = check_amg(amg);
    if (rc) return rc;
    if (!out) return fail(WDIRAC_EINVAL, "null output");
    hipStream_t st = (hipStream_t)stream;
    const Geom &g = amg->op->g;
    const size_t fb = (size_t)12 * g.V * sizeof(double2);
    hipError_t e = hipSuccess;
    if (what == WDIRAC_AMG_TEST_VECTORS) {
        e = hipMemcpyAsync(out, amg->test, fb * amg->ag.N, hipMemcpyDeviceToDevice, st);
    } else if (what == WDIRAC_AMG_INTERPOLATION) {
        e = gather_launch(amg, reinterpret_cast<double2 *>(out), 1, st);
    } else if (what == WDIRAC_AMG_COARSE_OPERATOR) {
        e = hipMemcpyAsync(out, amg->Dc, (size_t)amg->ag.Vc * 5 * 4 * amg->ag.N * amg->ag.N * sizeof(double2),
                           hipMemcpyDeviceToDevice, st);
    } else {
        return fail(WDIRAC_EINVAL, "unknown export");
    }
    if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("AMG export: ") + hipGetErrorString(e));
    return WDIRAC_OK;
}

}  // extern "C"
