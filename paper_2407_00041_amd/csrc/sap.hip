// Schwarz alternating procedure (SAP) on non-overlapping lattice blocks: the
// domain-decomposition smoother that Sec. 1.3 names (additive and red-black
// multiplicative Schwarz) used as the flexible preconditioner M_j^{-1} of
// FGMRES (Algorithm 2).
//
// A block of b_T x b_Z x b_Y x b_X sites (at most 256) is one work-group, one
// lane per site.  Its block operator D_B is D with the hops that leave the
// block dropped; the local solve is mr_iters minimal-residual steps
// (e = 0, rho = r_B; q = D_B rho, alpha = <q, rho>/<q, q>, e += alpha rho,
// rho -= alpha q), run entirely on chip: the block's rho lives in LDS so
// every lane reads its in-block neighbours there, the two dot products are
// reduced across the work-group through LDS in a fixed order (deterministic),
// and at FP32 the block's forward links are staged in LDS and its compact
// clover blocks held in registers, so the MR steps read no memory at all.
// The residual r_B = (b - D x)_B that starts a block solve is computed by the
// same kernel from the full operator (neighbour values of x from the other
// colour's blocks in memory).  One launch per colour (red-black) or one for all
// blocks (additive) per cycle; x is FP64 in memory, the block arithmetic is
// FP64 or FP32 (the operator data of that precision), dot products are
// accumulated in FP64.
//
// Blocks of one colour are enumerated in pairs along a direction with an
// even block count (the last such of T, Z, Y, X): the i-th block of colour c
// takes the other block coordinates from i and the paired coordinate so that
// the coordinate sum has parity c.
#include <algorithm>

#include "sap.h"
#include "stencil.h"

namespace wd {

namespace {

constexpr int kSapMaxBlock = 256;

template <int P> using TOf = typename Store<P>::T;

// keeps the compiler from hoisting one hop's loads above the previous hop's arithmetic (register pressure)
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// FP64 field value at site s, converted to the arithmetic type
template <typename T> __device__ __forceinline__ void load_x(const double2 *f, int V, int s, cx<T> v[12]) {
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const double2 a = f[(size_t)k * V + s];
        v[k] = {(T)a.x, (T)a.y};
    }
}

// lexicographic block coordinates of the i-th block of a pass
__device__ __forceinline__ void block_coords(const SapGeom &sg, int colour, int i, int bc[4]) {
    int ext[4] = {sg.nb[0], sg.nb[1], sg.nb[2], sg.nb[3]};
    const int m = colour >= 0 ? sg.pair_dir : -1;
    if (m >= 0) ext[m] >>= 1;
    int r = i;
    bc[3] = r % ext[3]; r /= ext[3];
    bc[2] = r % ext[2]; r /= ext[2];
    bc[1] = r % ext[1];
    bc[0] = r / ext[1];
    if (m >= 0) {
        int other = 0;
#pragma unroll
        for (int mu = 0; mu < 4; mu++)
            if (mu != m) other += bc[mu];
        bc[m] = 2 * bc[m] + ((colour + other) & 1);
    }
}

// site-local term A(x) psi: clover blocks kept in registers (FP32 compact) or loaded at each use
template <int P, bool REGC> struct SiteTerm {
    using T = TOf<P>;
    T cr[2][REGC ? 28 : 1];
    __device__ __forceinline__ void init(const OpData &d, int V, int s) {
        if constexpr (REGC) {
            Store<P>::load_clover_compact(d.clover, V, 0, s, cr[0]);
            Store<P>::load_clover_compact(d.clover, V, 1, s, cr[1]);
        }
    }
    __device__ __forceinline__ void apply(const OpData &d, int V, int s, const cx<T> in[12], cx<T> out[12]) const {
#pragma unroll
        for (int b = 0; b < 2; b++) {
            if constexpr (REGC) {
                clover_block_compact((T)d.diag, cr[b], &in[6 * b], &out[6 * b]);
            } else if (d.clover_compact) {
                T r[28];
                Store<P>::load_clover_compact(d.clover, V, b, s, r);
                clover_block_compact((T)d.diag, r, &in[6 * b], &out[6 * b]);
            } else {
                T dd[6];
                cx<T> uu[15];
                Store<P>::load_clover(d.clover, V, b, s, dd, uu);
                clover_block(dd, uu, &in[6 * b], &out[6 * b]);
            }
        }
    }
};

// deterministic sum over the work-group of three doubles (every lane gets the totals)
__device__ __forceinline__ void group_sum3(double v[3], double (*red)[3]) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < 3; k++) v[k] += __shfl_xor(v[k], o, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < 3; k++) red[w][k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; k++) {
        double t = 0.0;
        for (int q = 0; q < nw; q++) t += red[q][k];
        v[k] = t;
    }
}

// One Schwarz pass: every block of the pass (colour c, or all blocks for c < 0) computes its residual
// r_B = (b - D x)_B, solves D_B e = r_B approximately by nmr MR steps and writes x_out = x_in + e on its
// sites.  xzero: x_in is zero everywhere (r = b); own_zero: x_in is zero on the pass's blocks (their
// in-block terms are skipped, halo values come from x_in).  LDSL: links staged in LDS (FP32, two rows);
// REGC: compact clover blocks in registers (FP32).
template <int P, bool LDSL, bool REGC>
__global__ __launch_bounds__(kSapMaxBlock) void sap_pass_kernel(const double2 *__restrict__ b, const double2 *xin,
                                                                double2 *xout, size_t rhs_stride, OpData d, Geom g,
                                                                SapGeom sg, int colour, int xzero, int own_zero,
                                                                int nmr, int apbc, double bscale) {
    using T = TOf<P>;
    constexpr int SF = -1, SB = +1;  // forward / backward projector signs of D
    __shared__ cx<T> rho_lds[12][kSapMaxBlock];
    __shared__ f4v link_lds[LDSL ? 12 : 1][LDSL ? kSapMaxBlock : 1];
    __shared__ double red[kSapMaxBlock / 64][3];
    // FP64: the correction e is kept in the lane's LDS slot too (registers hold the hop in flight)
    constexpr bool ELDS = P == WDIRAC_F64;
    __shared__ cx<T> e_lds[ELDS ? 12 : 1][ELDS ? kSapMaxBlock : 1];

    const int V = g.V;
    const int l = threadIdx.x;
    const bool active = l < sg.bvol;
    b += blockIdx.y * rhs_stride;
    if (xin) xin += blockIdx.y * rhs_stride;
    xout += blockIdx.y * rhs_stride;

    int bc[4];
    block_coords(sg, colour, blockIdx.x, bc);
    int lc[4], s = 0;
    {
        int r = active ? l : 0;
        lc[3] = r % sg.b[3]; r /= sg.b[3];
        lc[2] = r % sg.b[2]; r /= sg.b[2];
        lc[1] = r % sg.b[1];
        lc[0] = r / sg.b[1];
#pragma unroll
        for (int mu = 0; mu < 4; mu++) s += (bc[mu] * sg.b[mu] + lc[mu]) * g.stride[mu];
    }
    // in-block neighbours (local index, or -1 when the hop leaves the block) and T-boundary crossings
    int nf[4], nbk[4];
    bool wf = false, wb = false;
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        const int st = sg.lstr[mu], B = sg.b[mu];
        nf[mu] = lc[mu] + 1 < B ? l + st : (sg.span[mu] ? l - (B - 1) * st : -1);
        nbk[mu] = lc[mu] > 0 ? l - st : (sg.span[mu] ? l + (B - 1) * st : -1);
    }
    if (sg.span[0]) {
        wf = lc[0] == sg.b[0] - 1;
        wb = lc[0] == 0;
    }

    SiteTerm<P, REGC> A;
    if (active) A.init(d, V, s);
    if constexpr (LDSL) {
        if (active) {
            const f4v *q = static_cast<const f4v *>(d.links);
#pragma unroll
            for (int e = 0; e < 12; e++) link_lds[e][l] = q[op_idx(e, 12, s)];
        }
    }

    // ---- residual r = b - D x at the own site, straight into the lane's LDS slot
    {
        cx<T> acc[12];
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = mk<T>(0, 0);
        if (active && !xzero) {
            if (!own_zero) {
                cx<T> xs[12];
                load_x<T>(xin, V, s, xs);
                A.apply(d, V, s, xs, acc);
            }
            // global neighbours of s
            int c[4] = {bc[0] * sg.b[0] + lc[0], bc[1] * sg.b[1] + lc[1], bc[2] * sg.b[2] + lc[2],
                        bc[3] * sg.b[3] + lc[3]};
#define WD_SAP_RES_HOP(MU)                                                                                        \
            {                                                                                                     \
                const int st = g.stride[MU], L = g.n[MU];                                                         \
                if (!own_zero || nf[MU] < 0) {                                                                    \
                    const int sn = c[MU] == L - 1 ? s - (L - 1) * st : s + st;                                   \
                    const T f = (MU == 0 && apbc && c[0] == L - 1) ? T(0.5) : T(-0.5);                            \
                    cx<T> U[9], p[12], h[6], chi[6];                                                              \
                    Store<P>::load_link(d.links, V, MU, s, U, d.rows);                                            \
                    load_x<T>(xin, V, sn, p);                                                                     \
                    project<MU, SF>(p, h, f);                                                                     \
                    su3_mul<false>(U, h, chi);                                                                    \
                    reconstruct<MU, SF>(acc, chi);                                                                \
                }                                                                                                 \
                if (!own_zero || nbk[MU] < 0) {                                                                   \
                    const int sn = c[MU] == 0 ? s + (L - 1) * st : s - st;                                       \
                    const T f = (MU == 0 && apbc && c[0] == 0) ? T(0.5) : T(-0.5);                                \
                    cx<T> U[9], p[12], h[6], chi[6];                                                              \
                    Store<P>::load_link(d.links, V, MU, sn, U, d.rows);                                           \
                    load_x<T>(xin, V, sn, p);                                                                     \
                    project<MU, SB>(p, h, f);                                                                     \
                    su3_mul<true>(U, h, chi);                                                                     \
                    reconstruct<MU, SB>(acc, chi);                                                                \
                }                                                                                                 \
            }
            sched_fence();
            WD_SAP_RES_HOP(0)
            sched_fence();
            WD_SAP_RES_HOP(1)
            sched_fence();
            WD_SAP_RES_HOP(2)
            sched_fence();
            WD_SAP_RES_HOP(3)
            sched_fence();
#undef WD_SAP_RES_HOP
        }
#pragma unroll
        for (int k = 0; k < 12; k++) {
            cx<T> r = mk<T>(0, 0);
            if (active) {
                const double2 a = b[(size_t)k * V + s];
                r = mk<T>((T)(bscale * a.x), (T)(bscale * a.y)) - acc[k];
            }
            rho_lds[k][l] = r;
        }
    }

    // ---- minimal-residual steps on D_B e = rho; rho lives only in LDS (each lane updates its own slot once
    // every lane has finished reading its neighbours, i.e. after the reduction's barrier)
    cx<T> e[ELDS ? 1 : 12];
#pragma unroll
    for (int k = 0; k < 12; k++) {
        if constexpr (ELDS) e_lds[k][l] = mk<T>(0, 0);
        else e[k] = mk<T>(0, 0);
    }
    const T fh = T(-0.5);
    for (int it = 0; it < nmr; it++) {
        __syncthreads();
        cx<T> q[12];
#pragma unroll
        for (int k = 0; k < 12; k++) q[k] = mk<T>(0, 0);
        if (active) {
            {
                cx<T> own[12];
#pragma unroll
                for (int k = 0; k < 12; k++) own[k] = rho_lds[k][l];
                A.apply(d, V, s, own, q);
            }
#define WD_SAP_BLK_HOP(MU)                                                                                        \
            if (nf[MU] >= 0) {                                                                                    \
                const int n = nf[MU];                                                                             \
                const T f = (MU == 0 && apbc && wf) ? T(0.5) : fh;                                                \
                cx<T> U[9], p[12], h[6], chi[6];                                                                  \
                if constexpr (LDSL) {                                                                             \
                    _Pragma("unroll") for (int e3 = 0; e3 < 3; e3++) {                                            \
                        const f4v a = link_lds[3 * MU + e3][l];                                                   \
                        U[2 * e3] = {a.x, a.y};                                                                   \
                        U[2 * e3 + 1] = {a.z, a.w};                                                               \
                    }                                                                                             \
                    third_row(U);                                                                                 \
                } else {                                                                                          \
                    Store<P>::load_link(d.links, V, MU, s, U, d.rows);                                            \
                }                                                                                                 \
                _Pragma("unroll") for (int k = 0; k < 12; k++) p[k] = rho_lds[k][n];                              \
                project<MU, SF>(p, h, f);                                                                         \
                su3_mul<false>(U, h, chi);                                                                        \
                reconstruct<MU, SF>(q, chi);                                                                      \
            }                                                                                                     \
            if (nbk[MU] >= 0) {                                                                                   \
                const int n = nbk[MU];                                                                            \
                const T f = (MU == 0 && apbc && wb) ? T(0.5) : fh;                                                \
                cx<T> U[9], p[12], h[6], chi[6];                                                                  \
                if constexpr (LDSL) {                                                                             \
                    _Pragma("unroll") for (int e3 = 0; e3 < 3; e3++) {                                            \
                        const f4v a = link_lds[3 * MU + e3][n];                                                   \
                        U[2 * e3] = {a.x, a.y};                                                                   \
                        U[2 * e3 + 1] = {a.z, a.w};                                                               \
                    }                                                                                             \
                    third_row(U);                                                                                 \
                } else {                                                                                          \
                    const int sn = s + (n - l) / sg.lstr[MU] * g.stride[MU];                                      \
                    Store<P>::load_link(d.links, V, MU, sn, U, d.rows);                                           \
                }                                                                                                 \
                _Pragma("unroll") for (int k = 0; k < 12; k++) p[k] = rho_lds[k][n];                              \
                project<MU, SB>(p, h, f);                                                                         \
                su3_mul<true>(U, h, chi);                                                                         \
                reconstruct<MU, SB>(q, chi);                                                                      \
            }
            sched_fence();
            WD_SAP_BLK_HOP(0)
            sched_fence();
            WD_SAP_BLK_HOP(1)
            sched_fence();
            WD_SAP_BLK_HOP(2)
            sched_fence();
            WD_SAP_BLK_HOP(3)
            sched_fence();
#undef WD_SAP_BLK_HOP
        }
        // <q, rho> and <q, q> over the block, accumulated in FP64
        double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const cx<T> r = rho_lds[k][l];
            const double qr = q[k].r, qi = q[k].i, rr = r.r, ri = r.i;
            v[0] += qr * rr + qi * ri;
            v[1] += qr * ri - qi * rr;
            v[2] += qr * qr + qi * qi;
        }
        group_sum3(v, red);  // its barrier also ends every lane's reads of rho_lds for this step
        const double ar = v[2] > 0.0 ? v[0] / v[2] : 0.0, ai = v[2] > 0.0 ? v[1] / v[2] : 0.0;
        const cx<T> alpha = {(T)ar, (T)ai};
        const bool more = it + 1 < nmr;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const cx<T> r = rho_lds[k][l];
            if constexpr (ELDS) e_lds[k][l] = e_lds[k][l] + cmul(alpha, r);
            else e[k] = e[k] + cmul(alpha, r);
            if (more) rho_lds[k][l] = r - cmul(alpha, q[k]);
        }
    }

    // ---- x_out = x_in + e
    if (active) {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            cx<T> ek;
            if constexpr (ELDS) ek = e_lds[k][l];
            else ek = e[k];
            double2 o = make_double2((double)ek.r, (double)ek.i);
            if (!xzero && !own_zero) {
                const double2 a = xin[(size_t)k * V + s];
                o.x += a.x;
                o.y += a.y;
            }
            xout[(size_t)k * V + s] = o;
        }
    }
}

template <int P, bool LDSL, bool REGC>
hipError_t launch_pass(const dirac_op *op, const SapGeom &sg, int colour, int nblk, const double2 *b,
                       const double2 *xin, double2 *xout, bool xzero, bool own_zero, int nmr, int nrhs,
                       double bscale, hipStream_t st) {
    const int threads = (sg.bvol + 63) / 64 * 64;
    const int apbc = (op->flags & WDIRAC_ANTIPERIODIC_T) ? 1 : 0;
    hipLaunchKernelGGL((sap_pass_kernel<P, LDSL, REGC>), dim3(nblk, nrhs), dim3(threads), 0, st, b, xin, xout,
                       (size_t)12 * op->g.V, op->data(P), op->g, sg, colour, xzero ? 1 : 0, own_zero ? 1 : 0, nmr,
                       apbc, bscale);
    return hipGetLastError();
}

hipError_t sap_pass(const dirac_op *op, const sap_params &p, const SapGeom &sg, int colour, const double2 *b,
                    const double2 *xin, double2 *xout, bool xzero, bool own_zero, int nrhs, double bs,
                    hipStream_t st) {
    int nblk = sg.nblocks;
    int dec = colour;
    if (colour >= 0) {
        if (sg.pair_dir < 0) {
            if (colour == 1) return hipSuccess;  // a single block, of colour 0
            dec = -1;
        } else {
            nblk = sg.nblocks / 2;
        }
    }
    if (p.prec == WDIRAC_F64)
        return launch_pass<WDIRAC_F64, false, false>(op, sg, dec, nblk, b, xin, xout, xzero, own_zero, p.mr_iters,
                                                     nrhs, bs, st);
    const bool ldsl = op->link_rows == 2, regc = op->clover_compact;
    if (ldsl && regc)
        return launch_pass<WDIRAC_F32, true, true>(op, sg, dec, nblk, b, xin, xout, xzero, own_zero, p.mr_iters,
                                                   nrhs, bs, st);
    if (ldsl)
        return launch_pass<WDIRAC_F32, true, false>(op, sg, dec, nblk, b, xin, xout, xzero, own_zero, p.mr_iters,
                                                    nrhs, bs, st);
    if (regc)
        return launch_pass<WDIRAC_F32, false, true>(op, sg, dec, nblk, b, xin, xout, xzero, own_zero, p.mr_iters,
                                                    nrhs, bs, st);
    return launch_pass<WDIRAC_F32, false, false>(op, sg, dec, nblk, b, xin, xout, xzero, own_zero, p.mr_iters, nrhs,
                                                 bs, st);
}

}  // namespace

int sap_geometry(const dirac_op *op, const sap_params *p, SapGeom &sg) {
    if (!op || !p) return fail(WDIRAC_EINVAL, "null operator or SAP parameters");
    if (p->prec != WDIRAC_F64 && p->prec != WDIRAC_F32)
        return fail(WDIRAC_EINVAL, "SAP precision must be WDIRAC_F64 or WDIRAC_F32");
    if (!op->data(p->prec).links) return fail(WDIRAC_EUNSUPPORTED, "SAP precision not materialised at create");
    if (p->cycles < 1 || p->mr_iters < 1) return fail(WDIRAC_EINVAL, "SAP cycles and mr_iters must be >= 1");
    if (p->additive != 0 && p->additive != 1) return fail(WDIRAC_EINVAL, "SAP additive must be 0 or 1");
    long long vol = 1;
    sg.pair_dir = -1;
    for (int mu = 0; mu < 4; mu++) {
        const int B = p->block[mu], L = op->g.n[mu];
        if (B < 1 || L % B) return fail(WDIRAC_EINVAL, "SAP block extents must divide the lattice extents");
        sg.b[mu] = B;
        sg.nb[mu] = L / B;
        if (sg.nb[mu] != 1 && sg.nb[mu] % 2)
            return fail(WDIRAC_EINVAL, "SAP blocks per direction must be even or 1 (red-black colouring)");
        sg.span[mu] = sg.nb[mu] == 1 ? 1 : 0;
        if (sg.nb[mu] % 2 == 0) sg.pair_dir = mu;
        vol *= B;
    }
    if (vol > kSapMaxBlock) return fail(WDIRAC_EINVAL, "SAP blocks may hold at most 256 sites");
    sg.bvol = (int)vol;
    sg.lstr[3] = 1;
    sg.lstr[2] = sg.b[3];
    sg.lstr[1] = sg.b[3] * sg.b[2];
    sg.lstr[0] = sg.b[3] * sg.b[2] * sg.b[1];
    sg.nblocks = op->g.V / sg.bvol;
    return WDIRAC_OK;
}

size_t sap_workspace(const dirac_op *op, const sap_params *p, int nrhs) {
    return (p->additive && p->cycles > 1) ? field_rhs_bytes(WDIRAC_F64, op->g.V) * (size_t)nrhs : 0;
}

hipError_t sap_apply(const dirac_op *op, const sap_params &p, const SapGeom &sg, double2 *x, const double2 *b,
                     int nrhs, double2 *work, double bscale, hipStream_t st) {
    if (!p.additive) {
        for (int cyc = 0; cyc < p.cycles; cyc++)
            for (int c = 0; c < 2; c++) {
                const hipError_t e =
                    sap_pass(op, p, sg, c, b, x, x, cyc == 0 && c == 0, cyc == 0 && c == 1, nrhs, bscale, st);
                if (e != hipSuccess) return e;
            }
        return hipSuccess;
    }
    // additive: every block from the same x, so consecutive cycles alternate between x and the workspace, the
    // last one writing x
    double2 *bufs[2] = {x, work};
    int out = (p.cycles % 2) ? 0 : 1;
    const double2 *in = nullptr;
    for (int cyc = 0; cyc < p.cycles; cyc++) {
        const hipError_t e = sap_pass(op, p, sg, -1, b, in, bufs[out], cyc == 0, false, nrhs, bscale, st);
        if (e != hipSuccess) return e;
        in = bufs[out];
        out ^= 1;
    }
    return hipSuccess;
}

}  // namespace wd

using namespace wd;

extern "C" {

size_t dirac_sap_workspace_bytes(const dirac_op *op, const sap_params *p, int nrhs) {
    SapGeom sg;
    if (nrhs < 1 || sap_geometry(op, p, sg)) return 0;
    return sap_workspace(op, p, nrhs);
}

int dirac_sap(const dirac_op *op, double *x, const double *b, int nrhs, const sap_params *p, void *work,
              size_t work_bytes, void *stream) {
    SapGeom sg;
    int rc = sap_geometry(op, p, sg);
    if (rc) return rc;
    if (!x || !b) return fail(WDIRAC_EINVAL, "null field pointer");
    if (nrhs < 1) return fail(WDIRAC_EINVAL, "nrhs must be >= 1");
    const size_t n = field_rhs_bytes(WDIRAC_F64, op->g.V) * (size_t)nrhs;
    const char *xb = reinterpret_cast<const char *>(x), *bb = reinterpret_cast<const char *>(b);
    if (xb < bb + n && bb < xb + n) return fail(WDIRAC_EINVAL, "x overlaps b");
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(work)) & 15)
        return fail(WDIRAC_EINVAL, "field pointers must be 16-byte aligned");
    const size_t need = sap_workspace(op, p, nrhs);
    if (need && (!work || work_bytes < need)) return fail(WDIRAC_EINVAL, "SAP workspace too small");
    if (need) {
        const char *wb = static_cast<const char *>(work);
        if ((wb < xb + n && xb < wb + need) || (wb < bb + n && bb < wb + need))
            return fail(WDIRAC_EINVAL, "SAP workspace overlaps x or b");
    }
    const hipError_t e = sap_apply(op, *p, sg, reinterpret_cast<double2 *>(x), reinterpret_cast<const double2 *>(b),
                                   nrhs, static_cast<double2 *>(work), 1.0, (hipStream_t)stream);
    if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("SAP launch: ") + hipGetErrorString(e));
    return WDIRAC_OK;
}

}  // extern "C"
