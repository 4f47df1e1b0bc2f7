// Even-odd (red-black) reduction of D x = b, one parity at a time.
//
// With D = A + H (A(x): the site-local term, mass plus the clover term of
// Eqs. (1.11)-(1.12); H: the hopping sum of Eq. (1.13), which only couples
// sites of opposite parity), eliminating the odd sites gives
//   S x_e = b_e - H_eo A_oo^{-1} b_o,   S = A_ee - H_eo A_oo^{-1} H_oe,
//   x_o   = A_oo^{-1} (b_o - H_oe x_e).
// Red-black site colouring is among the splittings the paper's solver
// library uses for its Schwarz smoothers (Sec. 1.3); here it halves the
// Krylov vectors of FGMRES and improves the conditioning of the system.
//
// parity_kernel: one lane per site of the output parity.  It forms, in
// registers, an optional self term (the input itself or A(x) times it), the
// eight hops from the opposite-parity field (spin projection, SU(3) product,
// reconstruction: the same device functions as the full-lattice stencil),
// and optionally multiplies the sum by A(x)^{-1}, stored per site in the
// packed clover layout.  Parity fields list one parity's sites in
// lexicographic order, i.e. at half-lattice index s >> 1 (n_X even), so a
// neighbour's index is its full-lattice index shifted right by one.
//
// Work-groups are dealt like the full stencil's T-sweep: the eight XCDs
// (work-groups go to them round-robin) each take 1/8 of every T-slice of the
// half lattice and advance through the slices together, so T-neighbour
// slices are still in the Infinity Cache and Z/Y neighbours mostly in the
// same XCD's L2.
#include <algorithm>
#include <mutex>
#include <vector>

#include "schur.h"
#include "stencil.h"

namespace wd {

namespace {

// full-lattice site (and coordinates) of half-lattice index i of parity p
__device__ __forceinline__ int parity_site(const Geom &g, int i, int p, int c[4]) {
    const int X2 = g.n[3] >> 1;
    int r = i / X2;
    const int xh = i - r * X2;
    c[2] = r % g.n[2];
    r /= g.n[2];
    c[1] = r % g.n[1];
    c[0] = r / g.n[1];
    c[3] = 2 * xh + ((p + c[0] + c[1] + c[2]) & 1);
    return ((c[0] * g.n[1] + c[1]) * g.n[2] + c[2]) * g.n[3] + c[3];
}

// Fence between hops.  The kernel is one basic block, so the compiler would
// issue every hop's loads first and do all the arithmetic afterwards (all
// eight hops in flight, far beyond the register file).  The empty asm takes
// the accumulators as in/out operands, so a hop's arithmetic must be done
// before it, and clobbers memory, so the next hop's loads stay after it.
// WD_PARITY_FENCE = 1: a fence after every hop; 2: after each direction's pair of hops.
#ifndef WD_PARITY_FENCE
#define WD_PARITY_FENCE 1
#endif
template <typename T, int NR>
__device__ __forceinline__ void hop_boundary(cx<T> (&acc)[NR][12], int level = 1) {
    if (level < WD_PARITY_FENCE) return;
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int k = 0; k < 12; k++) asm volatile("" : "+v"(acc[r][k].r), "+v"(acc[r][k].i) : : "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// Right-hand sides of one launch: a work-group row (blockIdx.y) takes NR
// consecutive entries, so each lane loads its links and A(x) or A(x)^{-1}
// once for all of them.
constexpr int kParMax = 16;
constexpr int kParNr = 2;  // right-hand sides per lane
// FP16S with at least four right-hand sides in a launch: four per lane (147-151 VGPRs, 3 waves/SIMD instead of
// 4), so a lane's links and A or A^-1 serve four of them (measured at 48^3 x 96: S 0.84 -> 0.77 ms per RHS on
// 4 RHS).  With two or three the idle slots would cost the occupancy for nothing (0.82 -> 0.89 ms per launch on 2).
constexpr int kParNrF16 = 4;
#ifndef WD_PARITY_COLUMN
#define WD_PARITY_COLUMN 1
#endif
#ifndef WD_PARITY_COLUMN_F16
#define WD_PARITY_COLUMN_F16 0
#endif
constexpr bool kParColumnWalk = WD_PARITY_COLUMN != 0;
struct ParityTable {
    void *out[kParMax];
    const void *self[kParMax];
    const void *hop[kParMax];
    int n;
};

template <int P, int MU, bool DAG, int ROWS, int NR>
__device__ __forceinline__ void parity_hops(const OpData &d, const Geom &g, const ParityTable &tab, int r0, int nr,
                                            int Vh, int s, const int c[4], bool apbc, typename Store<P>::T fh,
                                            cx<typename Store<P>::T> (&acc)[NR][12]) {
    using T = typename Store<P>::T;
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    const int st = g.stride[MU], L = g.n[MU];
    const int sf = (c[MU] == L - 1) ? s - (L - 1) * st : s + st;
    const int sb = (c[MU] == 0) ? s + (L - 1) * st : s - st;
    cx<T> U[9];
    {
        const T f = (MU == 0 && apbc && c[0] == g.n[0] - 1) ? -fh : fh;
        Store<P>::load_link(d.links, g.V, MU, s, U, ROWS);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (r < nr) {
                cx<T> p[12], h[6], chi[6];
                Store<P>::load_spinor(tab.hop[r0 + r], Vh, sf >> 1, p);
                project<MU, SF>(p, h, f);
                su3_mul<false>(U, h, chi);
                reconstruct<MU, SF>(acc[r], chi);
            }
        }
    }
    hop_boundary<T, NR>(acc, 1);
    {
        const T f = (MU == 0 && apbc && c[0] == 0) ? -fh : fh;
        Store<P>::load_link(d.links, g.V, MU, sb, U, ROWS);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (r < nr) {
                cx<T> p[12], h[6], chi[6];
                Store<P>::load_spinor(tab.hop[r0 + r], Vh, sb >> 1, p);
                project<MU, SB>(p, h, f);
                su3_mul<true>(U, h, chi);
                reconstruct<MU, SB>(acc[r], chi);
            }
        }
    }
    hop_boundary<T, NR>(acc, 2);
}

// SELF: 0 none, 1 the input, 2 A(x) times the input.  HOP: add fh * 2 * H hop
// (fh = -1/2 adds H, +1/2 subtracts it).  INV: multiply the sum by A(x)^{-1}.
// ROWS: stored rows per link (a compile-time constant: a run-time choice
// between the two link formats costs the FP64 kernels spills).  NR: right-
// hand sides per lane (register block).
template <int P, bool DAG, int SELF, bool HOP, bool INV, int ROWS, int NR>
__global__ __launch_bounds__(256) void parity_kernel(ParityTable tab, OpData d, const void *cinv, Geom g, int parity,
                                                     int apbc, typename Store<P>::T fh, int tpr) {
    using T = typename Store<P>::T;
    const int Vh = g.V >> 1;
    int i;
    {
        // block -> (XCD k, T-slice t, tile within the slice's k-th eighth)
        const int hs = Vh / g.n[0];
        const int k = blockIdx.x & 7, j = blockIdx.x >> 3;
        const int t = j / tpr, tile = j - t * tpr;
        const int r0 = t * hs + (int)(((long long)k * hs) >> 3);
        const int r1 = t * hs + (int)(((long long)(k + 1) * hs) >> 3);
        i = r0 + tile * (int)blockDim.x + (int)threadIdx.x;
        if (i >= r1) return;
    }
    const int r0 = (int)blockIdx.y * NR;
    const int nr = min(NR, tab.n - r0);
    int c[4];
    const int s = parity_site(g, i, parity, c);
    cx<T> acc[NR][12];
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[r][k] = mk<T>(0, 0);
    if (SELF == 1) {
#pragma unroll
        for (int r = 0; r < NR; r++)
            if (r < nr) Store<P>::load_spinor(tab.self[r0 + r], Vh, i, acc[r]);
    } else if (SELF == 2) {
#pragma unroll
        for (int b = 0; b < 2; b++) {
            if (d.clover_compact) {
                T cr[28];
                Store<P>::load_clover_compact(d.clover, g.V, b, s, cr);
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    if (r < nr) {
                        cx<T> x[6];
                        Store<P>::load_half(tab.self[r0 + r], Vh, i, b, x);
                        clover_block_compact((T)d.diag, cr, x, &acc[r][6 * b]);
                    }
                }
            } else {
                T dd[6];
                cx<T> uu[15];
                Store<P>::load_clover(d.clover, g.V, b, s, dd, uu);
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    if (r < nr) {
                        cx<T> x[6];
                        Store<P>::load_half(tab.self[r0 + r], Vh, i, b, x);
                        clover_block(dd, uu, x, &acc[r][6 * b]);
                    }
                }
            }
        }
    }
    if (HOP) {
        hop_boundary<T, NR>(acc, 2);
        parity_hops<P, 0, DAG, ROWS, NR>(d, g, tab, r0, nr, Vh, s, c, apbc != 0, fh, acc);
        parity_hops<P, 1, DAG, ROWS, NR>(d, g, tab, r0, nr, Vh, s, c, apbc != 0, fh, acc);
        parity_hops<P, 2, DAG, ROWS, NR>(d, g, tab, r0, nr, Vh, s, c, apbc != 0, fh, acc);
        parity_hops<P, 3, DAG, ROWS, NR>(d, g, tab, r0, nr, Vh, s, c, apbc != 0, fh, acc);
    }
    if (INV) {
#pragma unroll
        for (int b = 0; b < 2; b++) {
            T dd[6];
            cx<T> uu[15];
            Store<P>::load_clover(cinv, g.V, b, s, dd, uu);
#pragma unroll
            for (int r = 0; r < NR; r++) {
                if (r < nr) {
                    cx<T> y[6];
                    clover_block(dd, uu, &acc[r][6 * b], y);
#pragma unroll
                    for (int k = 0; k < 6; k++) acc[r][6 * b + k] = y[k];
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++)
        if (r < nr) Store<P>::store_spinor(tab.out[r0 + r], Vh, i, acc[r]);
}

// Column walk of the parity kernel: a lane takes one (z, y, x) column and the
// sites of the output parity in a T-chunk of kParChunk slices, i.e. every
// second t.  The forward T neighbour psi(t+1) it loads at step t is also the
// backward T neighbour of its next site t+2, so that hop's half-spinor
// U_T(t+1)^H (1 + s gamma_T) psi(t+1) is formed once and carried in registers
// (one spinor load per site saved).  Work-groups are dealt as in the T-sweep
// above: each XCD takes 1/8 of the columns of every T-chunk.
#ifndef WD_PARITY_CHUNK
#define WD_PARITY_CHUNK 4
#endif
constexpr int kParChunk = WD_PARITY_CHUNK;  // T-slices per chunk (kParChunk / 2 sites per lane)

template <int P, bool DAG, int SELF, bool HOP, bool INV, int ROWS, int NR, int CH>
__global__ __launch_bounds__(256) void parity_column_kernel(ParityTable tab, OpData d, const void *cinv, Geom g,
                                                            int parity, int apbc, typename Store<P>::T fh,
                                                            int tpr) {
    using T = typename Store<P>::T;
    static_assert(HOP, "the column walk carries T hops");
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    const int Vh = g.V >> 1, C = g.stride[0], nT = g.n[0];
    int col, t0;
    {
        const int k = blockIdx.x & 7, j = blockIdx.x >> 3;
        const int tc = j / tpr, tile = j - tc * tpr;
        const int q0 = (int)(((long long)k * C) >> 3), q1 = (int)(((long long)(k + 1) * C) >> 3);
        col = q0 + tile * (int)blockDim.x + (int)threadIdx.x;
        if (col >= q1) return;
        t0 = tc * CH;
    }
    const int t1 = min(t0 + CH, nT);
    const int r0 = (int)blockIdx.y * NR;
    const int nr = min(NR, tab.n - r0);
    int c[4];
    c[3] = col % g.n[3];
    c[2] = (col / g.n[3]) % g.n[2];
    c[1] = col / (g.n[3] * g.n[2]);
    int t = t0 + ((parity + t0 + c[1] + c[2] + c[3]) & 1);
    cx<T> chiT[NR][6];
    {
        // backward T hop of the first site, from scratch
        const int tm = (t == 0) ? nT - 1 : t - 1;
        const T f = (apbc && t == 0) ? -fh : fh;
        cx<T> U[9];
        Store<P>::load_link(d.links, g.V, 0, tm * C + col, U, ROWS);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (r < nr) {
                cx<T> p[12], h[6];
                Store<P>::load_spinor(tab.hop[r0 + r], Vh, (tm * C + col) >> 1, p);
                project<0, SB>(p, h, f);
                su3_mul<true>(U, h, chiT[r]);
            }
        }
    }
    for (; t < t1; t += 2) {
        c[0] = t;
        const int s = t * C + col, i = s >> 1;
        cx<T> acc[NR][12];
#pragma unroll
        for (int r = 0; r < NR; r++)
#pragma unroll
            for (int k = 0; k < 12; k++) acc[r][k] = mk<T>(0, 0);
        if (SELF == 1) {
#pragma unroll
            for (int r = 0; r < NR; r++)
                if (r < nr) Store<P>::load_spinor(tab.self[r0 + r], Vh, i, acc[r]);
        } else if (SELF == 2) {
#pragma unroll
            for (int b = 0; b < 2; b++) {
                if (d.clover_compact) {
                    T cr[28];
                    Store<P>::load_clover_compact(d.clover, g.V, b, s, cr);
#pragma unroll
                    for (int r = 0; r < NR; r++) {
                        if (r < nr) {
                            cx<T> x[6];
                            Store<P>::load_half(tab.self[r0 + r], Vh, i, b, x);
                            clover_block_compact((T)d.diag, cr, x, &acc[r][6 * b]);
                        }
                    }
                } else {
                    T dd[6];
                    cx<T> uu[15];
                    Store<P>::load_clover(d.clover, g.V, b, s, dd, uu);
#pragma unroll
                    for (int r = 0; r < NR; r++) {
                        if (r < nr) {
                            cx<T> x[6];
                            Store<P>::load_half(tab.self[r0 + r], Vh, i, b, x);
                            clover_block(dd, uu, x, &acc[r][6 * b]);
                        }
                    }
                }
            }
        }
        hop_boundary<T, NR>(acc, 2);
        // T: the forward hop loads psi(t+1); the carried backward hop is added; when t + 2 is this lane's next
        // site, psi(t+1) also yields that site's backward half-spinor (the link U_T(t+1) loaded for it)
        {
            const bool wrap = (t == nT - 1);
            const int tp = wrap ? 0 : t + 1;
            const T ff = (apbc && wrap) ? -fh : fh;
            const bool next = CH > 2 && t + 2 < t1;  // chunks of 2 slices: one site per lane, nothing carried
            cx<T> U[9], Un[9];
            Store<P>::load_link(d.links, g.V, 0, s, U, ROWS);
            if (next) Store<P>::load_link(d.links, g.V, 0, tp * C + col, Un, ROWS);
#pragma unroll
            for (int r = 0; r < NR; r++) {
                if (r < nr) {
                    cx<T> p[12], h[6], chi[6];
                    Store<P>::load_spinor(tab.hop[r0 + r], Vh, (tp * C + col) >> 1, p);
                    project<0, SF>(p, h, ff);
                    su3_mul<false>(U, h, chi);
                    reconstruct<0, SF>(acc[r], chi);
                    reconstruct<0, SB>(acc[r], chiT[r]);
                    if (next) {
                        project<0, SB>(p, h, fh);
                        su3_mul<true>(Un, h, chiT[r]);
                    }
                }
            }
        }
        hop_boundary<T, NR>(acc, 1);
        parity_hops<P, 1, DAG, ROWS, NR>(d, g, tab, r0, nr, Vh, s, c, apbc != 0, fh, acc);
        parity_hops<P, 2, DAG, ROWS, NR>(d, g, tab, r0, nr, Vh, s, c, apbc != 0, fh, acc);
        parity_hops<P, 3, DAG, ROWS, NR>(d, g, tab, r0, nr, Vh, s, c, apbc != 0, fh, acc);
        if (INV) {
#pragma unroll
            for (int b = 0; b < 2; b++) {
                T dd[6];
                cx<T> uu[15];
                Store<P>::load_clover(cinv, g.V, b, s, dd, uu);
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    if (r < nr) {
                        cx<T> y[6];
                        clover_block(dd, uu, &acc[r][6 * b], y);
#pragma unroll
                        for (int k = 0; k < 6; k++) acc[r][6 * b + k] = y[k];
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NR; r++)
            if (r < nr) Store<P>::store_spinor(tab.out[r0 + r], Vh, i, acc[r]);
    }
}

template <int P, bool DAG, int SELF, bool HOP, bool INV>
hipError_t launch_mode(const dirac_op *op, int parity, const ParityItem *items, size_t nitems, double fh,
                       hipStream_t st) {
    using T = typename Store<P>::T;
    const int Vh = op->g.V >> 1;
    const int hs = Vh / op->g.n[0];                 // half-lattice sites per T-slice
    const int tpr = ((hs + 7) / 8 + 255) / 256;     // 256-site tiles per eighth of a slice
    const int apbc = (op->flags & WDIRAC_ANTIPERIODIC_T) ? 1 : 0;
    const bool rows2 = op->link_rows == 2 || !HOP;
    for (size_t a = 0; a < nitems; a += kParMax) {
        ParityTable tab;
        tab.n = (int)std::min<size_t>(kParMax, nitems - a);
        for (int q = 0; q < tab.n; q++) {
            tab.out[q] = items[a + q].out;
            tab.self[q] = items[a + q].self;
            tab.hop[q] = items[a + q].hop;
        }
        // pairs (or fours, see kParNrF16) for every count, a lone last right-hand side included: a single-RHS
        // instantiation may round differently, and results must not depend on how right-hand sides are grouped
        // (the per-RHS arithmetic of the pair and four instantiations is the same code, unrolled)
        if constexpr (HOP && (P != WDIRAC_F16S || WD_PARITY_COLUMN_F16)) {
            if (kParColumnWalk) {
                // the column walk: T-chunks of CH slices, each XCD 1/8 of the columns
                constexpr int CH = P == WDIRAC_F16S ? 2 : kParChunk;
                const int C = op->g.stride[0];
                const int tpc = ((C + 7) / 8 + 255) / 256;
                const dim3 gc((op->g.n[0] + CH - 1) / CH * 8 * tpc, (tab.n + kParNr - 1) / kParNr);
                if (rows2)
                    hipLaunchKernelGGL((parity_column_kernel<P, DAG, SELF, HOP, INV, 2, kParNr, CH>), gc, dim3(256),
                                       0, st, tab, op->data(P), op->cinv(P), op->g, parity, apbc, (T)fh, tpc);
                else
                    hipLaunchKernelGGL((parity_column_kernel<P, DAG, SELF, HOP, INV, 3, kParNr, CH>), gc, dim3(256),
                                       0, st, tab, op->data(P), op->cinv(P), op->g, parity, apbc, (T)fh, tpc);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
                continue;
            }
        }
        if constexpr (P == WDIRAC_F16S) {
            if (tab.n >= kParNrF16) {
                const dim3 g4(op->g.n[0] * 8 * tpr, (tab.n + kParNrF16 - 1) / kParNrF16);
                if (rows2)
                    hipLaunchKernelGGL((parity_kernel<P, DAG, SELF, HOP, INV, 2, kParNrF16>), g4, dim3(256), 0, st,
                                       tab, op->data(P), op->cinv(P), op->g, parity, apbc, (T)fh, tpr);
                else
                    hipLaunchKernelGGL((parity_kernel<P, DAG, SELF, HOP, INV, 3, kParNrF16>), g4, dim3(256), 0, st,
                                       tab, op->data(P), op->cinv(P), op->g, parity, apbc, (T)fh, tpr);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
                continue;
            }
        }
        const dim3 grid(op->g.n[0] * 8 * tpr, (tab.n + kParNr - 1) / kParNr);
        if (rows2)
            hipLaunchKernelGGL((parity_kernel<P, DAG, SELF, HOP, INV, 2, kParNr>), grid, dim3(256), 0, st, tab,
                               op->data(P), op->cinv(P), op->g, parity, apbc, (T)fh, tpr);
        else
            hipLaunchKernelGGL((parity_kernel<P, DAG, SELF, HOP, INV, 3, kParNr>), grid, dim3(256), 0, st, tab,
                               op->data(P), op->cinv(P), op->g, parity, apbc, (T)fh, tpr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int P>
hipError_t launch_p(int mode, bool dag, const dirac_op *op, int parity, const ParityItem *it, size_t n,
                    hipStream_t st) {
    switch (mode) {
    case kParHopInv:
        return dag ? launch_mode<P, true, 0, true, true>(op, parity, it, n, -0.5, st)
                   : launch_mode<P, false, 0, true, true>(op, parity, it, n, -0.5, st);
    case kParCloverSub:
        return dag ? launch_mode<P, true, 2, true, false>(op, parity, it, n, 0.5, st)
                   : launch_mode<P, false, 2, true, false>(op, parity, it, n, 0.5, st);
    case kParApply: return launch_mode<P, false, 2, true, false>(op, parity, it, n, -0.5, st);
    case kParInvSelf: return launch_mode<P, false, 1, false, true>(op, parity, it, n, 0.0, st);
    case kParSelfSub: return launch_mode<P, false, 1, true, false>(op, parity, it, n, 0.5, st);
    case kParInvSelfSub: return launch_mode<P, false, 1, true, true>(op, parity, it, n, 0.5, st);
    default: return hipErrorInvalidValue;
    }
}

// full <-> parity fields: K 16-byte vectors per site (+ the FP16S scale)
template <int K, bool SCALE, bool MERGE>
__global__ __launch_bounds__(256) void parity_copy_kernel(char *__restrict__ full, char *__restrict__ even,
                                                          char *__restrict__ odd, Geom g, size_t rb_full,
                                                          size_t rb_half) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int V = g.V, Vh = V >> 1;
    if (s >= V) return;
    int r = s, c3 = r % g.n[3];
    r /= g.n[3];
    int c2 = r % g.n[2];
    r /= g.n[2];
    int c1 = r % g.n[1], c0 = r / g.n[1];
    const int p = (c0 + c1 + c2 + c3) & 1;
    char *h = (p ? odd : even) + (size_t)blockIdx.y * rb_half;
    char *f = full + (size_t)blockIdx.y * rb_full;
    uint4 *hv = reinterpret_cast<uint4 *>(h);
    uint4 *fv = reinterpret_cast<uint4 *>(f);
    const int j = s >> 1;
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (MERGE) fv[(size_t)k * V + s] = hv[(size_t)k * Vh + j];
        else hv[(size_t)k * Vh + j] = fv[(size_t)k * V + s];
    }
    if (SCALE) {
        float *hs = reinterpret_cast<float *>(h + (size_t)48 * Vh);
        float *fs = reinterpret_cast<float *>(f + (size_t)48 * V);
        if (MERGE) fs[s] = hs[j];
        else hs[j] = fs[s];
    }
}

template <bool MERGE>
hipError_t parity_copy(const dirac_op *op, int prec, void *full, void *even, void *odd, int nrhs, hipStream_t st) {
    const int V = op->g.V;
    const dim3 grid((V + 255) / 256, nrhs);
    const size_t rf = field_rhs_bytes(prec, V), rh = field_rhs_bytes(prec, V >> 1);
    char *f = static_cast<char *>(full), *e = static_cast<char *>(even), *o = static_cast<char *>(odd);
    if (prec == WDIRAC_F64)
        hipLaunchKernelGGL((parity_copy_kernel<12, false, MERGE>), grid, dim3(256), 0, st, f, e, o, op->g, rf, rh);
    else if (prec == WDIRAC_F32)
        hipLaunchKernelGGL((parity_copy_kernel<6, false, MERGE>), grid, dim3(256), 0, st, f, e, o, op->g, rf, rh);
    else
        hipLaunchKernelGGL((parity_copy_kernel<3, true, MERGE>), grid, dim3(256), 0, st, f, e, o, op->g, rf, rh);
    return hipGetLastError();
}

// In-place Gauss-Jordan inversion with partial pivoting of one 6x6 complex
// block; returns false when a pivot is below tiny.
__device__ bool invert6(cx<double> a[6][6], double tiny) {
    int piv[6];
    for (int k = 0; k < 6; k++) {
        int p = k;
        double best = a[k][k].r * a[k][k].r + a[k][k].i * a[k][k].i;
        for (int i = k + 1; i < 6; i++) {
            const double m = a[i][k].r * a[i][k].r + a[i][k].i * a[i][k].i;
            if (m > best) {
                best = m;
                p = i;
            }
        }
        if (!(sqrt(best) > tiny)) return false;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < 6; j++) {
                const cx<double> t = a[k][j];
                a[k][j] = a[p][j];
                a[p][j] = t;
            }
        const cx<double> inv = {a[k][k].r / best, -a[k][k].i / best};
        a[k][k] = mk<double>(1, 0);
        for (int j = 0; j < 6; j++) a[k][j] = cmul(a[k][j], inv);
        for (int i = 0; i < 6; i++) {
            if (i == k) continue;
            const cx<double> f = a[i][k];
            a[i][k] = mk<double>(0, 0);
            for (int j = 0; j < 6; j++) a[i][j] = a[i][j] - cmul(f, a[k][j]);
        }
    }
    for (int k = 5; k >= 0; k--)
        if (piv[k] != k)
            for (int i = 0; i < 6; i++) {
                const cx<double> t = a[i][k];
                a[i][k] = a[i][piv[k]];
                a[i][piv[k]] = t;
            }
    return true;
}

__global__ __launch_bounds__(256) void clover_invert_kernel(double2 *__restrict__ inv, const double2 *__restrict__ can,
                                                            int V, double diag, double csw, int *__restrict__ bad) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    for (int b = 0; b < 2; b++) {
        const double2 *c = can + (size_t)42 * s + 21 * b;
        cx<double> a[6][6];
        double scale = 0;
        for (int i = 0; i < 6; i++) a[i][i] = mk<double>(diag + csw * c[i].x, 0.0);
        int k = 6;
        for (int i = 0; i < 6; i++)
            for (int j = i + 1; j < 6; j++, k++) {
                a[i][j] = mk<double>(csw * c[k].x, csw * c[k].y);
                a[j][i] = mk<double>(csw * c[k].x, -csw * c[k].y);
            }
        for (int i = 0; i < 6; i++)
            for (int j = 0; j < 6; j++) scale = fmax(scale, fabs(a[i][j].r) + fabs(a[i][j].i));
        if (!invert6(a, 1e-12 * scale)) {
            *bad = 1;
            for (int i = 0; i < 6; i++)
                for (int j = 0; j < 6; j++) a[i][j] = mk<double>(0, 0);
        }
        double2 *o = inv + (size_t)42 * s + 21 * b;
        for (int i = 0; i < 6; i++) o[i] = make_double2(a[i][i].r, 0.0);
        k = 6;
        for (int i = 0; i < 6; i++)
            for (int j = i + 1; j < 6; j++, k++)  // Hermitian part of the computed inverse
                o[k] = make_double2(0.5 * (a[i][j].r + a[j][i].r), 0.5 * (a[i][j].i - a[j][i].i));
    }
}

}  // namespace

hipError_t parity_launch_items(int mode, int prec, bool dag, const dirac_op *op, int parity, const ParityItem *items,
                               size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    switch (prec) {
    case WDIRAC_F64: return launch_p<WDIRAC_F64>(mode, dag, op, parity, items, n, st);
    case WDIRAC_F32: return launch_p<WDIRAC_F32>(mode, dag, op, parity, items, n, st);
    case WDIRAC_F16S: return launch_p<WDIRAC_F16S>(mode, dag, op, parity, items, n, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t parity_launch_list(int mode, int prec, bool dag, const dirac_op *op, int parity,
                              const std::vector<ParityItem> &items, hipStream_t st) {
    return parity_launch_items(mode, prec, dag, op, parity, items.data(), items.size(), st);
}

hipError_t parity_launch(int mode, int prec, bool dag, const dirac_op *op, int parity, void *out, const void *self,
                         const void *hop, int nrhs, hipStream_t st) {
    const size_t rb = field_rhs_bytes(prec, op->g.V / 2);
    std::vector<ParityItem> items;
    for (int r = 0; r < nrhs; r++)
        items.push_back({static_cast<char *>(out) + r * rb,
                         self ? static_cast<const char *>(self) + r * rb : nullptr,
                         hop ? static_cast<const char *>(hop) + r * rb : nullptr});
    return parity_launch_list(mode, prec, dag, op, parity, items, st);
}

hipError_t schur_apply_list(int prec, bool dag, const dirac_op *op, const std::vector<SchurItem> &items,
                            hipStream_t st) {
    std::vector<ParityItem> a, b;
    for (const SchurItem &it : items) {
        a.push_back({it.tmp, nullptr, it.in});
        b.push_back({it.out, it.in, it.tmp});
    }
    hipError_t e = parity_launch_list(kParHopInv, prec, dag, op, 1, a, st);
    if (e != hipSuccess) return e;
    return parity_launch_list(kParCloverSub, prec, dag, op, 0, b, st);
}

hipError_t schur_apply(int prec, bool dag, const dirac_op *op, void *out, const void *in, void *tmp, int nrhs,
                       hipStream_t st) {
    hipError_t e = parity_launch(kParHopInv, prec, dag, op, 1, tmp, nullptr, in, nrhs, st);
    if (e != hipSuccess) return e;
    return parity_launch(kParCloverSub, prec, dag, op, 0, out, in, tmp, nrhs, st);
}

hipError_t parity_split_launch(const dirac_op *op, int prec, void *even, void *odd, const void *full, int nrhs,
                               hipStream_t st) {
    return parity_copy<false>(op, prec, const_cast<void *>(full), even, odd, nrhs, st);
}

hipError_t parity_merge_launch(const dirac_op *op, int prec, void *full, const void *even, const void *odd,
                               int nrhs, hipStream_t st) {
    return parity_copy<true>(op, prec, full, const_cast<void *>(even), const_cast<void *>(odd), nrhs, st);
}

// Device scratch of dirac_apply_schur_noalloc: the odd-parity intermediate A_oo^{-1} H_oe x of nrhs fields,
// at most kSchurScratchBytes.  Every device that runs the library holds one copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns on that device (schur_scratch_init).
constexpr size_t kSchurScratchBytes = (size_t)128 << 20;
__device__ __align__(256) char schur_scratch[kSchurScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_addr[kScratchDevices] = {};
}  // namespace

int schur_scratch_init(int device) {
    if (device < 0 || device >= kScratchDevices) return fail(WDIRAC_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_addr[device]) return WDIRAC_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(schur_scratch));
    if (e != hipSuccess || !p)
        return fail(WDIRAC_EHIP, std::string("hipGetSymbolAddress of the Schur scratch: ") + hipGetErrorString(e));
    g_scratch_addr[device] = p;
    return WDIRAC_OK;
}

void *schur_scratch_addr(int device) {
    if (device < 0 || device >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return g_scratch_addr[device];
}

hipError_t clover_invert_launch(double2 *inv_can, const double2 *can, int V, double diag, double csw, int *bad,
                                hipStream_t st) {
    hipLaunchKernelGGL(clover_invert_kernel, dim3((V + 255) / 256), dim3(256), 0, st, inv_can, can, V, diag, csw,
                       bad);
    return hipGetLastError();
}

}  // namespace wd

using namespace wd;

namespace {

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
    return x < y + nb && y < x + na;
}

bool misaligned(const void *p) { return reinterpret_cast<uintptr_t>(p) & 15; }

// operator prepared for even-odd work at this precision
int check_parity(const dirac_op *op, int prec, int nrhs) {
    if (!op) return fail(WDIRAC_EINVAL, "null operator");
    if (nrhs < 1) return fail(WDIRAC_EINVAL, "nrhs must be >= 1");
    if (prec != WDIRAC_F64 && prec != WDIRAC_F32 && prec != WDIRAC_F16S)
        return fail(WDIRAC_EINVAL, "unknown precision " + std::to_string(prec));
    if (!(op->flags & WDIRAC_EVEN_ODD)) return fail(WDIRAC_EUNSUPPORTED, "operator created without WDIRAC_EVEN_ODD");
    if (!op->data(prec).links || !op->cinv(prec))
        return fail(WDIRAC_EUNSUPPORTED, "precision " + std::to_string(prec) + " not materialised at create");
    return WDIRAC_OK;
}

// out (n bytes) must not overlap `hop`, and equals or is disjoint from `self`
int check_out(const void *out, const void *self, const void *hop, size_t n) {
    if (!out) return fail(WDIRAC_EINVAL, "null field pointer");
    if (misaligned(out) || misaligned(self) || misaligned(hop))
        return fail(WDIRAC_EINVAL, "field pointers must be 16-byte aligned");
    if (hop && overlaps(out, n, hop, n)) return fail(WDIRAC_EINVAL, "output overlaps a field read at neighbours");
    if (self && self != out && overlaps(out, n, self, n))
        return fail(WDIRAC_EINVAL, "output partially overlaps the same-parity input");
    return WDIRAC_OK;
}

int hip_result(hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return WDIRAC_OK;
}

}  // namespace

extern "C" {

size_t dirac_parity_field_bytes(const dirac_op *op, int prec, int nrhs) {
    if (!op || nrhs < 0) return 0;
    return field_rhs_bytes(prec, op->g.V / 2) * (size_t)nrhs;
}

int dirac_parity_split(const dirac_op *op, void *even, void *odd, const void *full, int nrhs, int prec,
                       void *stream) {
    int rc = check_parity(op, prec, nrhs);
    if (rc) return rc;
    if (!even || !odd || !full) return fail(WDIRAC_EINVAL, "null field pointer");
    const size_t nh = field_rhs_bytes(prec, op->g.V / 2) * nrhs, nf = field_rhs_bytes(prec, op->g.V) * nrhs;
    if (misaligned(even) || misaligned(odd) || misaligned(full))
        return fail(WDIRAC_EINVAL, "field pointers must be 16-byte aligned");
    if (overlaps(even, nh, odd, nh) || overlaps(even, nh, full, nf) || overlaps(odd, nh, full, nf))
        return fail(WDIRAC_EINVAL, "split buffers overlap");
    return hip_result(parity_split_launch(op, prec, even, odd, full, nrhs, (hipStream_t)stream), "split launch");
}

int dirac_parity_merge(const dirac_op *op, void *full, const void *even, const void *odd, int nrhs, int prec,
                       void *stream) {
    int rc = check_parity(op, prec, nrhs);
    if (rc) return rc;
    if (!even || !odd || !full) return fail(WDIRAC_EINVAL, "null field pointer");
    const size_t nh = field_rhs_bytes(prec, op->g.V / 2) * nrhs, nf = field_rhs_bytes(prec, op->g.V) * nrhs;
    if (misaligned(even) || misaligned(odd) || misaligned(full))
        return fail(WDIRAC_EINVAL, "field pointers must be 16-byte aligned");
    if (overlaps(full, nf, even, nh) || overlaps(full, nf, odd, nh)) return fail(WDIRAC_EINVAL, "merge buffers overlap");
    return hip_result(parity_merge_launch(op, prec, full, even, odd, nrhs, (hipStream_t)stream), "merge launch");
}

int dirac_apply_schur(const dirac_op *op, void *out, const void *in, void *tmp, int nrhs, int prec, int dagger,
                      void *stream) {
    int rc = check_parity(op, prec, nrhs);
    if (rc) return rc;
    if (!in || !tmp) return fail(WDIRAC_EINVAL, "null field pointer");
    const size_t nh = field_rhs_bytes(prec, op->g.V / 2) * nrhs;
    rc = check_out(out, nullptr, in, nh);
    if (rc) return rc;
    rc = check_out(tmp, nullptr, in, nh);
    if (rc) return rc;
    if (overlaps(out, nh, tmp, nh)) return fail(WDIRAC_EINVAL, "out overlaps tmp");
    return hip_result(schur_apply(prec, dagger != 0, op, out, in, tmp, nrhs, (hipStream_t)stream), "schur launch");
}

int dirac_apply_schur_noalloc(const dirac_op *op, void *out, const void *in, int nrhs, int prec, int dagger,
                              void *stream) {
    int rc = check_parity(op, prec, nrhs);
    if (rc) return rc;
    if (!in) return fail(WDIRAC_EINVAL, "null field pointer");
    const size_t rb = field_rhs_bytes(prec, op->g.V / 2), nh = rb * nrhs;
    if (nh > kSchurScratchBytes)
        return fail(WDIRAC_EINVAL, "the odd-parity intermediate needs " + std::to_string(nh) +
                                       " bytes, more than the static scratch of " +
                                       std::to_string(kSchurScratchBytes) + " bytes");
    rc = check_out(out, nullptr, in, nh);
    if (rc) return rc;
    char *tmp = static_cast<char *>(schur_scratch_addr(op->device));
    if (!tmp) return fail(WDIRAC_EHIP, "the Schur scratch of this device was not set up at create");
    hipStream_t st = (hipStream_t)stream;
    // chunks of right-hand sides with their tables on the stack: nothing is allocated
    constexpr int kChunk = 16;
    ParityItem a[kChunk], b[kChunk];
    for (int r0 = 0; r0 < nrhs; r0 += kChunk) {
        const int n = std::min(kChunk, nrhs - r0);
        for (int q = 0; q < n; q++) {
            const size_t off = (size_t)(r0 + q) * rb;
            a[q] = {tmp + off, nullptr, static_cast<const char *>(in) + off};
            b[q] = {static_cast<char *>(out) + off, static_cast<const char *>(in) + off, tmp + off};
        }
        rc = hip_result(parity_launch_items(kParHopInv, prec, dagger != 0, op, 1, a, n, st), "schur launch");
        if (rc) return rc;
        rc = hip_result(parity_launch_items(kParCloverSub, prec, dagger != 0, op, 0, b, n, st), "schur launch");
        if (rc) return rc;
    }
    return WDIRAC_OK;
}

int dirac_schur_prepare(const dirac_op *op, void *bhat, const void *b_even, const void *b_odd, void *tmp, int nrhs,
                        int prec, void *stream) {
    int rc = check_parity(op, prec, nrhs);
    if (rc) return rc;
    if (!b_even || !b_odd || !tmp) return fail(WDIRAC_EINVAL, "null field pointer");
    const size_t nh = field_rhs_bytes(prec, op->g.V / 2) * nrhs;
    rc = check_out(tmp, b_odd, nullptr, nh);
    if (rc) return rc;
    rc = check_out(bhat, b_even, tmp, nh);
    if (rc) return rc;
    if (overlaps(tmp, nh, b_even, nh)) return fail(WDIRAC_EINVAL, "tmp overlaps b_even (written before it is read)");
    hipStream_t st = (hipStream_t)stream;
    rc = hip_result(parity_launch(kParInvSelf, prec, false, op, 1, tmp, b_odd, nullptr, nrhs, st), "prepare launch");
    if (rc) return rc;
    return hip_result(parity_launch(kParSelfSub, prec, false, op, 0, bhat, b_even, tmp, nrhs, st), "prepare launch");
}

int dirac_schur_reconstruct(const dirac_op *op, void *x_odd, const void *x_even, const void *b_odd, int nrhs,
                            int prec, void *stream) {
    int rc = check_parity(op, prec, nrhs);
    if (rc) return rc;
    if (!x_even || !b_odd) return fail(WDIRAC_EINVAL, "null field pointer");
    const size_t nh = field_rhs_bytes(prec, op->g.V / 2) * nrhs;
    rc = check_out(x_odd, b_odd, x_even, nh);
    if (rc) return rc;
    return hip_result(parity_launch(kParInvSelfSub, prec, false, op, 1, x_odd, b_odd, x_even, nrhs,
                                    (hipStream_t)stream),
                      "reconstruct launch");
}

}  // extern "C"
