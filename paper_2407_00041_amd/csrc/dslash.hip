// Fused Wilson-clover stencil (Eq. (1.13); D = D_sc - D_nc of Eqs. (2.5)-(2.7)).
//
// One lane owns one lattice site and a register block of NR right-hand
// sides, and performs in registers what the paper splits into 16 kernel
// launches plus a self-coupling kernel (Algorithm 4 and the clover kernel):
// the self-coupling product A(x) psi(x), then for each of the 8 neighbours
// the spin projection to a half-spinor h = u + s B_mu d (the prp kernels of
// Listing 4.2), the SU(3) product with U_mu(x) or U_mu(x-mu)^H, and the
// reconstruction of the lower half as s B_mu^H (U h) (the back-substitution
// of Sec. 2.2).  Every link and clover entry is loaded once per site and
// register block and used for all NR right-hand sides; nothing but the
// result is written.
//
// Gamma basis: gamma_mu = [[0, B_mu], [B_mu^H, 0]], B_T = 1, B_Z = -i s3,
// B_Y = -i s2, B_X = -i s1, so the projector (I + s gamma_mu) maps
// (u, d) -> (h, s B_mu^H h) with h = u + s B_mu d.  D uses s = -1 for the
// forward hop and s = +1 for the backward hop; D^H swaps them.
//
// Work decomposition: a work item is (tile of up to 256 consecutive sites,
// register block of right-hand sides).  Items are dealt so that the
// work-group running on XCD k (work-groups go to the 8 XCDs round-robin)
// always gets tiles of the same 1/8 of every T-slice, and all XCDs advance
// through the T-slices together: the T-neighbours of a slice are then read
// while the slice is still in the Infinity Cache, and the Z-neighbours
// mostly come from the same XCD's L2.  The register blocks of one tile are
// consecutive items on the same XCD, so their shared links and clover stay
// in that XCD's L2 while it can hold them.  With fewer work-groups than
// items (an optional persistent grid) each work-group strides through the
// item list.
#include "spinor_io.h"
#include "stencil.h"
#include "dslash.h"

namespace wd {

struct Nbr {
    int fwd[4], bwd[4];
    bool fwd_wrapT, bwd_wrapT;
};

__device__ __forceinline__ Nbr neighbours(const Geom &g, int s) {
    Nbr n;
    int c[4];
    int r = s;
    c[3] = r % g.n[3]; r /= g.n[3];
    c[2] = r % g.n[2]; r /= g.n[2];
    c[1] = r % g.n[1];
    c[0] = r / g.n[1];
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        int st = g.stride[mu], L = g.n[mu];
        n.fwd[mu] = (c[mu] == L - 1) ? s - (L - 1) * st : s + st;
        n.bwd[mu] = (c[mu] == 0) ? s + (L - 1) * st : s - st;
    }
    n.fwd_wrapT = c[0] == g.n[0] - 1;
    n.bwd_wrapT = c[0] == 0;
    return n;
}

// Scheduling fences between hops bound how far the compiler hoists the
// loads of later hops (and with them the register pressure).
#ifndef WD_HOP_FENCE
#define WD_HOP_FENCE 1
#endif
__device__ __forceinline__ void hop_fence(int level) {
    if (WD_HOP_FENCE >= level) __builtin_amdgcn_sched_barrier(0);
}

template <int P, int MU, bool DAG, int NR>
__device__ __forceinline__ void hop_pair(const Chunk<NR> &ch, const OpData &d, int V, int s, const Nbr &nb,
                                         bool apbc, cx<typename Store<P>::T> (&acc)[NR][12]) {
    using T = typename Store<P>::T;
    constexpr int SF = DAG ? +1 : -1;  // forward projector (I + SF gamma)
    constexpr int SB = -SF;            // backward projector
    cx<T> U[9];
    // forward: -1/2 (I + SF gamma) (x) U_mu(x) psi(x+mu)
    {
        const T f = (MU == 0 && apbc && nb.fwd_wrapT) ? T(0.5) : T(-0.5);
        Store<P>::load_link(d.links, V, MU, s, U, d.rows);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (r < ch.nr) {
                cx<T> p[12], h[6], chi[6];
                Store<P>::load_spinor(ch.in[r], V, nb.fwd[MU], p);
                project<MU, SF>(p, h, f);
                su3_mul<false>(U, h, chi);
                reconstruct<MU, SF>(acc[r], chi);
            }
        }
    }
    hop_fence(2);
    // backward: -1/2 (I + SB gamma) (x) U_mu(x-mu)^H psi(x-mu)
    {
        const T f = (MU == 0 && apbc && nb.bwd_wrapT) ? T(0.5) : T(-0.5);
        Store<P>::load_link(d.links, V, MU, nb.bwd[MU], U, d.rows);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (r < ch.nr) {
                cx<T> p[12], h[6], chi[6];
                Store<P>::load_spinor(ch.in[r], V, nb.bwd[MU], p);
                project<MU, SB>(p, h, f);
                su3_mul<true>(U, h, chi);
                reconstruct<MU, SB>(acc[r], chi);
            }
        }
    }
}

template <int P, bool DAG, int NR>
__device__ __forceinline__ void site_apply(const Chunk<NR> &ch, const OpData &d, const Geom &g, int s, bool apbc) {
    using T = typename Store<P>::T;
    const int V = g.V;
    cx<T> acc[NR][12];
#pragma unroll
    for (int b = 0; b < 2; b++) {
        if (d.clover_compact) {
            T cr[28];
            Store<P>::load_clover_compact(d.clover, V, b, s, cr);
#pragma unroll
            for (int r = 0; r < NR; r++) {
                if (r < ch.nr) {
                    cx<T> p[6];
                    Store<P>::load_half(ch.in[r], V, s, b, p);
                    clover_block_compact((T)d.diag, cr, p, &acc[r][6 * b]);
                }
            }
        } else {
            T dd[6];
            cx<T> uu[15];
            Store<P>::load_clover(d.clover, V, b, s, dd, uu);
#pragma unroll
            for (int r = 0; r < NR; r++) {
                if (r < ch.nr) {
                    cx<T> p[6];
                    Store<P>::load_half(ch.in[r], V, s, b, p);
                    clover_block(dd, uu, p, &acc[r][6 * b]);
                }
            }
        }
    }
    const Nbr nb = neighbours(g, s);
    hop_fence(1);
    hop_pair<P, 0, DAG, NR>(ch, d, V, s, nb, apbc, acc);
    hop_fence(1);
    hop_pair<P, 1, DAG, NR>(ch, d, V, s, nb, apbc, acc);
    hop_fence(1);
    hop_pair<P, 2, DAG, NR>(ch, d, V, s, nb, apbc, acc);
    hop_fence(1);
    hop_pair<P, 3, DAG, NR>(ch, d, V, s, nb, apbc, acc);
    hop_fence(1);
#pragma unroll
    for (int r = 0; r < NR; r++)
        if (r < ch.nr) Store<P>::store_spinor(ch.out[r], V, s, acc[r]);
}

// Register T-sweep (tile order 3): one lane walks the sites t0..t1-1 of one
// column (z, y, x).  psi(t+1) is loaded once as the forward T neighbour and
// kept as the next step's own spinor, and the backward T hop of site t+1,
// -1/2 (I + SB gamma_T) (x) U_T(t)^H psi(t), is formed at step t and carried
// in registers, so no T-neighbour spinor or backward T link is re-read.
template <int P, bool DAG, int NR>
__device__ __forceinline__ void column_sweep(const Chunk<NR> &ch, const OpData &d, const Geom &g, int c, int t0,
                                             int t1, bool apbc) {
    using T = typename Store<P>::T;
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    const int V = g.V, S = g.stride[0], nT = g.n[0];
    // neighbour columns in Z, Y, X
    int cf[4], cb[4];
    {
        int r = c, q[4];
        q[3] = r % g.n[3]; r /= g.n[3];
        q[2] = r % g.n[2];
        q[1] = r / g.n[2];
#pragma unroll
        for (int mu = 1; mu < 4; mu++) {
            const int st = g.stride[mu], L = g.n[mu];
            cf[mu] = (q[mu] == L - 1) ? c - (L - 1) * st : c + st;
            cb[mu] = (q[mu] == 0) ? c + (L - 1) * st : c - st;
        }
    }
    cx<T> self[NR][12], chiT[NR][6];
    {
        const int tm = (t0 == 0) ? nT - 1 : t0 - 1;
        const T f = (apbc && t0 == 0) ? T(0.5) : T(-0.5);
        cx<T> U[9];
        Store<P>::load_link(d.links, V, 0, tm * S + c, U, d.rows);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (r < ch.nr) {
                cx<T> p[12], h[6];
                Store<P>::load_spinor(ch.in[r], V, tm * S + c, p);
                project<0, SB>(p, h, f);
                su3_mul<true>(U, h, chiT[r]);
                Store<P>::load_spinor(ch.in[r], V, t0 * S + c, self[r]);
            }
        }
    }
    for (int t = t0; t < t1; t++) {
        const int s = t * S + c;
        cx<T> acc[NR][12];
        // self coupling
#pragma unroll
        for (int b = 0; b < 2; b++) {
            if (d.clover_compact) {
                T cr[28];
                Store<P>::load_clover_compact(d.clover, V, b, s, cr);
#pragma unroll
                for (int r = 0; r < NR; r++)
                    if (r < ch.nr) clover_block_compact((T)d.diag, cr, &self[r][6 * b], &acc[r][6 * b]);
            } else {
                T dd[6];
                cx<T> uu[15];
                Store<P>::load_clover(d.clover, V, b, s, dd, uu);
#pragma unroll
                for (int r = 0; r < NR; r++)
                    if (r < ch.nr) clover_block(dd, uu, &self[r][6 * b], &acc[r][6 * b]);
            }
        }
        // backward T hop (carried), then the one for site t+1
        const bool last = (t == nT - 1);
        // U_T(s) serves both T hops of the step; the copy parked in the lane's LDS slot between them spares a
        // second load through the L2, which by then has often evicted it (measured: -75 B read per site)
        __shared__ cx<T> ut_lds[256][9];
        {
            const T f = (apbc && last) ? T(0.5) : T(-0.5);
            cx<T> U[9];
            Store<P>::load_link(d.links, V, 0, s, U, d.rows);
#pragma unroll
            for (int e = 0; e < 9; e++) ut_lds[threadIdx.x][e] = U[e];
#pragma unroll
            for (int r = 0; r < NR; r++) {
                if (r < ch.nr) {
                    reconstruct<0, SB>(acc[r], chiT[r]);
                    cx<T> h[6];
                    project<0, SB>(self[r], h, f);
                    su3_mul<true>(U, h, chiT[r]);
                }
            }
        }
        hop_fence(1);
        Nbr nb;
#pragma unroll
        for (int mu = 1; mu < 4; mu++) {
            nb.fwd[mu] = t * S + cf[mu];
            nb.bwd[mu] = t * S + cb[mu];
        }
        nb.fwd[0] = nb.bwd[0] = s;
        nb.fwd_wrapT = nb.bwd_wrapT = false;
        hop_pair<P, 1, DAG, NR>(ch, d, V, s, nb, false, acc);
        hop_fence(1);
        hop_pair<P, 2, DAG, NR>(ch, d, V, s, nb, false, acc);
        hop_fence(1);
        hop_pair<P, 3, DAG, NR>(ch, d, V, s, nb, false, acc);
        hop_fence(1);
        // forward T hop; psi(t+1) becomes the next step's own spinor
        {
            const int sp = (last ? 0 : t + 1) * S + c;
            const T f = (apbc && last) ? T(0.5) : T(-0.5);
            cx<T> U[9];
#pragma unroll
            for (int e = 0; e < 9; e++) U[e] = ut_lds[threadIdx.x][e];
#pragma unroll
            for (int r = 0; r < NR; r++) {
                if (r < ch.nr) {
                    cx<T> h[6], chi[6];
                    Store<P>::load_spinor(ch.in[r], V, sp, self[r]);
                    project<0, SF>(self[r], h, f);
                    su3_mul<false>(U, h, chi);
                    reconstruct<0, SF>(acc[r], chi);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NR; r++)
            if (r < ch.nr) Store<P>::store_spinor(ch.out[r], V, s, acc[r]);
        hop_fence(1);
    }
}

// site range [lo, hi) of tile slot vb (see TileMap in dslash.h)
__device__ __forceinline__ void tile_range(const TileMap &m, int vb, int &lo, int &hi) {
    if (m.order == kOrderTSweep) {
        const int k = vb & 7, j = vb >> 3;
        const int t = j / m.tiles_per_range, tile = j - t * m.tiles_per_range;
        const int base = t * m.slice;
        const int r0 = base + (int)(((long long)k * m.slice) >> 3);
        const int r1 = base + (int)(((long long)(k + 1) * m.slice) >> 3);
        lo = r0 + tile * m.block;
        hi = min(lo + m.block, r1);
    } else if (m.order == kOrderZPlanes) {
        const int k = vb & 7, j = vb >> 3;
        const int q = j / m.plane_tiles, tile = j - q * m.plane_tiles;
        const int zb = q / m.nt, t = q - zb * m.nt;
        const int z = zb * 8 + k;
        const int plane = m.slice / m.nz;
        lo = hi = 0;
        if (z < m.nz) {
            const int base = (t * m.nz + z) * plane;
            lo = base + tile * m.block;
            hi = min(lo + m.block, base + plane);
        }
    } else {
        int tile = vb;
        if (m.order == kOrderXcdChunk) {
            // contiguous ranges of tiles per XCD
            const int q = m.ntiles >> 3, rr = m.ntiles & 7;
            const int k = vb & 7, j = vb >> 3;
            tile = k * q + (k < rr ? k : rr) + j;
        }
        lo = tile * m.block;
        hi = min(lo + m.block, m.V);
    }
}

// site of lane l of tile slot vb in kOrderZGroups (-1: no site): XCD k takes the groups of zw consecutive z-planes
// (zw p, ..., zw p + zw - 1) with p = k mod 8, group-block by group-block, each block's T-planes in order; a tile
// is 64 consecutive (y, x) sites, wave w of the work-group in plane zw p + w
__device__ __forceinline__ int zgroup_site(const TileMap &m, int vb, int l) {
    const int k = vb & 7, j = vb >> 3;
    const int nxyb = (m.plane_tiles + m.xyb - 1) / m.xyb;
    const int tl = j % m.xyb, q = j / m.xyb;
    const int t = q % m.nt, r = q / m.nt;
    const int xyb = r % nxyb, zb = r / nxyb;
    const int tile = xyb * m.xyb + tl;
    const int z = m.zw * (zb * 8 + k) + (l >> 6);
    const int plane = m.slice / m.nz;
    const int xy = tile * 64 + (l & 63);
    if (z >= m.nz || tile >= m.plane_tiles || xy >= plane) return -1;
    return (t * m.nz + z) * plane + xy;
}

// Minimum waves per SIMD the register allocation must allow, per precision
// and register block (the compiler otherwise trades occupancy for early
// load hoisting).  Values from launch sweeps at 48^3 x 96.
#ifndef WD_OCC_F64_1
#define WD_OCC_F64_1 2
#endif
#ifndef WD_OCC_F64_2
#define WD_OCC_F64_2 2
#endif
#ifndef WD_OCC_F64_4
#define WD_OCC_F64_4 1
#endif
#ifndef WD_OCC_F32_1
#define WD_OCC_F32_1 4
#endif
#ifndef WD_OCC_F32_2
#define WD_OCC_F32_2 4
#endif
#ifndef WD_OCC_F32_4
#define WD_OCC_F32_4 3
#endif
#ifndef WD_OCC_F16_1
#define WD_OCC_F16_1 6
#endif
#ifndef WD_OCC_F16_2
#define WD_OCC_F16_2 4
#endif
#ifndef WD_OCC_F16_4
#define WD_OCC_F16_4 3
#endif
template <int P, int NR> constexpr int occupancy() {
    return P == WDIRAC_F64 ? (NR == 1 ? WD_OCC_F64_1 : NR == 2 ? WD_OCC_F64_2 : WD_OCC_F64_4)
         : P == WDIRAC_F32 ? (NR == 1 ? WD_OCC_F32_1 : NR == 2 ? WD_OCC_F32_2 : WD_OCC_F32_4)
                           : (NR == 1 ? WD_OCC_F16_1 : NR == 2 ? WD_OCC_F16_2 : WD_OCC_F16_4);
}

template <int P, bool DAG, int NR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(occupancy<P, NR>())))
void dslash_kernel(ChunkTable<NR> tab, OpData d, Geom g, TileMap m, int apbc) {
    const int nitems = m.nslots * tab.nchunks;   // nslots is a multiple of 8
    for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
        // XCD-affine dealing: w % 8 == vb % 8, consecutive items of one XCD
        // walk through the register blocks of a tile before the next tile
        const int xcd = w & 7, q = w >> 3;
        const int vb = (q / tab.nchunks) * 8 + xcd;
        const int c = q - (q / tab.nchunks) * tab.nchunks;
        int lo, hi;
        tile_range(m, vb, lo, hi);
        const int s = lo + (int)threadIdx.x;
        if (s < hi) site_apply<P, DAG, NR>(tab.c[c], d, g, s, apbc != 0);
    }
}

// the column sweep carries psi(t+1) and the T half-spinors: fewer waves
#ifndef WD_OCCC_F64_1
#define WD_OCCC_F64_1 2
#endif
#ifndef WD_OCCC_F32_1
#define WD_OCCC_F32_1 3
#endif
#ifndef WD_OCCC_F16_1
#define WD_OCCC_F16_1 4
#endif
template <int P, int NR> constexpr int occupancy_col() {
    return P == WDIRAC_F64 ? (NR == 1 ? WD_OCCC_F64_1 : 1)
                           : P == WDIRAC_F32 ? (NR == 1 ? WD_OCCC_F32_1 : NR == 2 ? 2 : 1)
                                             : (NR == 1 ? WD_OCCC_F16_1 : NR == 2 ? 2 : 1);
}

template <int P, bool DAG, int NR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(occupancy_col<P, NR>())))
void dslash_column_kernel(ChunkTable<NR> tab, OpData d, Geom g, TileMap m, int apbc) {
    const int nitems = m.nslots * tab.nchunks;
    for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
        const int xcd = w & 7, q = w >> 3;
        const int vb = (q / tab.nchunks) * 8 + xcd;
        const int c = q - (q / tab.nchunks) * tab.nchunks;
        // columns of XCD k's 1/8 of a slice (or of its patches), T-chunk tc
        const int k = vb & 7, j = vb >> 3;
        const int tc = j / m.tiles_per_range, tile = j - tc * m.tiles_per_range;
        const int t0 = tc * m.tchunk, t1 = min(t0 + m.tchunk, g.n[0]);
        int col = -1;
        if (m.order == kOrderPatch) {
            const int p0 = (int)(((long long)k * m.patches) >> 3), p1 = (int)(((long long)(k + 1) * m.patches) >> 3);
            const int pi = p0 + tile;
            const int lx = (int)threadIdx.x % kPatchX, ly = ((int)threadIdx.x / kPatchX) % kPatchY,
                      lz = (int)threadIdx.x / (kPatchX * kPatchY);
            const int px = pi % m.npx, py = (pi / m.npx) % m.npy, pzi = pi / (m.npx * m.npy);
            const int x = px * kPatchX + lx, y = py * kPatchY + ly, z = pzi * m.pz + lz;
            if (pi < p1 && x < g.n[3] && y < g.n[2] && z < g.n[1]) col = (z * g.n[2] + y) * g.n[3] + x;
        } else {
            const int r0 = (int)(((long long)k * m.slice) >> 3), r1 = (int)(((long long)(k + 1) * m.slice) >> 3);
            const int cc = r0 + tile * m.block + (int)threadIdx.x;
            if (cc < r1) col = cc;
        }
        if (col >= 0 && t0 < t1) column_sweep<P, DAG, NR>(tab.c[c], d, g, col, t0, t1, apbc != 0);
    }
}

// Link-stationary multi-RHS stencil (FP32 compute, two-row links): a lane
// loads the 8 links it needs (rows 0 and 1 of U_mu(x) and U_mu(x-mu), 96
// registers) and stages its own clover blocks in LDS once, then walks every
// right-hand side of the launch reading only spinors.  Links and clover
// are thus read from memory once per launch instead of once per register
// block, which a 4 MB L2 per XCD cannot provide when many right-hand sides
// stream through.  The LDS slots are private to their lane (no barrier).
// Per right-hand side the arithmetic is that of dslash_kernel (same order).
template <int P, bool DAG>
__global__ __launch_bounds__(kStationaryBlock) __attribute__((amdgpu_waves_per_eu(2)))
void dslash_stationary_kernel(RhsTable tab, OpData d, Geom g, TileMap m, int apbc) {
    using T = typename Store<P>::T;
    static_assert(P != WDIRAC_F64, "FP64 links do not fit in registers");
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    __shared__ float4 lds[18][kStationaryBlock];
    int s;
    if (m.order == kOrderZGroups) {
        s = zgroup_site(m, blockIdx.x, threadIdx.x);
        if (s < 0) return;
    } else {
        int lo, hi;
        tile_range(m, blockIdx.x, lo, hi);
        s = lo + (int)threadIdx.x;
        if (s >= hi) return;
    }
    const int V = g.V;
    const int tid = threadIdx.x;
    const bool compact = d.clover_compact != 0;
#pragma unroll
    for (int b = 0; b < 2; b++) {
        if (compact) {
            T cr[28];
            Store<P>::load_clover_compact(d.clover, V, b, s, cr);
#pragma unroll
            for (int k = 0; k < 7; k++)
                lds[7 * b + k][tid] = make_float4(-2 * cr[4 * k], -2 * cr[4 * k + 1], -2 * cr[4 * k + 2], -2 * cr[4 * k + 3]);
        } else {
            T dd[6];
            cx<T> uu[15];
            Store<P>::load_clover(d.clover, V, b, s, dd, uu);
            lds[9 * b + 0][tid] = make_float4(-2 * dd[0], -2 * dd[1], -2 * dd[2], -2 * dd[3]);
            lds[9 * b + 1][tid] = make_float4(-2 * dd[4], -2 * dd[5], -2 * uu[0].r, -2 * uu[0].i);
#pragma unroll
            for (int k = 0; k < 7; k++)
                lds[9 * b + 2 + k][tid] = make_float4(-2 * uu[1 + 2 * k].r, -2 * uu[1 + 2 * k].i, -2 * uu[2 + 2 * k].r,
                                                      -2 * uu[2 + 2 * k].i);
        }
    }
    const T dg = T(-2) * (T)d.diag;
    const Nbr nb = neighbours(g, s);
    cx<T> Lf[4][6], Lb[4][6];
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        cx<T> U[9];
        Store<P>::load_link(d.links, V, mu, s, U, 2);
#pragma unroll
        for (int e = 0; e < 6; e++) Lf[mu][e] = U[e];
        Store<P>::load_link(d.links, V, mu, nb.bwd[mu], U, 2);
#pragma unroll
        for (int e = 0; e < 6; e++) Lb[mu][e] = U[e];
    }
    // everything up to the store is accumulated scaled by -2 (exact): the clover
    // blocks were staged times -2, the hop projections drop their factor -1/2
    // (an anti-periodic T wrap keeps a sign), and -1/2 is applied once at the end
    const T ffT = (apbc && nb.fwd_wrapT) ? T(-1) : T(1);
    const T fbT = (apbc && nb.bwd_wrapT) ? T(-1) : T(1);
    for (int r = 0; r < tab.n; r++) {
        const void *in = tab.in[r];
        cx<T> acc[12];
        {
            cx<T> self[12];
            Store<P>::load_spinor(in, V, s, self);
#pragma unroll
            for (int b = 0; b < 2; b++) {
                if (compact) {
                    T cr[28];
#pragma unroll
                    for (int k = 0; k < 7; k++) {
                        const float4 q = lds[7 * b + k][tid];
                        cr[4 * k] = q.x; cr[4 * k + 1] = q.y; cr[4 * k + 2] = q.z; cr[4 * k + 3] = q.w;
                    }
                    clover_block_compact(dg, cr, &self[6 * b], &acc[6 * b]);
                } else {
                    T dd[6];
                    cx<T> uu[15];
                    const float4 a0 = lds[9 * b][tid], a1 = lds[9 * b + 1][tid];
                    dd[0] = a0.x; dd[1] = a0.y; dd[2] = a0.z; dd[3] = a0.w; dd[4] = a1.x; dd[5] = a1.y;
                    uu[0] = {a1.z, a1.w};
#pragma unroll
                    for (int k = 0; k < 7; k++) {
                        const float4 q = lds[9 * b + 2 + k][tid];
                        uu[1 + 2 * k] = {q.x, q.y};
                        uu[2 + 2 * k] = {q.z, q.w};
                    }
                    clover_block(dd, uu, &self[6 * b], &acc[6 * b]);
                }
            }
        }
        hop_fence(1);
#define WD_STAT_HOP(MU)                                                         \
        {                                                                       \
            cx<T> U[9], p[12], h[6], chi[6];                                    \
            _Pragma("unroll") for (int e = 0; e < 6; e++) U[e] = Lf[MU][e];     \
            third_row(U);                                                       \
            Store<P>::load_spinor(in, V, nb.fwd[MU], p);                        \
            if (MU == 0) project<MU, SF>(p, h, ffT); else project_unit<MU, SF>(p, h); \
            su3_mul<false>(U, h, chi);                                          \
            reconstruct<MU, SF>(acc, chi);                                      \
        }                                                                       \
        {                                                                       \
            cx<T> U[9], p[12], h[6], chi[6];                                    \
            _Pragma("unroll") for (int e = 0; e < 6; e++) U[e] = Lb[MU][e];     \
            third_row(U);                                                       \
            Store<P>::load_spinor(in, V, nb.bwd[MU], p);                        \
            if (MU == 0) project<MU, SB>(p, h, fbT); else project_unit<MU, SB>(p, h); \
            su3_mul<true>(U, h, chi);                                           \
            reconstruct<MU, SB>(acc, chi);                                      \
        }                                                                       \
        hop_fence(1);
        WD_STAT_HOP(0)
        WD_STAT_HOP(1)
        WD_STAT_HOP(2)
        WD_STAT_HOP(3)
#undef WD_STAT_HOP
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = T(-0.5) * acc[k];
        Store<P>::store_spinor(tab.out[r], V, s, acc);
    }
}

// ---------------------------------------------------------------------------
// host side

TileMap make_tilemap(const Geom &g, int order, int block, int tchunk) {
    TileMap m;
    m.order = order;
    m.block = block;
    m.V = g.V;
    m.slice = g.V / g.n[0];
    m.tchunk = tchunk < 1 ? 1 : (tchunk > g.n[0] ? g.n[0] : tchunk);
    m.patches = m.npx = m.npy = 0;
    m.pz = block / (kPatchX * kPatchY);
    m.nt = g.n[0];
    m.nz = g.n[1];
    m.zw = 1;
    m.xyb = 1;
    m.plane_tiles = 0;
    if (order == kOrderColumn) {
        const int per_range = (m.slice + 7) / 8;
        m.tiles_per_range = (per_range + block - 1) / block;
        m.ntiles = (g.n[0] + m.tchunk - 1) / m.tchunk * 8 * m.tiles_per_range;
    } else if (order == kOrderPatch) {
        m.npx = (g.n[3] + kPatchX - 1) / kPatchX;
        m.npy = (g.n[2] + kPatchY - 1) / kPatchY;
        m.patches = m.npx * m.npy * ((g.n[1] + m.pz - 1) / m.pz);
        m.tiles_per_range = (m.patches + 7) / 8;
        m.ntiles = (g.n[0] + m.tchunk - 1) / m.tchunk * 8 * m.tiles_per_range;
    } else if (order == kOrderZGroups) {
        m.zw = block / 64;
        m.plane_tiles = (m.slice / m.nz + 63) / 64;
        m.xyb = (tchunk >= 1 && tchunk < m.plane_tiles) ? tchunk : m.plane_tiles;
        const int nxyb = (m.plane_tiles + m.xyb - 1) / m.xyb;
        m.ntiles = ((m.nz + m.zw - 1) / m.zw + 7) / 8 * nxyb * m.nt * m.xyb * 8;
    } else if (order == kOrderZPlanes) {
        m.plane_tiles = (m.slice / m.nz + block - 1) / block;
        m.ntiles = (m.nz + 7) / 8 * m.nt * m.plane_tiles * 8;
    } else if (order == kOrderTSweep) {
        const int per_range = (m.slice + 7) / 8;
        m.tiles_per_range = (per_range + block - 1) / block;
        m.ntiles = g.n[0] * 8 * m.tiles_per_range;
    } else {
        m.tiles_per_range = 0;
        m.ntiles = (g.V + block - 1) / block;
    }
    m.nslots = (m.ntiles + 7) / 8 * 8;
    return m;
}

static Tuning g_tuning;
static std::mutex g_tuning_mu;

std::mutex &tuning_mutex() { return g_tuning_mu; }
Tuning &tuning_unlocked() { return g_tuning; }
Tuning tuning_snapshot() {
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    return g_tuning;
}

// Work-groups of one kernel instance that fit on the device at once.
template <int P, bool DAG, int NR>
static int resident_blocks(int block) {
    static int cached[5] = {0, 0, 0, 0, 0};
    const int slot = block / 64;
    if (!cached[slot]) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dslash_kernel<P, DAG, NR>, block, 0) != hipSuccess ||
            cus * per_cu < 8) {
            (void)hipGetLastError();
            return 8;
        }
        cached[slot] = cus * per_cu / 8 * 8;
    }
    return cached[slot];
}

template <int P, bool DAG, int NR>
static int resident_blocks_col(int block) {
    static int cached[5] = {0, 0, 0, 0, 0};
    const int slot = block / 64;
    if (!cached[slot]) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dslash_column_kernel<P, DAG, NR>, block, 0) !=
                hipSuccess ||
            cus * per_cu < 8) {
            (void)hipGetLastError();
            return 8;
        }
        cached[slot] = cus * per_cu / 8 * 8;
    }
    return cached[slot];
}

template <int P, bool DAG, int NR>
static hipError_t launch_chunks(const std::vector<Chunk<NR>> &chunks, const OpData &d, const Geom &g, int apbc,
                                bool persistent, const LaunchCfg &cfg, hipStream_t st) {
    const Tuning tu = tuning_snapshot();
    const TileMap m = make_tilemap(g, cfg.order, cfg.block, cfg.tchunk);
    for (size_t c0 = 0; c0 < chunks.size(); c0 += kMaxChunks) {
        ChunkTable<NR> tab;
        tab.nchunks = (int)std::min(chunks.size() - c0, (size_t)kMaxChunks);
        for (int i = 0; i < tab.nchunks; i++) tab.c[i] = chunks[c0 + i];
        const long long items = (long long)m.nslots * tab.nchunks;
        long long grid = items;
        if ((persistent && tu.persistent_blocks > 0) || cfg.persistent) {
            // a persistent grid: at most the resident work-groups, each striding
            // through the item list (by default the hardware dispatcher hands
            // out one work-group per item in order, which measured faster)
            long long cap = is_column_order(m.order) ? resident_blocks_col<P, DAG, NR>(cfg.block)
                                                    : resident_blocks<P, DAG, NR>(cfg.block);
            if (tu.persistent_blocks > 0 && tu.persistent_blocks < cap) cap = tu.persistent_blocks / 8 * 8;
            if (cap < 8) cap = 8;
            if (grid > cap) grid = cap;
        }
        if (grid > (1LL << 30)) return hipErrorInvalidValue;
        if (is_column_order(m.order))
            hipLaunchKernelGGL((dslash_column_kernel<P, DAG, NR>), dim3((unsigned)grid), dim3(cfg.block), 0, st, tab,
                               d, g, m, apbc);
        else
            hipLaunchKernelGGL((dslash_kernel<P, DAG, NR>), dim3((unsigned)grid), dim3(cfg.block), 0, st, tab, d, g,
                               m, apbc);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Group the right-hand sides of all batches, in order, into register blocks
// of at most NR (a block may span batches).
template <int P, bool DAG, int NR>
static hipError_t launch_nr(const dirac_batch *batches, int nbatch, const OpData &d, const Geom &g, int apbc,
                            bool persistent, const LaunchCfg &cfg, hipStream_t st) {
    const size_t rb = field_rhs_bytes(P, g.V);
    std::vector<std::pair<const void *, void *>> rhs;
    for (int b = 0; b < nbatch; b++)
        for (int r = 0; r < batches[b].nrhs; r++)
            rhs.emplace_back(static_cast<const char *>(batches[b].in) + r * rb,
                             static_cast<char *>(batches[b].out) + r * rb);
    std::vector<Chunk<NR>> chunks;
    for (size_t r0 = 0; r0 < rhs.size(); r0 += NR) {
        Chunk<NR> c;
        c.nr = (int)std::min<size_t>(NR, rhs.size() - r0);
        for (int r = 0; r < NR; r++) {
            const size_t rr = r0 + std::min(r, c.nr - 1);
            c.in[r] = rhs[rr].first;
            c.out[r] = rhs[rr].second;
        }
        chunks.push_back(c);
    }
    return launch_chunks<P, DAG, NR>(chunks, d, g, apbc, persistent, cfg, st);
}

// Link-stationary launch: all right-hand sides of all batches, in groups of
// `group` (2 .. kMaxStationaryRhs - 1; else kMaxStationaryRhs) per launch,
// one work-group of kStationaryBlock lanes per tile.  Measurements below are
// FP32 and FP16S, 41 RHS at 48^3 x 96, all results bit-identical.
// - Plane tiles (zw = 1: 128 consecutive sites of one (t, z) plane; each XCD
//   walks the T-planes of every eighth z in T order) keep a site's
//   T-neighbours in work-groups that run at the same time, a few right-hand
//   sides apart; with T-slice tiles the next slice only started after the
//   current one had walked every right-hand side (FP32 44.0 -> 39.5 ms, FP16S
//   27.5 -> 25.7 ms).  Both z-neighbours are planes of other XCDs.
// - Z-pair tiles (zw >= 2: the two waves take the same 64 (y, x) sites of
//   planes z and z + 1) read one of the two z-neighbours inside the
//   work-group (FP32 groups of 12: 33.7 ms; four z-planes in 256-lane
//   work-groups were slower, 41 ms).  With zw = 4 an XCD walks its z-pairs
//   along T in blocks of about eight x-rows before the next block, so a
//   T-neighbour's tile ran only a few work-groups earlier (FP32 groups of
//   16: 30.3 ms; FP16S in one launch 24.3 ms; blocks of whole rows measured
//   faster than ragged ones).
// - Smaller groups re-read the links and clover once per launch but shorten
//   the time between the uses of a neighbour spinor (FP32 plane tiles: groups
//   of 6 36.4 ms, all in one launch 39.7 ms; FP16S is fastest in one launch).
template <int P, bool DAG>
static hipError_t launch_stationary(const dirac_batch *batches, int nbatch, const OpData &d, const Geom &g,
                                    int apbc, int group, int zw, hipStream_t st) {
    const size_t rb = field_rhs_bytes(P, g.V);
    std::vector<std::pair<const void *, void *>> rhs;
    for (int b = 0; b < nbatch; b++)
        for (int r = 0; r < batches[b].nrhs; r++)
            rhs.emplace_back(static_cast<const char *>(batches[b].in) + r * rb,
                             static_cast<char *>(batches[b].out) + r * rb);
    static_assert(kStationaryBlock == 128, "z-pair tiles are two waves");
    // zw = 4: z-pair tiles walked along T in (y, x) blocks of about eight x-rows (0: whole planes)
    const int xyb = zw == 4 ? (8 * g.n[3] + 63) / 64 : 0;
    const TileMap m = make_tilemap(g, zw >= 2 ? kOrderZGroups : kOrderZPlanes, kStationaryBlock, xyb);
    const size_t grp = (group >= 2 && group < kMaxStationaryRhs) ? (size_t)group : (size_t)kMaxStationaryRhs;
    for (size_t r0 = 0; r0 < rhs.size(); r0 += grp) {
        RhsTable tab;
        tab.n = (int)std::min(grp, rhs.size() - r0);
        for (int i = 0; i < kMaxStationaryRhs; i++) {
            const size_t k = r0 + std::min(i, tab.n - 1);
            tab.in[i] = rhs[k].first;
            tab.out[i] = rhs[k].second;
        }
        hipLaunchKernelGGL((dslash_stationary_kernel<P, DAG>), dim3((unsigned)m.nslots), dim3(kStationaryBlock), 0, st,
                           tab, d, g, m, apbc);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int P, bool DAG>
static hipError_t launch_p(const dirac_batch *batches, int nbatch, const OpData &d, const Geom &g, int apbc,
                           bool persistent, LaunchCfg cfg, hipStream_t st) {
    int total = 0;
    for (int b = 0; b < nbatch; b++) total += batches[b].nrhs;
    if (cfg.order == kOrderStationary) {
        if constexpr (P != WDIRAC_F64) {
            if (d.rows == 2)
                return launch_stationary<P, DAG>(batches, nbatch, d, g, apbc, cfg.tchunk, cfg.nr, st);
        }
        cfg.order = kOrderTSweep;  // FP64 or full links: the register-blocked site kernel
    }
    if (total == 1) cfg.nr = 1;
    if (is_column_order(cfg.order) && P == WDIRAC_F64 && cfg.nr > 2) cfg.nr = 2;  // register budget
    if (cfg.nr >= 4) return launch_nr<P, DAG, 4>(batches, nbatch, d, g, apbc, persistent, cfg, st);
    if (cfg.nr >= 2) return launch_nr<P, DAG, 2>(batches, nbatch, d, g, apbc, persistent, cfg, st);
    return launch_nr<P, DAG, 1>(batches, nbatch, d, g, apbc, persistent, cfg, st);
}

hipError_t dslash_launch_cfg(const dirac_batch *batches, int nbatch, int prec, bool dagger, const OpData &d,
                             const Geom &g, int apbc, bool persistent, const LaunchCfg &cfg, hipStream_t st) {
    switch (prec) {
    case WDIRAC_F64:
        return dagger ? launch_p<WDIRAC_F64, true>(batches, nbatch, d, g, apbc, persistent, cfg, st)
                      : launch_p<WDIRAC_F64, false>(batches, nbatch, d, g, apbc, persistent, cfg, st);
    case WDIRAC_F32:
        return dagger ? launch_p<WDIRAC_F32, true>(batches, nbatch, d, g, apbc, persistent, cfg, st)
                      : launch_p<WDIRAC_F32, false>(batches, nbatch, d, g, apbc, persistent, cfg, st);
    case WDIRAC_F16S:
        return dagger ? launch_p<WDIRAC_F16S, true>(batches, nbatch, d, g, apbc, persistent, cfg, st)
                      : launch_p<WDIRAC_F16S, false>(batches, nbatch, d, g, apbc, persistent, cfg, st);
    }
    return hipErrorInvalidValue;
}

// The configuration of a launch: the autotuned one for this lattice,
// precision, right-hand-side count and link format if there is one, else
// the process-wide defaults.
hipError_t dslash_launch_batches(const dirac_batch *batches, int nbatch, int prec, bool dagger, const OpData &d,
                                 const Geom &g, int apbc, bool persistent, hipStream_t st) {
    int total = 0;
    for (int b = 0; b < nbatch; b++) total += batches[b].nrhs;
    const Tuning tu = tuning_snapshot();
    LaunchCfg cfg{tu.order, tu.block, tu.tchunk, (prec >= 0 && prec < 3) ? tu.nr[prec] : 1};
    if (!tu.explicit_launch) tuned_cfg(g, prec, total, d.rows, d.clover_compact, cfg);
    return dslash_launch_cfg(batches, nbatch, prec, dagger, d, g, apbc, persistent, cfg, st);
}

}  // namespace wd
