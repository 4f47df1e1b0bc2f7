// Launch-side types of the stencil kernels (internal).
#pragma once

#include <mutex>
#include <vector>

#include "common.h"

namespace wd {

// A register block: up to NR right-hand sides handled by the same lanes.
template <int NR> struct Chunk {
    const void *in[NR];
    void *out[NR];
    int nr;  // valid entries; the rest repeat the last valid pointers
};

constexpr int kMaxChunks = 24;  // register blocks per launch (kernel-argument budget)

template <int NR> struct ChunkTable {
    Chunk<NR> c[kMaxChunks];
    int nchunks;
};

// Tile orders (site range of a tile slot)
constexpr int kOrderLinear = 0;    // tile slot = tile, lexicographic
constexpr int kOrderXcdChunk = 1;  // each XCD gets a contiguous 1/8 of the lattice
constexpr int kOrderTSweep = 2;    // each XCD gets 1/8 of every T-slice; slices in order
constexpr int kOrderColumn = 3;    // lanes walk columns along T (register-carried T neighbours)
constexpr int kOrderPatch = 4;     // as kOrderColumn, a work-group's columns form a z-y-x patch
constexpr int kOrderStationary = 5;  // FP32/FP16S, two-row links: each lane keeps its links (registers) and
                                     // clover (LDS) for all right-hand sides of the launch; plane tiles
constexpr int kOrderZPlanes = 6;  // XCD k takes the (t, z) planes with z = k mod 8, z-block by z-block, each
                                   // z-block's planes in T order (tiles of one plane are consecutive)
constexpr int kOrderZGroups = 7;  // link-stationary kernel only: as kOrderZPlanes over pairs of consecutive
                                  // z-planes, a work-group's two waves take the same 64 (y, x) sites of each;
                                  // optionally walked along T in (y, x) blocks of xyb tiles
constexpr int kPatchX = 16, kPatchY = 4;  // patch extent in X and Y; Z extent = block / 64
constexpr int kStationaryBlock = 128;     // work-group size of the link-stationary kernel (LDS budget)
constexpr int kMaxStationaryRhs = 64;     // right-hand sides per link-stationary launch

struct RhsTable {
    const void *in[kMaxStationaryRhs];
    void *out[kMaxStationaryRhs];
    int n;
};
__host__ __device__ constexpr bool is_column_order(int order) { return order == kOrderColumn || order == kOrderPatch; }

struct TileMap {
    int order;
    int block;            // sites per tile = threads per work-group
    int V;
    int slice;            // sites per T-slice
    int tiles_per_range;  // kOrderTSweep / kOrderColumn: tiles per (slice, XCD) range
    int tchunk;           // kOrderColumn / kOrderPatch: sites per lane along T
    int ntiles;           // tile slots holding sites
    int nslots;           // ntiles rounded up to a multiple of 8
    int patches;          // kOrderPatch: patches per T-slice
    int npx, npy, pz;     // kOrderPatch: patches along X and Y, patch extent in Z
    int nt, nz;           // kOrderZPlanes / kOrderZGroups: lattice extents in T and Z
    int zw;               // kOrderZGroups: z-planes per work-group (block / 64)
    int xyb;              // kOrderZGroups: tiles per (y, x) block; the T-planes of a block run before the next block
    int plane_tiles;      // kOrderZPlanes: tiles per (t, z) plane
};

TileMap make_tilemap(const Geom &g, int order, int block, int tchunk);

// One launch configuration of the stencil.
struct LaunchCfg {
    int order, block, tchunk, nr;
    int persistent = 0;  // 1: a grid of the co-resident work-groups, each striding through the items
};

// Autotuned configurations, keyed by lattice, precision, right-hand-side
// bucket, link format and clover format (see tune.hip); returns false when
// none is stored.
bool tuned_cfg(const Geom &g, int prec, int nrhs, int rows, int compact, LaunchCfg &out);

// Process-wide launch parameters (set through dirac_tune_set).
struct Tuning {
    int block = 256;             // threads per work-group: 64, 128, 192 or 256
    int order = kOrderTSweep;    // tile order
    int tchunk = 4;              // kOrderColumn / kOrderPatch: T sites per lane
    int persistent_blocks = 0;   // cap on the persistent grid (0: all co-resident work-groups)
    int nr[3] = {2, 2, 2};       // register block size per precision (1, 2 or 4)
    bool explicit_launch = false;  // set by dirac_tune_set: use these values, ignore autotuned ones
};

// The process-wide parameters are guarded by tuning_mutex(): launches read a
// consistent copy (tuning_snapshot), dirac_tune_set changes them under the
// lock through tuning_unlocked().
std::mutex &tuning_mutex();
Tuning &tuning_unlocked();
Tuning tuning_snapshot();

hipError_t dslash_launch_batches(const dirac_batch *batches, int nbatch, int prec, bool dagger, const OpData &d,
                                 const Geom &g, int apbc, bool persistent, hipStream_t st);
// same, with an explicit launch configuration (the autotuner's timing runs)
hipError_t dslash_launch_cfg(const dirac_batch *batches, int nbatch, int prec, bool dagger, const OpData &d,
                             const Geom &g, int apbc, bool persistent, const LaunchCfg &cfg, hipStream_t st);

}  // namespace wd
