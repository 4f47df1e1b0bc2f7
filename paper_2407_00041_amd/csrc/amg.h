// Two-level aggregation multigrid (internal declarations).
#pragma once

#include "common.h"
#include "sap.h"

namespace wd {

constexpr int kAmgMaxTv = 32;       // test vectors (2N <= 64 coarse unknowns per coarse site: one wavefront)
constexpr int kAmgThreads = 256;    // work-group of the per-aggregate kernels
constexpr int kAmgChunk = 8;        // test vectors per pass of the per-aggregate reductions

// Coarse-lattice geometry of an aggregation.
struct AmgGeom {
    int a[4];      // aggregate extents T, Z, Y, X
    int nc[4];     // coarse extents
    int cstr[4];   // coarse site strides
    int na;        // sites per aggregate
    int Vc;        // coarse sites
    int N;         // test vectors
};

// x = M r for one right-hand side (the two-level preconditioner), r scaled by rscale first; x and r native FP64,
// distinct.  Blocking (the coarse GMRES reads its Hessenberg columns on the host).
int amg_precond_one(const dirac_amg *amg, double2 *x, const double2 *r, double rscale, hipStream_t st);

}  // namespace wd

struct dirac_amg {
    const dirac_op *op = nullptr;
    int device = 0;             // the operator's device (destroy does not read op)
    amg_params p{};
    wd::AmgGeom ag{};
    wd::SapGeom sg{};
    // device buffers (owned; one allocation carved into pieces)
    void *mem = nullptr;
    double2 *test = nullptr;    // N native FP64 fields: the current test vectors
    void *P = nullptr;          // [Vc][N][12][na] double2 or float2 (p.prec): column (a, s, k) on the
                                // components 6s..6s+5 of a's sites
    double2 *Dc = nullptr;      // [Vc][5][2N][2N]: self block, then the blocks to the +T, +Z, +Y, +X neighbours
    // preconditioner workspace (one right-hand side)
    double2 *cb = nullptr;      // coarse basis, coarse_restart + 1 vectors
    double2 *crhs = nullptr, *csol = nullptr;          // coarse right-hand side and solution
    double2 *f1 = nullptr, *f2 = nullptr, *fsap = nullptr;  // fine temporaries of M, SAP workspace
    double2 *f3 = nullptr;                                  // M v of the setup passes
    double2 *partial = nullptr, *scal = nullptr;             // reduction partials, device scalars
    int *flag = nullptr;                                     // device status word of the setup kernels
    double2 *pinned = nullptr;                               // host staging of the coarse Hessenberg columns
    size_t pinned_n = 0;
    long long coarse_iters = 0;                              // D_c applications (all coarse solves so far)
    long long coarse_solves = 0;
};
