// Schwarz alternating procedure on lattice blocks (internal declarations).
#pragma once

#include "common.h"

namespace wd {

// Blocking of the lattice for SAP (checked by sap_geometry).
struct SapGeom {
    int b[4];      // block extents T, Z, Y, X
    int nb[4];     // blocks per direction (each even or 1)
    int span[4];   // 1 where one block spans the direction (its hops there stay inside, periodically)
    int lstr[4];   // strides of the block-local site index
    int bvol;      // sites per block (<= 256)
    int nblocks;   // blocks in the lattice
    int pair_dir;  // a direction with an even block count (colour pairs), -1 when there is a single block
};

int sap_geometry(const dirac_op *op, const sap_params *p, SapGeom &sg);
// device workspace of dirac_sap for nrhs right-hand sides (additive cycles > 1 alternate between two fields)
size_t sap_workspace(const dirac_op *op, const sap_params *p, int nrhs);
// x = SAP(bscale b) from x = 0 (native FP64 fields, nrhs consecutive right-hand sides); work: sap_workspace bytes
hipError_t sap_apply(const dirac_op *op, const sap_params &p, const SapGeom &sg, double2 *x, const double2 *b,
                     int nrhs, double2 *work, double bscale, hipStream_t st);

}  // namespace wd
