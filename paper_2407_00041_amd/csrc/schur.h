// Even-odd (red-black) kernels: parity-split fields and the reduced operator
// S = A_ee - H_eo A_oo^{-1} H_oe on the even sites (D = A + H, A the
// site-local term of Eq. (1.13) with the clover term of Eqs. (1.11)-(1.12),
// H the hopping sum, which couples only sites of opposite parity).
#pragma once

#include <vector>

#include "common.h"

namespace wd {

// A parity field lists the V/2 sites of one parity (t + z + y + x) mod 2 in
// increasing lexicographic order; with n_X even that is half-lattice index
// s >> 1 for full-lattice site s.  Native layouts as for full fields with V/2.

// One launch over the V/2 sites of parity `parity` (output parity), per RHS:
enum ParityMode : int {
    kParHopInv = 0,   // out = A^{-1} (H hop)
    kParCloverSub,    // out = A self - H hop
    kParApply,        // out = A self + H hop     ((D x)_p from x_p and x_{1-p})
    kParInvSelf,      // out = A^{-1} self
    kParSelfSub,      // out = self - H hop
    kParInvSelfSub,   // out = A^{-1} (self - H hop)
};

// `self` may equal `out` (each site reads only its own entries before
// writing them); `hop` must not overlap `out`.  dag selects H^H for
// kParHopInv and kParCloverSub (the adjoint of S).  Fields of nrhs right-hand
// sides back to back, or a list of separate ones; pairs of right-hand sides
// share each lane's loads of the links and of A or A^{-1}.
struct ParityItem {
    void *out;
    const void *self;
    const void *hop;
};
hipError_t parity_launch(int mode, int prec, bool dag, const dirac_op *op, int parity, void *out, const void *self,
                         const void *hop, int nrhs, hipStream_t st);
hipError_t parity_launch_list(int mode, int prec, bool dag, const dirac_op *op, int parity,
                              const std::vector<ParityItem> &items, hipStream_t st);
// the same from a plain array of n items (no host allocation)
hipError_t parity_launch_items(int mode, int prec, bool dag, const dirac_op *op, int parity, const ParityItem *items,
                               size_t n, hipStream_t st);

// Static device scratch of dirac_apply_schur_noalloc: resolve its address on the current device (once per device;
// called by dirac_create with the operator's device current).
int schur_scratch_init(int device);
void *schur_scratch_addr(int device);

// S x (or S^H x) for nrhs even fields: tmp (nrhs odd fields) receives A_oo^{-1} H_oe x.
hipError_t schur_apply(int prec, bool dag, const dirac_op *op, void *out, const void *in, void *tmp, int nrhs,
                       hipStream_t st);
struct SchurItem {
    void *out;
    const void *in;
    void *tmp;
};
hipError_t schur_apply_list(int prec, bool dag, const dirac_op *op, const std::vector<SchurItem> &items,
                            hipStream_t st);

// full <-> (even, odd)
hipError_t parity_split_launch(const dirac_op *op, int prec, void *even, void *odd, const void *full, int nrhs,
                               hipStream_t st);
hipError_t parity_merge_launch(const dirac_op *op, int prec, void *full, const void *even, const void *odd,
                               int nrhs, hipStream_t st);

// canonical [V][42] unit term C -> canonical packed inverse of (diag + csw C),
// chirality block by block; *bad is set to 1 where a block is (nearly) singular
hipError_t clover_invert_launch(double2 *inv_can, const double2 *can, int V, double diag, double csw, int *bad,
                                hipStream_t st);

}  // namespace wd
