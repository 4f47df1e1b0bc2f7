// Entry points whose kernels are not built yet: they report EUNSUPPORTED.
#include "common.h"

using namespace wd;

extern "C" {

size_t fgmres_workspace_bytes(const dirac_op *, const fgmres_params *, int) { return 0; }

int fgmres_solve(const dirac_op *, double *, const double *, int, const fgmres_params *, fgmres_stats *, void *,
                 size_t, void *) {
    return fail(WDIRAC_EUNSUPPORTED, "fgmres_solve: not built yet");
}

int dirac_force(const dirac_op *, double *, const double *, const double *, int, int, void *) {
    return fail(WDIRAC_EUNSUPPORTED, "dirac_force: not built yet");
}

}
