// Entry points whose kernels are not built yet: they report EUNSUPPORTED.
#include "common.h"

using namespace wd;

extern "C" {

int dirac_force(const dirac_op *, double *, const double *, const double *, int, int, void *) {
    return fail(WDIRAC_EUNSUPPORTED, "dirac_force: not built yet");
}

}
