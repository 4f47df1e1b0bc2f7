// C ABI of the library: operator handle, applies, layout conversion.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "common.h"
#include "dslash.h"
#include "schur.h"

namespace wd {

hipError_t pack_launch(void *nat, const double *can, int nrhs, int prec, int V, hipStream_t st);
hipError_t unpack_launch(double *can, const void *nat, int nrhs, int prec, int V, hipStream_t st);
hipError_t clover_build_launch(double *out, const double *links, const Geom &g, hipStream_t st);
hipError_t operator_to_native(dirac_op *op, const double *links_can_dev, const double *clover_can_dev,
                              hipStream_t st);
hipError_t su3_deviation(const double *links_can_dev, int V, double *out, hipStream_t st);
hipError_t clover_structure_deviation(const double *clover_can_dev, int V, double *out, hipStream_t st);
hipError_t clover_inverse_to_native(dirac_op *op, const double *inv_can_dev, hipStream_t st);
hipError_t nonfinite_any(const double *dev, size_t n, bool *out, hipStream_t st);
hipError_t force_links_layout(double *dst, const double *canon, int V, hipStream_t st);
size_t force_links_bytes(int V);

static thread_local std::string g_err;
constexpr double kSu3Tol = 1e-12;  // largest |U U^H - 1|, |det U - 1| accepted for two-row storage
constexpr double kCloverTol = 1e-10;  // largest |C_00 + C_11| / max(1, |C|) accepted for compact clover storage

void set_error(const std::string &msg) { g_err = msg; }

// WDIRAC_LOG: 0 (default) silent, 1 every failing call's status and message on stderr, 2 also solver and setup
// progress
int log_level() {
    static const int level = [] {
        const char *e = std::getenv("WDIRAC_LOG");
        return e ? std::atoi(e) : 0;
    }();
    return level;
}

int fail(int code, const std::string &msg) {
    g_err = msg;
    if (log_level() >= 1) std::fprintf(stderr, "[wdirac] status %d: %s\n", code, msg.c_str());
    return code;
}

Geom make_geom(const int dims[4]) {
    Geom g;
    long long V = 1;
    for (int k = 0; k < 4; k++) {
        g.n[k] = dims[k];
        V *= dims[k];
    }
    g.V = (int)V;
    g.stride[3] = 1;
    g.stride[2] = dims[3];
    g.stride[1] = dims[3] * dims[2];
    g.stride[0] = dims[3] * dims[2] * dims[1];
    return g;
}

static bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
    return x < y + nb && y < x + na;
}

int check_apply(const dirac_op *op, const void *out, const void *in, int nrhs, int prec) {
    if (!op) return fail(WDIRAC_EINVAL, "null operator");
    if (!out || !in) return fail(WDIRAC_EINVAL, "null field pointer");
    if (nrhs < 1) return fail(WDIRAC_EINVAL, "nrhs must be >= 1");
    if (prec != WDIRAC_F64 && prec != WDIRAC_F32 && prec != WDIRAC_F16S)
        return fail(WDIRAC_EINVAL, "unknown precision " + std::to_string(prec));
    if (!op->data(prec).links)
        return fail(WDIRAC_EUNSUPPORTED, "precision " + std::to_string(prec) + " not materialised at create");
    size_t n = field_rhs_bytes(prec, op->g.V) * (size_t)nrhs;
    if (overlap(out, n, in, n)) return fail(WDIRAC_EINVAL, "out overlaps in");
    if ((reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(in)) & 15)
        return fail(WDIRAC_EINVAL, "field pointers must be 16-byte aligned");
    return WDIRAC_OK;
}

}  // namespace wd

using namespace wd;

extern "C" {

const char *dirac_last_error(void) { return g_err.c_str(); }

const char *dirac_version(void) { return "wdirac 0.1 (gfx950)"; }

long long dirac_volume(const dirac_op *op) { return op ? op->g.V : 0; }

size_t dirac_field_bytes(const dirac_op *op, int prec, int nrhs) {
    if (!op || nrhs < 0) return 0;
    return field_rhs_bytes(prec, op->g.V) * (size_t)nrhs;
}

int dirac_destroy(dirac_op *op) {
    if (!op) return WDIRAC_OK;
    void *bufs[] = {op->links64, op->clover64, op->links32, op->clover32, op->links16, op->clover16,
                    op->links_force, op->cinv64, op->cinv32, op->cinv16};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    delete op;
    return WDIRAC_OK;
}

int dirac_create(dirac_op **out, const int dims[4], const double *links, const double *clover, double m0,
                 double csw, unsigned flags) {
    if (!out) return fail(WDIRAC_EINVAL, "null handle pointer");
    *out = nullptr;
    if (!dims || !links) return fail(WDIRAC_EINVAL, "null dims or links");
    long long V = 1;
    for (int k = 0; k < 4; k++) {
        if (dims[k] < 2) return fail(WDIRAC_EINVAL, "every lattice extent must be >= 2");
        V *= dims[k];
    }
    // native offsets are 32-bit: 36 link entries per site must stay addressable
    if (V * 36 >= (1LL << 31)) return fail(WDIRAC_EINVAL, "lattice too large (V*36 >= 2^31)");
    if ((flags & WDIRAC_EVEN_ODD) && (dims[0] % 2 || dims[1] % 2 || dims[2] % 2 || dims[3] % 2))
        return fail(WDIRAC_EINVAL, "WDIRAC_EVEN_ODD needs every lattice extent even");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(WDIRAC_EUNSUPPORTED, "no HIP device");
    dirac_op *op = new dirac_op();
    op->g = make_geom(dims);
    op->m0 = m0;
    op->csw = csw;
    op->flags = flags;
    (void)hipGetDevice(&op->device);
    op->link_rows = (flags & WDIRAC_COMPRESS_LINKS) ? 2 : 3;
    op->clover_compact = (flags & WDIRAC_COMPRESS_CLOVER) != 0;
    const size_t lr = (size_t)op->link_rows * 3;  // stored complex entries per link
    const size_t cr = op->clover_compact ? 56 : 72;  // stored reals per site of the clover
    const size_t nl = (size_t)V * 36 * 16, nc = (size_t)V * 42 * 16;
    double *lc = nullptr, *cc = nullptr, *ic = nullptr;
    int *bad = nullptr;
    int rc = WDIRAC_OK;
    auto alloc = [&](void **p, size_t n) -> bool {
        if (hipMalloc(p, n) != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(WDIRAC_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
            return false;
        }
        return true;
    };
    hipStream_t st = nullptr;
    do {
        const size_t Vt = (size_t)op_sites(V);  // operator data are site-tiled (op_idx)
        if (!alloc((void **)&op->links64, Vt * 4 * lr * 16) || !alloc((void **)&op->clover64, Vt * cr * 8))
            break;
        if ((flags & WDIRAC_WITH_F32) && (!alloc((void **)&op->links32, Vt * 4 * lr * 8) ||
                                          !alloc((void **)&op->clover32, Vt * cr * 4)))
            break;
        if ((flags & WDIRAC_WITH_F16) && (!alloc((void **)&op->links16, Vt * 4 * lr * 4) ||
                                          !alloc((void **)&op->clover16, Vt * cr * 2)))
            break;
        if (flags & WDIRAC_EVEN_ODD) {
            if (!alloc((void **)&op->cinv64, Vt * 72 * 8) || !alloc((void **)&ic, nc) ||
                !alloc((void **)&bad, sizeof(int)))
                break;
            if ((flags & WDIRAC_WITH_F32) && !alloc((void **)&op->cinv32, Vt * 72 * 4)) break;
            if ((flags & WDIRAC_WITH_F16) && !alloc((void **)&op->cinv16, Vt * 72 * 2)) break;
        }
        // the canonical links (lc) serve the set-up kernels only; the force keeps its own component-major copy
        if (!alloc((void **)&op->links_force, force_links_bytes((int)V)) || !alloc((void **)&lc, nl) ||
            !alloc((void **)&cc, nc))
            break;
        if (hipMemcpy(lc, links, nl, hipMemcpyHostToDevice) != hipSuccess) {
            rc = fail(WDIRAC_EHIP, "copy of links to the device failed");
            break;
        }
        {
            bool nf = false;
            if (nonfinite_any(lc, nl / sizeof(double), &nf, st) != hipSuccess) {
                rc = fail(WDIRAC_EHIP, "finiteness check of the links failed to run");
                break;
            }
            if (nf) {
                rc = fail(WDIRAC_EINVAL, "the links contain a NaN or Inf entry");
                break;
            }
        }
        if (op->link_rows == 2) {
            double dev = 0;
            if (su3_deviation(lc, (int)V, &dev, st) != hipSuccess) {
                rc = fail(WDIRAC_EHIP, "SU(3) check failed to run");
                break;
            }
            if (!(dev <= kSu3Tol)) {
                rc = fail(WDIRAC_EINVAL, "two-row link storage needs SU(3) links; largest deviation " +
                                             std::to_string(dev) + " exceeds 1e-12");
                break;
            }
        }
        if (clover) {
            if (hipMemcpy(cc, clover, nc, hipMemcpyHostToDevice) != hipSuccess) {
                rc = fail(WDIRAC_EHIP, "copy of clover to the device failed");
                break;
            }
            bool nf = false;
            if (nonfinite_any(cc, nc / sizeof(double), &nf, st) != hipSuccess) {
                rc = fail(WDIRAC_EHIP, "finiteness check of the clover failed to run");
                break;
            }
            if (nf) {
                rc = fail(WDIRAC_EINVAL, "the clover term contains a NaN or Inf entry");
                break;
            }
        } else if (csw != 0.0) {
            op->clover_from_links = true;
            if (clover_build_launch(cc, lc, op->g, st) != hipSuccess) {
                rc = fail(WDIRAC_EHIP, "clover build launch failed");
                break;
            }
        } else if (hipMemsetAsync(cc, 0, nc, st) != hipSuccess) {
            rc = fail(WDIRAC_EHIP, "memset failed");
            break;
        }
        if (op->clover_compact) {
            double dev = 0;
            if (clover_structure_deviation(cc, (int)V, &dev, st) != hipSuccess) {
                rc = fail(WDIRAC_EHIP, "clover structure check failed to run");
                break;
            }
            if (!(dev <= kCloverTol)) {
                rc = fail(WDIRAC_EINVAL, "compact clover storage needs C_00 + C_11 = 0 in each chirality block; "
                                         "largest relative deviation " + std::to_string(dev) + " exceeds 1e-10");
                break;
            }
        }
        if (operator_to_native(op, lc, cc, st) != hipSuccess ||
            force_links_layout(op->links_force, lc, (int)V, st) != hipSuccess) {
            rc = fail(WDIRAC_EHIP, "layout conversion launch failed");
            break;
        }
        if (flags & WDIRAC_EVEN_ODD) {
            int found = 0;
            if (hipMemsetAsync(bad, 0, sizeof(int), st) != hipSuccess ||
                clover_invert_launch(reinterpret_cast<double2 *>(ic), reinterpret_cast<const double2 *>(cc), (int)V,
                                     4.0 + m0, csw, bad, st) != hipSuccess ||
                clover_inverse_to_native(op, ic, st) != hipSuccess ||
                hipMemcpy(&found, bad, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
                rc = fail(WDIRAC_EHIP, "inverse of the site-local term failed to run");
                break;
            }
            if (found) {
                rc = fail(WDIRAC_EINVAL, "a chirality block of A(x) = (4 + m0) + csw C(x) is singular");
                break;
            }
        }
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            rc = fail(WDIRAC_EHIP, std::string("operator setup failed: ") + hipGetErrorString(e));
            break;
        }
    } while (false);
    if (lc) (void)hipFree(lc);
    if (cc) (void)hipFree(cc);
    if (ic) (void)hipFree(ic);
    if (bad) (void)hipFree(bad);
    // the static scratch of the allocation-free even-odd entry point, resolved once on this (current) device
    if (rc == WDIRAC_OK && (flags & WDIRAC_EVEN_ODD)) rc = schur_scratch_init(op->device);
    if (rc != WDIRAC_OK) {
        dirac_destroy(op);
        return rc;
    }
    *out = op;
    return WDIRAC_OK;
}

static int apply_common(const dirac_op *op, void *out, const void *in, int nrhs, int prec, bool dagger,
                        void *stream) {
    int rc = check_apply(op, out, in, nrhs, prec);
    if (rc) return rc;
    dirac_batch b{out, in, nrhs};
    hipError_t e = dslash_launch_batches(&b, 1, prec, dagger, op->data(prec), op->g,
                                         (op->flags & WDIRAC_ANTIPERIODIC_T) ? 1 : 0, false, (hipStream_t)stream);
    if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("dslash launch: ") + hipGetErrorString(e));
    return WDIRAC_OK;
}

int dirac_apply_batched(const dirac_op *op, const dirac_batch *batches, int nbatch, int prec, int dagger,
                        void *stream) {
    if (!op || !batches || nbatch < 1) return fail(WDIRAC_EINVAL, "bad batched-apply arguments");
    for (int b = 0; b < nbatch; b++) {
        int rc = check_apply(op, batches[b].out, batches[b].in, batches[b].nrhs, prec);
        if (rc) return rc;
        const size_t n = field_rhs_bytes(prec, op->g.V) * (size_t)batches[b].nrhs;
        for (int c = 0; c < nbatch; c++) {
            if (c == b) continue;
            const size_t m = field_rhs_bytes(prec, op->g.V) * (size_t)batches[c].nrhs;
            if (overlap(batches[b].out, n, batches[c].out, m) || overlap(batches[b].out, n, batches[c].in, m))
                return fail(WDIRAC_EINVAL, "an output of batch " + std::to_string(b) + " overlaps batch " +
                                               std::to_string(c));
        }
    }
    hipError_t e = dslash_launch_batches(batches, nbatch, prec, dagger != 0, op->data(prec), op->g,
                                         (op->flags & WDIRAC_ANTIPERIODIC_T) ? 1 : 0, true, (hipStream_t)stream);
    if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("batched dslash launch: ") + hipGetErrorString(e));
    return WDIRAC_OK;
}

int dirac_tune_set(const char *key, int value) {
    if (!key) return fail(WDIRAC_EINVAL, "null key");
    std::lock_guard<std::mutex> lk(tuning_mutex());
    Tuning &t = tuning_unlocked();
    std::string k(key);
    if (k == "explicit") {
        t.explicit_launch = value != 0;
        return WDIRAC_OK;
    }
    if (k != "persistent_blocks") t.explicit_launch = true;  // a launch knob set by hand wins over tuned ones
    if (k == "block") {
        if (value < 64 || value > 256 || value % 64) return fail(WDIRAC_EINVAL, "block must be 64, 128, 192 or 256");
        t.block = value;
    } else if (k == "order") {
        if (value < 0 || value > 6) return fail(WDIRAC_EINVAL, "order must be 0 .. 6");
        t.order = value;
    } else if (k == "tchunk") {
        if (value < 1 || value > 4096) return fail(WDIRAC_EINVAL, "tchunk must be in [1, 4096]");
        t.tchunk = value;
    } else if (k == "persistent_blocks") {
        if (value != 0 && value < 8) return fail(WDIRAC_EINVAL, "persistent_blocks must be 0 or >= 8");
        t.persistent_blocks = value;
    } else if (k == "nr_f64" || k == "nr_f32" || k == "nr_f16s") {
        if (value != 1 && value != 2 && value != 4) return fail(WDIRAC_EINVAL, "register block must be 1, 2 or 4");
        t.nr[k == "nr_f64" ? 0 : k == "nr_f32" ? 1 : 2] = value;
    } else {
        return fail(WDIRAC_EINVAL, "unknown tuning key " + k);
    }
    return WDIRAC_OK;
}

int dirac_tune_get(const char *key, int *value) {
    if (!key || !value) return fail(WDIRAC_EINVAL, "null argument");
    const Tuning t = tuning_snapshot();
    std::string k(key);
    if (k == "block") *value = t.block;
    else if (k == "explicit") *value = t.explicit_launch ? 1 : 0;
    else if (k == "order") *value = t.order;
    else if (k == "tchunk") *value = t.tchunk;
    else if (k == "persistent_blocks") *value = t.persistent_blocks;
    else if (k == "nr_f64") *value = t.nr[0];
    else if (k == "nr_f32") *value = t.nr[1];
    else if (k == "nr_f16s") *value = t.nr[2];
    else return fail(WDIRAC_EINVAL, "unknown tuning key " + k);
    return WDIRAC_OK;
}

int dirac_apply(const dirac_op *op, void *out, const void *in, int nrhs, int prec, void *stream) {
    return apply_common(op, out, in, nrhs, prec, false, stream);
}

int dirac_apply_adjoint(const dirac_op *op, void *out, const void *in, int nrhs, int prec, void *stream) {
    return apply_common(op, out, in, nrhs, prec, true, stream);
}

int dirac_pack(const dirac_op *op, void *native, const double *canonical, int nrhs, int prec, void *stream) {
    if (!op || !native || !canonical || nrhs < 1) return fail(WDIRAC_EINVAL, "bad pack arguments");
    if (prec != WDIRAC_F64 && prec != WDIRAC_F32 && prec != WDIRAC_F16S) return fail(WDIRAC_EINVAL, "unknown precision");
    if (overlap(native, field_rhs_bytes(prec, op->g.V) * nrhs, canonical, (size_t)op->g.V * 192 * nrhs))
        return fail(WDIRAC_EINVAL, "pack buffers overlap");
    hipError_t e = pack_launch(native, canonical, nrhs, prec, op->g.V, (hipStream_t)stream);
    if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("pack launch: ") + hipGetErrorString(e));
    return WDIRAC_OK;
}

int dirac_unpack(const dirac_op *op, double *canonical, const void *native, int nrhs, int prec, void *stream) {
    if (!op || !native || !canonical || nrhs < 1) return fail(WDIRAC_EINVAL, "bad unpack arguments");
    if (prec != WDIRAC_F64 && prec != WDIRAC_F32 && prec != WDIRAC_F16S) return fail(WDIRAC_EINVAL, "unknown precision");
    if (overlap(native, field_rhs_bytes(prec, op->g.V) * nrhs, canonical, (size_t)op->g.V * 192 * nrhs))
        return fail(WDIRAC_EINVAL, "unpack buffers overlap");
    hipError_t e = unpack_launch(canonical, native, nrhs, prec, op->g.V, (hipStream_t)stream);
    if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("unpack launch: ") + hipGetErrorString(e));
    return WDIRAC_OK;
}

int dirac_clover_term(const int dims[4], const double *links_dev, double *clover_dev, void *stream) {
    if (!dims || !links_dev || !clover_dev) return fail(WDIRAC_EINVAL, "null argument");
    long long V = 1;
    for (int k = 0; k < 4; k++) {
        if (dims[k] < 2) return fail(WDIRAC_EINVAL, "every lattice extent must be >= 2");
        V *= dims[k];
    }
    if (V * 42 >= (1LL << 31)) return fail(WDIRAC_EINVAL, "lattice too large");
    Geom g = make_geom(dims);
    hipError_t e = clover_build_launch(clover_dev, links_dev, g, (hipStream_t)stream);
    if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("clover launch: ") + hipGetErrorString(e));
    return WDIRAC_OK;
}

}  // extern "C"
