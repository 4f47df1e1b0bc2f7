// FGMRES (Algorithm 2, Sec. 1.2) on the device, for several right-hand sides.
//
// Every right-hand side runs its own restarted FGMRES: its own Krylov basis,
// Hessenberg matrix and termination test.  The right-hand sides advance in
// lockstep only so that their operator applications (lines 4 and 9 of the
// algorithm) go out as one batched stencil launch.
//
// Steps per right-hand side, in the algorithm's order:
//   restart   r = b - D x (FP64 operator), beta = |r|, v_1 = r / beta
//   step j    z_j = M_j^{-1} v_j;  w = D z_j;
//             h_ij = <w, v_i> and w -= h_ij v_i for i <= j (classical
//             Gram-Schmidt: all inner products in one pass over the basis,
//             then one update pass; this gives the same h and w as the
//             paper's modified loop in exact arithmetic);
//             h_{j+1,j} = |w|, v_{j+1} = w / h_{j+1,j}
//   cycle end y = argmin |beta e_1 - H y| (Givens rotations, applied as the
//             columns arrive, give the residual estimate |g_{j+1}| after
//             every step), x += Z y
// Termination as in Sec. 1.2: |b - D x| < tol |b - D x_0| at a restart, or
// maxit operator applications; a cycle also ends early once the estimate
// is below the target, and at |h_{j+1,j}| < tol/10 (near breakdown).
//
// Preconditioner M_j^{-1}: the identity (FGMRES_F64), or for the mixed
// modes an inner GMRES solve of D z = v_j with the FP32 or FP16S operator,
// stopped at the relative residual inner_tol or after inner_maxit
// applications.  The inner Krylov basis is stored in the inner operator's own
// native layout (FP32, or FP16 with per-site scales) and all its inner
// products accumulate in FP64.  Inner basis vectors are normalised lazily:
// the operator writes D W_k straight into the next basis slot, which is
// orthogonalised in place and kept unnormalised; the host tracks the stored
// norms c_k (W_k = c_k v_k) and folds them into the Hessenberg entries, the
// update coefficients and the final combination, so no separate scaling or
// conversion pass runs per inner step.  The outer residual,
// orthogonalisation and update stay FP64, so the outer loop is an iterative
// refinement of the low-precision solves.
//
// Host work per Arnoldi step: one stream synchronisation, to read the new
// Hessenberg column (a few complex numbers) and decide how to continue.
#include <chrono>
#include <complex>
#include <string>
#include <vector>

#include "blas.h"
#include "dslash.h"

namespace wd {

int check_apply(const dirac_op *op, const void *out, const void *in, int nrhs, int prec);

using zc = std::complex<double>;

namespace {

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

struct Layout {
    size_t f64, f32, f16, scal;  // bytes of one field / scalar block
    size_t per_rhs;
};

int inner_prec(int mode) { return mode == FGMRES_MIXED_F32 ? WDIRAC_F32 : WDIRAC_F16S; }

// entries of each per-RHS scalar array (Hessenberg column, coefficients)
int kmax_of(const fgmres_params *p) {
    const int m = p->restart, mi = p->mode == FGMRES_F64 ? 0 : p->inner_restart;
    return (m > mi ? m : mi) + 2;
}

Layout layout(const dirac_op *op, const fgmres_params *p) {
    Layout L;
    const long long V = op->g.V;
    L.f64 = align256(field_rhs_bytes(WDIRAC_F64, V));
    L.f32 = align256(field_rhs_bytes(WDIRAC_F32, V));
    L.f16 = align256(field_rhs_bytes(WDIRAC_F16S, V));
    const int m = p->restart, mi = p->mode == FGMRES_F64 ? 0 : p->inner_restart;
    const int kmax = kmax_of(p);
    L.scal = align256(sizeof(double2) * ((size_t)kRedBlocks * (kGS + 1) + 3 * (size_t)kmax + 8));
    L.per_rhs = (size_t)(m + 2) * L.f64 + L.scal;  // V[0..m], w
    if (p->mode != FGMRES_F64) {
        L.per_rhs += (size_t)m * L.f64;                                          // Z[0..m)
        L.per_rhs += (size_t)(mi + 1) * (p->mode == FGMRES_MIXED_F32 ? L.f32 : L.f16);  // inner W[0..mi]
    }
    return L;
}

// Hessenberg least-squares state of one (F)GMRES cycle, Givens-updated
struct Arnoldi {
    int m = 0, j = 0;
    std::vector<zc> H;  // (m+1) x m, column-major, rotated in place
    std::vector<zc> sn;
    std::vector<double> cs;
    std::vector<zc> g;
    void reset(int m_, double beta) {
        m = m_;
        j = 0;
        H.assign((size_t)(m + 1) * m, zc(0));
        sn.assign(m, zc(0));
        cs.assign(m, 0.0);
        g.assign(m + 1, zc(0));
        g[0] = beta;
    }
    zc &h(int i, int k) { return H[(size_t)k * (m + 1) + i]; }
    // add column j (entries 0..j+1); returns |g_{j+1}|
    double add_column(const zc *col) {
        for (int i = 0; i <= j + 1; i++) h(i, j) = col[i];
        for (int i = 0; i < j; i++) {
            zc a = h(i, j), b = h(i + 1, j);
            h(i, j) = cs[i] * a + sn[i] * b;
            h(i + 1, j) = -std::conj(sn[i]) * a + cs[i] * b;
        }
        zc a = h(j, j), b = h(j + 1, j);
        double r = std::sqrt(std::norm(a) + std::norm(b));
        if (r == 0.0) {
            cs[j] = 1.0;
            sn[j] = 0.0;
        } else if (std::abs(a) == 0.0) {
            cs[j] = 0.0;
            sn[j] = std::conj(b) / std::abs(b);
        } else {
            cs[j] = std::abs(a) / r;
            sn[j] = (a / std::abs(a)) * std::conj(b) / r;
        }
        h(j, j) = cs[j] * a + sn[j] * b;
        h(j + 1, j) = 0.0;
        g[j + 1] = -std::conj(sn[j]) * g[j];
        g[j] = cs[j] * g[j];
        j++;
        return std::abs(g[j]);
    }
    // y solving the leading j x j triangular system R y = g
    std::vector<zc> solve() const {
        std::vector<zc> y(j);
        for (int i = j - 1; i >= 0; i--) {
            zc s = g[i];
            for (int k = i + 1; k < j; k++) s -= H[(size_t)k * (m + 1) + i] * y[k];
            const zc d = H[(size_t)i * (m + 1) + i];
            y[i] = d == zc(0) ? zc(0) : s / d;
        }
        return y;
    }
};

enum class Phase { Residual, Arnoldi, Done };

struct Rhs {
    // device
    double2 *x = nullptr;
    const double2 *b = nullptr;
    std::vector<void *> V, Z;  // outer basis (F64), preconditioned vectors (F64)
    double2 *w = nullptr;
    std::vector<void *> Vi;    // inner basis, inner operator precision, unnormalised
    std::vector<double> ic;    // stored norms of the inner basis vectors (host)
    double2 *partial = nullptr, *hcol = nullptr, *coef = nullptr, *hcol2 = nullptr, *nrm = nullptr;
    // host
    Phase phase = Phase::Residual;
    Arnoldi outer, inner;
    double r0norm = -1, relres = 1;
    bool breakdown = false, converged = false, inner_done = false;
    long long applies = 0, inner_applies = 0, restarts = 0;
    std::vector<double> hist;
};

struct Ctx {
    const dirac_op *op;
    const fgmres_params *p;
    hipStream_t st;
    long long N;  // complex numbers per field
    int V;
    int apbc;
    double2 *pinned;  // host staging for scalar reads (hipHostMalloc)
    size_t pinned_n;
};

hipError_t apply_many(const Ctx &c, int prec, const std::vector<dirac_batch> &b) {
    if (b.empty()) return hipSuccess;
    return dslash_launch_batches(b.data(), (int)b.size(), prec, false, c.op->data(prec), c.op->g, c.apbc, false, c.st);
}

#define WD_TRY(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(WDIRAC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Read device scalars (pointer, count) into the pinned staging buffer with
// stream-ordered copies and ONE stream synchronisation.
int fetch(const Ctx &c, const std::vector<std::pair<const double2 *, int>> &src, std::vector<std::vector<zc>> &out) {
    out.assign(src.size(), {});
    size_t off = 0;
    for (size_t k = 0; k < src.size(); k++) {
        if (off + src[k].second > c.pinned_n) return fail(WDIRAC_EINVAL, "internal: staging buffer too small");
        WD_TRY(hipMemcpyAsync(c.pinned + off, src[k].first, src[k].second * sizeof(double2), hipMemcpyDeviceToHost,
                              c.st));
        off += src[k].second;
    }
    WD_TRY(hipStreamSynchronize(c.st));
    off = 0;
    for (size_t k = 0; k < src.size(); k++) {
        for (int i = 0; i < src[k].second; i++) out[k].push_back(zc(c.pinned[off + i].x, c.pinned[off + i].y));
        off += src[k].second;
    }
    return WDIRAC_OK;
}

std::vector<double2> to_d2(const std::vector<zc> &v) {
    std::vector<double2> t(v.size());
    for (size_t i = 0; i < v.size(); i++) t[i] = make_double2(v[i].real(), v[i].imag());
    return t;
}

// Inner GMRES on the low-precision operator for every listed right-hand
// side: z = M^{-1} v with v = V[j] (unit norm) and z = Z[j].
int inner_solve(const Ctx &c, std::vector<Rhs *> &list) {
    const fgmres_params &p = *c.p;
    const int prec = inner_prec(p.mode);
    const int mi = p.inner_restart;
    const int maxit = p.inner_maxit < mi ? p.inner_maxit : mi;
    for (Rhs *r : list) {
        WD_TRY(site_scale(WDIRAC_F64, prec, r->V[r->outer.j], r->Vi[0], 1.0, c.V, c.st));
        r->inner.reset(mi, 1.0);
        r->ic.assign(1, 1.0);
        r->inner_done = false;
    }
    std::vector<Rhs *> act = list;
    std::vector<double> mult;
    while (!act.empty()) {
        // W_{k+1} = D W_k for every active right-hand side, one batched launch
        std::vector<dirac_batch> b;
        for (Rhs *r : act) b.push_back({r->Vi[r->inner.j + 1], r->Vi[r->inner.j], 1});
        WD_TRY(apply_many(c, prec, b));
        for (Rhs *r : act) {
            const int k = r->inner.j;
            r->inner_applies++;
            // dots d_i = W_i^H W_{k+1} = c_i c_k h_ik; then W_{k+1} -= sum_i d_i / c_i^2 W_i
            WD_TRY(site_mdot(prec, r->Vi.data(), k + 1, r->Vi[k + 1], c.V, r->partial, r->hcol, c.st));
            mult.resize(k + 1);
            for (int i = 0; i <= k; i++) mult[i] = 1.0 / (r->ic[i] * r->ic[i]);
            WD_TRY(site_axpy(prec, r->Vi.data(), k + 1, r->hcol, mult.data(), r->Vi[k + 1], c.V, r->partial,
                             r->hcol + k + 1, c.st));
        }
        std::vector<std::pair<const double2 *, int>> src;
        for (Rhs *r : act) src.emplace_back(r->hcol, r->inner.j + 2);
        std::vector<std::vector<zc>> h;
        int rc = fetch(c, src, h);
        if (rc) return rc;
        std::vector<Rhs *> next;
        for (size_t q = 0; q < act.size(); q++) {
            Rhs *r = act[q];
            const int k = r->inner.j;
            const double ck = r->ic[k];
            std::vector<zc> col(k + 2);
            for (int i = 0; i <= k; i++) col[i] = h[q][i] / (r->ic[i] * ck);
            const double nrm = std::sqrt(std::max(h[q][k + 1].real(), 0.0));  // |W_{k+1}| = c_k h_{k+1,k}
            const double hn = nrm / ck;
            col[k + 1] = hn;
            const double est = r->inner.add_column(col.data());
            const bool stop = est < p.inner_tol || r->inner.j >= maxit || hn == 0.0;
            if (stop) {
                r->inner_done = true;
                continue;
            }
            if (nrm > 1e-20 && nrm < 1e20) {
                r->ic.push_back(nrm);
            } else {  // keep stored magnitudes well inside the FP32 range
                WD_TRY(site_scale(prec, prec, r->Vi[k + 1], r->Vi[k + 1], 1.0 / nrm, c.V, c.st));
                r->ic.push_back(1.0);
            }
            next.push_back(r);
        }
        act.swap(next);
    }
    // z_j = sum_i y_i v_i = sum_i (y_i / c_i) W_i, accumulated in FP64
    for (Rhs *r : list) {
        std::vector<zc> y = r->inner.solve();
        for (size_t i = 0; i < y.size(); i++) y[i] /= r->ic[i];
        const std::vector<double2> yd = to_d2(y);
        WD_TRY(site_combine(prec, r->Vi.data(), (int)yd.size(), yd.data(), static_cast<double2 *>(r->Z[r->outer.j]),
                            c.V, c.st));
    }
    return WDIRAC_OK;
}

}  // namespace

size_t solver_workspace(const dirac_op *op, const fgmres_params *p, int nrhs) {
    return layout(op, p).per_rhs * (size_t)nrhs;
}

int solve(const dirac_op *op, double *x, const double *b, int nrhs, const fgmres_params *p, fgmres_stats *st,
          void *work, size_t work_bytes, hipStream_t stream) {
    const auto t0 = std::chrono::steady_clock::now();
    const Layout L = layout(op, p);
    const int kmax = kmax_of(p);
    const size_t pinned_n = (size_t)nrhs * (kmax + 2);
    double2 *pinned = nullptr;
    if (hipHostMalloc((void **)&pinned, pinned_n * sizeof(double2), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(WDIRAC_ENOMEM, "pinned staging allocation failed");
    }
    struct PinnedGuard {
        double2 *p;
        ~PinnedGuard() { (void)hipHostFree(p); }
    } guard{pinned};
    Ctx c{op, p, stream, 12LL * op->g.V, op->g.V, (op->flags & WDIRAC_ANTIPERIODIC_T) ? 1 : 0, pinned, pinned_n};
    const bool mixed = p->mode != FGMRES_F64;
    const int m = p->restart;
    // carve the workspace
    std::vector<Rhs> R(nrhs);
    char *wp = static_cast<char *>(work);
    auto take = [&](size_t n) {
        char *q = wp;
        wp += n;
        return q;
    };
    for (int k = 0; k < nrhs; k++) {
        Rhs &r = R[k];
        r.x = reinterpret_cast<double2 *>(x) + (size_t)k * c.N;
        r.b = reinterpret_cast<const double2 *>(b) + (size_t)k * c.N;
        for (int i = 0; i <= m; i++) r.V.push_back(take(L.f64));
        r.w = reinterpret_cast<double2 *>(take(L.f64));
        if (mixed) {
            for (int i = 0; i < m; i++) r.Z.push_back(take(L.f64));
            const size_t fi = p->mode == FGMRES_MIXED_F32 ? L.f32 : L.f16;
            for (int i = 0; i <= p->inner_restart; i++) r.Vi.push_back(take(fi));
        } else {
            r.Z = std::vector<void *>(r.V.begin(), r.V.begin() + m);  // M = I: z_j = v_j
        }
        char *s = take(L.scal);
        r.partial = reinterpret_cast<double2 *>(s);
        r.hcol = r.partial + (size_t)kRedBlocks * (kGS + 1);
        r.coef = r.hcol + kmax;
        r.hcol2 = r.coef + kmax;
        r.nrm = r.hcol2 + kmax;
        if (reinterpret_cast<char *>(r.nrm + 1) > s + L.scal) return fail(WDIRAC_EINVAL, "internal: scalar block overflow");
    }
    if ((size_t)(wp - static_cast<char *>(work)) > work_bytes) return fail(WDIRAC_EINVAL, "workspace too small");

    bool any = true;
    while (any) {
        // preconditioning of the right-hand sides inside a cycle
        std::vector<Rhs *> arn, res;
        for (Rhs &r : R) {
            if (r.phase == Phase::Arnoldi) arn.push_back(&r);
            if (r.phase == Phase::Residual) res.push_back(&r);
        }
        if (mixed && !arn.empty()) {
            int rc = inner_solve(c, arn);
            if (rc) return rc;
        }
        // one batched FP64 application for all of them (lines 4 and 9)
        std::vector<dirac_batch> bat;
        for (Rhs *r : res) bat.push_back({r->w, r->x, 1});
        for (Rhs *r : arn) bat.push_back({r->w, r->Z[r->outer.j], 1});
        WD_TRY(apply_many(c, WDIRAC_F64, bat));
        for (Rhs *r : res) {
            r->applies++;
            WD_TRY(residual(r->b, r->w, static_cast<double2 *>(r->V[0]), c.N, r->partial, r->nrm, c.st));
        }
        for (Rhs *r : arn) {
            r->applies++;
            const int j = r->outer.j;
            WD_TRY(mdot<double2>(r->V.data(), j + 1, r->w, c.N, r->partial, r->hcol, c.st));
            WD_TRY(axpy_multi<double2>(r->V.data(), j + 1, r->hcol, r->w, c.N, r->partial, r->hcol + j + 1, c.st));
        }
        std::vector<std::pair<const double2 *, int>> src;
        for (Rhs *r : res) src.emplace_back(r->nrm, 1);
        for (Rhs *r : arn) src.emplace_back(r->hcol, r->outer.j + 2);
        std::vector<std::vector<zc>> got;
        if (!src.empty()) {
            int rc = fetch(c, src, got);
            if (rc) return rc;
        }
        // restarts: convergence test on the true residual
        for (size_t k = 0; k < res.size(); k++) {
            Rhs &r = *res[k];
            const double beta = std::sqrt(std::max(got[k][0].real(), 0.0));
            if (r.r0norm < 0) r.r0norm = beta;
            r.relres = r.r0norm > 0 ? beta / r.r0norm : 0.0;
            if (r.r0norm == 0.0 || r.relres < p->tol) {
                r.converged = true;
                r.phase = Phase::Done;
                continue;
            }
            if (r.applies >= p->maxit || r.breakdown) {
                r.phase = Phase::Done;
                continue;
            }
            r.restarts++;
            WD_TRY((scale<double2, double2>(r.V[0], r.V[0], nullptr, false, 1.0 / beta, c.N, c.st)));
            r.outer.reset(m, beta);
            r.phase = Phase::Arnoldi;
        }
        // Arnoldi steps: Hessenberg column, Givens, continue or end the cycle
        for (size_t k = 0; k < arn.size(); k++) {
            Rhs &r = *arn[k];
            const int j = r.outer.j;
            const std::vector<zc> &hk = got[res.size() + k];
            std::vector<zc> col(j + 2);
            for (int i = 0; i <= j; i++) col[i] = hk[i];
            const double hn = std::sqrt(std::max(hk[j + 1].real(), 0.0));
            col[j + 1] = hn;
            const double est = r.outer.add_column(col.data()) / r.r0norm;
            r.hist.push_back(est);
            bool end = false;
            if (hn < p->tol / 10.0) {
                r.breakdown = true;
                end = true;
            } else if (est < p->tol || r.applies >= p->maxit || r.outer.j >= m) {
                end = true;
            }
            if (!end) {
                WD_TRY((scale<double2, double2>(r.w, r.V[r.outer.j], nullptr, false, 1.0 / hn, c.N, c.st)));
                continue;
            }
            const std::vector<double2> y = to_d2(r.outer.solve());
            WD_TRY(update<double2>(r.Z.data(), (int)y.size(), y.data(), r.x, c.N, c.st));
            r.phase = Phase::Residual;
        }
        any = false;
        for (Rhs &r : R)
            if (r.phase != Phase::Done) any = true;
    }
    WD_TRY(hipStreamSynchronize(stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool all = true;
    for (int k = 0; k < nrhs; k++) {
        Rhs &r = R[k];
        all = all && r.converged;
        if (!st) continue;
        fgmres_stats &s = st[k];
        s.applies = r.applies;
        s.inner_applies = r.inner_applies;
        s.restarts = r.restarts;
        s.converged = r.converged ? 1 : 0;
        s.breakdown = r.breakdown ? 1 : 0;
        s.true_residual = r.relres;
        s.seconds = secs;
        s.nhist = (int)std::min<size_t>(r.hist.size(), FGMRES_HIST_MAX);
        for (int i = 0; i < s.nhist; i++) s.hist[i] = r.hist[i];
    }
    return all ? WDIRAC_OK : WDIRAC_ENOTCONV;
}

}  // namespace wd

using namespace wd;

extern "C" {

static int check_params(const dirac_op *op, const fgmres_params *p) {
    if (!op || !p) return fail(WDIRAC_EINVAL, "null operator or parameters");
    if (p->restart < 1 || p->restart > 1000) return fail(WDIRAC_EINVAL, "restart must be in [1, 1000]");
    if (!(p->tol > 0.0)) return fail(WDIRAC_EINVAL, "tol must be > 0");
    if (p->maxit < 1) return fail(WDIRAC_EINVAL, "maxit must be >= 1");
    if (p->mode != FGMRES_F64 && p->mode != FGMRES_MIXED_F32 && p->mode != FGMRES_MIXED_F16S)
        return fail(WDIRAC_EINVAL, "unknown solver mode");
    if (p->mode != FGMRES_F64) {
        if (p->inner_restart < 1 || p->inner_restart > 1000) return fail(WDIRAC_EINVAL, "inner_restart in [1, 1000]");
        if (p->inner_maxit < 1) return fail(WDIRAC_EINVAL, "inner_maxit must be >= 1");
        if (!(p->inner_tol > 0.0)) return fail(WDIRAC_EINVAL, "inner_tol must be > 0");
        if (!op->data(inner_prec(p->mode)).links)
            return fail(WDIRAC_EUNSUPPORTED, "inner precision not materialised at create");
    }
    return WDIRAC_OK;
}

size_t fgmres_workspace_bytes(const dirac_op *op, const fgmres_params *p, int nrhs) {
    if (nrhs < 1 || check_params(op, p)) return 0;
    return solver_workspace(op, p, nrhs);
}

int fgmres_solve(const dirac_op *op, double *x, const double *b, int nrhs, const fgmres_params *p,
                 fgmres_stats *st, void *work, size_t work_bytes, void *stream) {
    int rc = check_params(op, p);
    if (rc) return rc;
    if (!x || !b || !work) return fail(WDIRAC_EINVAL, "null x, b or workspace");
    if (nrhs < 1) return fail(WDIRAC_EINVAL, "nrhs must be >= 1");
    rc = check_apply(op, x, b, nrhs, WDIRAC_F64);
    if (rc) return rc;
    if (work_bytes < solver_workspace(op, p, nrhs)) return fail(WDIRAC_EINVAL, "workspace too small");
    if (reinterpret_cast<uintptr_t>(work) & 255) return fail(WDIRAC_EINVAL, "workspace must be 256-byte aligned");
    return solve(op, x, b, nrhs, p, st, work, work_bytes, (hipStream_t)stream);
}

}  // extern "C"
