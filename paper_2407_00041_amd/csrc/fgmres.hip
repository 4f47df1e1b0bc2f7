// FGMRES (Algorithm 2, Sec. 1.2) on the device, for several right-hand sides.
//
// Every right-hand side runs its own restarted FGMRES: its own Krylov basis,
// Hessenberg matrix and termination test.  The right-hand sides advance in
// lockstep only so that their operator applications (the restart residual
// and the product with the preconditioned vector) go out as one batched
// stencil launch.
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
// products accumulate in FP64.  The operator writes D W_k straight into the
// next basis slot, which is orthogonalised and normalised in place in one
// pass: the normalisation factor comes from the Pythagorean estimate
// |w|^2 - sum |h_ik|^2 (exact norms c_k of the stored vectors are measured
// in the same pass and folded into the Hessenberg entries, so the estimate
// only has to keep magnitudes near 1).  The inner cycle's Givens rotations,
// termination test and triangular solve run on the device, so a cycle needs
// no host decision: it is issued step by step with one host read of the
// active flags per step, or (params.graph) captured once per outer slot as a
// HIP graph and replayed.  The outer residual, orthogonalisation and update
// stay FP64, so the outer loop is an iterative refinement of the
// low-precision solves.

#include <algorithm>
#include <cstdio>
#include <chrono>
#include <cmath>
#include <complex>
#include <limits>
#include <map>
#include <string>
#include <vector>

#include "amg.h"
#include "blas.h"
#include "dslash.h"
#include "sap.h"
#include "schur.h"

namespace wd {

int check_apply(const dirac_op *op, const void *out, const void *in, int nrhs, int prec);

using zc = std::complex<double>;

namespace {

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

static_assert(kGSSite <= kMdot, "partial sums of a pass are laid out kMdot + 1 wide");

// Device-side state of one right-hand side's inner GMRES cycle (carved from
// its scalar block).
struct InnerDev {
    double2 *hdr;         // [0] = (completed steps j, active flag), [1] = (normalisation factor f, 0)
    double *ic;           // [mi + 1] norms c_k of the stored basis vectors (W_k = c_k v_k)
    double2 *H;           // [(mi + 1) mi] Hessenberg columns, column-major, Givens-rotated
    double *cs;           // [mi] rotation cosines
    double2 *sn;          // [mi] rotation sines
    double2 *g;           // [mi + 1] rotated right-hand side beta e_1
    double2 *coef;        // [mi + 1] update coefficients of a step; at the end y_i / c_i
    const double2 *hcol;  // [mi + 2] inner products of the current step (mdot / axpy results)
};

size_t inner_state_bytes(int mi) {
    const size_t n2 = 2 + (size_t)(mi + 1) * mi + mi + (mi + 1) + (mi + 1);  // double2 entries
    const size_t n1 = (size_t)(mi + 1) + mi;                                // double entries
    return n2 * sizeof(double2) + n1 * sizeof(double) + 64;
}

InnerDev carve_inner(char *base, int mi, const double2 *hcol) {
    InnerDev d;
    double2 *q = reinterpret_cast<double2 *>(base);
    d.hdr = q;
    q += 2;
    d.H = q;
    q += (size_t)(mi + 1) * mi;
    d.sn = q;
    q += mi;
    d.g = q;
    q += mi + 1;
    d.coef = q;
    q += mi + 1;
    double *r = reinterpret_cast<double *>(q);
    d.ic = r;
    r += mi + 1;
    d.cs = r;
    d.hcol = hcol;
    return d;
}

constexpr int kListMax = 16;  // right-hand sides per state-kernel launch
struct InnerList {
    InnerDev d[kListMax];
    int n;
    int mi;
};

__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 c_conj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 c_scale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double c_abs(double2 a) { return hypot(a.x, a.y); }
__device__ __forceinline__ double2 c_div(double2 a, double2 b) {  // a / b, b != 0
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// start of a cycle: v_0 = W_0 has unit norm, beta = 1
__global__ void k_inner_init(InnerList L) {
    const int t = threadIdx.x;
    if (t >= L.n) return;
    const InnerDev &d = L.d[t];
    d.hdr[0] = make_double2(0.0, 1.0);
    d.hdr[1] = make_double2(1.0, 0.0);
    d.ic[0] = 1.0;
    d.g[0] = make_double2(1.0, 0.0);
    for (int i = 1; i <= L.mi; i++) d.g[i] = make_double2(0.0, 0.0);
}

// step k, after the inner products d_i = W_i^H w (i <= k) and |w|^2 of
// w = D W_k: orthogonalisation coefficients d_i / c_i^2 and the factor f that
// brings the orthogonalised vector near unit norm (Pythagorean estimate;
// with severe cancellation f = 1/|w| instead)
__global__ void k_inner_prep(InnerList L, int k) {
    const int t = threadIdx.x;
    if (t >= L.n) return;
    const InnerDev &d = L.d[t];
    if (d.hdr[0].y == 0.0) return;
    const double w2 = d.hcol[k + 1].x;
    double proj = 0.0;
    for (int i = 0; i <= k; i++) {
        const double m = 1.0 / (d.ic[i] * d.ic[i]);
        const double2 h = d.hcol[i];
        d.coef[i] = c_scale(m, h);
        proj += (h.x * h.x + h.y * h.y) * m;
    }
    const double rem = w2 - proj;
    d.hdr[1].x = rem > 1e-8 * w2 ? 1.0 / sqrt(rem) : (w2 > 0.0 ? 1.0 / sqrt(w2) : 1.0);
}

// step k, after the in-place orthogonalisation: Hessenberg column k, Givens
// rotation, residual estimate |g_{k+1}|, termination test
__global__ void k_inner_givens(InnerList L, int k, double tol, int maxit) {
    const int t = threadIdx.x;
    if (t >= L.n) return;
    const InnerDev &d = L.d[t];
    if (d.hdr[0].y == 0.0) return;
    const int ld = L.mi + 1;
    double2 *col = d.H + (size_t)k * ld;
    const double ck = d.ic[k];
    for (int i = 0; i <= k; i++) col[i] = c_scale(1.0 / (d.ic[i] * ck), d.hcol[i]);
    const double nrm = sqrt(fmax(d.hcol[k + 1].x, 0.0));  // |W_{k+1}| = f c_k h_{k+1,k}
    const double hn = nrm / (d.hdr[1].x * ck);
    for (int i = 0; i < k; i++) {
        const double2 a = col[i], b = col[i + 1];
        col[i] = c_add(c_scale(d.cs[i], a), c_mul(d.sn[i], b));
        col[i + 1] = c_sub(c_scale(d.cs[i], b), c_mul(c_conj(d.sn[i]), a));
    }
    const double2 a = col[k];
    const double r = hypot(c_abs(a), hn);
    double cs;
    double2 sn;
    if (r == 0.0) {
        cs = 1.0;
        sn = make_double2(0.0, 0.0);
    } else if (c_abs(a) == 0.0) {
        cs = 0.0;
        sn = make_double2(1.0, 0.0);  // conj(b) / |b| with b = hn > 0 real
    } else {
        const double aa = c_abs(a);
        cs = aa / r;
        sn = c_scale(hn / (aa * r), a);  // (a / |a|) conj(b) / r with b = hn real
    }
    d.cs[k] = cs;
    d.sn[k] = sn;
    col[k] = c_add(c_scale(cs, a), c_scale(hn, sn));
    col[k + 1] = make_double2(0.0, 0.0);
    const double2 gk = d.g[k];
    d.g[k + 1] = c_scale(-1.0, c_mul(c_conj(sn), gk));
    d.g[k] = c_scale(cs, gk);
    d.ic[k + 1] = nrm;
    const int j = k + 1;
    const bool stop = c_abs(d.g[k + 1]) < tol || j >= maxit || hn == 0.0;
    d.hdr[0] = make_double2((double)j, stop ? 0.0 : 1.0);
}

// cycle end: y = R^{-1} g (leading j x j triangle), coef_i = y_i / c_i
__global__ void k_inner_solve(InnerList L) {
    const int t = threadIdx.x;
    if (t >= L.n) return;
    const InnerDev &d = L.d[t];
    const int j = (int)d.hdr[0].x, ld = L.mi + 1;
    for (int i = j - 1; i >= 0; i--) {
        double2 s = d.g[i];
        for (int q = i + 1; q < j; q++) s = c_sub(s, c_mul(d.H[(size_t)q * ld + i], d.coef[q]));
        const double2 dg = d.H[(size_t)i * ld + i];
        d.coef[i] = (dg.x == 0.0 && dg.y == 0.0) ? make_double2(0.0, 0.0) : c_div(s, dg);
    }
    for (int i = 0; i < j; i++) d.coef[i] = c_scale(1.0 / d.ic[i], d.coef[i]);
}

struct Layout {
    size_t f64, f32, f16, scal;  // bytes of one field / scalar block
    size_t per_rhs;
};

int inner_prec(int mode) { return mode == FGMRES_MIXED_F32 ? WDIRAC_F32 : WDIRAC_F16S; }
bool is_mixed(int mode) { return mode == FGMRES_MIXED_F32 || mode == FGMRES_MIXED_F16S; }

// entries of each per-RHS scalar array (Hessenberg column, coefficients)
int kmax_of(const fgmres_params *p) {
    const int m = p->restart, mi = is_mixed(p->mode) ? p->inner_restart : 0;
    return (m > mi ? m : mi) + 2;
}

// sites of the solved system's vectors: V, or V/2 for the even-odd reduced system
long long system_sites(const dirac_op *op, const fgmres_params *p) { return p->schur ? op->g.V / 2 : op->g.V; }

// entries of each right-hand side's partial-sum buffer: the all-vector inner products of the outer basis (up to
// kGS vectors per launch) and the passes of the per-site kernels
size_t partial_entries(const fgmres_params *p) {
    const int nv = std::min(p->restart + 1, kGS);
    const size_t outer = (size_t)kMdotChunks * ((nv + kMdot - 1) / kMdot) * (kMdot + 1);
    return std::max(outer, (size_t)kRedBlocks * (kMdot + 1));
}

Layout layout(const dirac_op *op, const fgmres_params *p) {
    Layout L;
    const long long V = system_sites(op, p);
    L.f64 = align256(field_rhs_bytes(WDIRAC_F64, V));
    L.f32 = align256(field_rhs_bytes(WDIRAC_F32, V));
    L.f16 = align256(field_rhs_bytes(WDIRAC_F16S, V));
    const int m = p->restart, mi = is_mixed(p->mode) ? p->inner_restart : 0;
    const int kmax = kmax_of(p);
    L.scal = align256(sizeof(double2) * (partial_entries(p) + 3 * (size_t)kmax + 8));
    if (is_mixed(p->mode)) L.scal += align256(inner_state_bytes(mi));
    L.per_rhs = (size_t)(m + 2) * L.f64 + L.scal;  // V[0..m], w
    if (p->mode != FGMRES_F64) L.per_rhs += (size_t)m * L.f64;  // Z[0..m)
    if (is_mixed(p->mode)) L.per_rhs += (size_t)(mi + 1) * (p->mode == FGMRES_MIXED_F32 ? L.f32 : L.f16);  // inner W
    if (p->mode == FGMRES_SAP) L.per_rhs += align256(sap_workspace(op, &p->sap, 1));
    if (p->schur) {
        L.per_rhs += 3 * L.f64;  // x_e, reduced right-hand side, odd scratch of S
        if (is_mixed(p->mode)) L.per_rhs += p->mode == FGMRES_MIXED_F32 ? L.f32 : L.f16;  // inner odd scratch
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
    double2 *x = nullptr;  // iterate of the solved system (the user's x, or x_e for the reduced system)
    const double2 *b = nullptr;
    double2 *xu = nullptr;  // reduced system: the user's full x and b, the reduced right-hand side, and the
    const double2 *bu = nullptr;  // odd-parity scratch of S at FP64 and at the inner precision
    double2 *bh = nullptr;
    void *t64 = nullptr, *ti = nullptr;
    std::vector<void *> V, Z;  // outer basis (F64), preconditioned vectors (F64)
    double2 *w = nullptr;
    std::vector<void *> Vi;    // inner basis, inner operator precision
    double2 *sapw = nullptr;   // SAP preconditioner's workspace
    InnerDev in;               // device state of the inner cycle
    double2 *partial = nullptr, *hcol = nullptr, *coef = nullptr, *hcol2 = nullptr, *nrm = nullptr;
    // host
    Phase phase = Phase::Residual;
    Arnoldi outer;
    // the outer basis is stored unnormalised: V[i] = cw[i] v_i, and Z[i] = sz[i] z_i (sz = cw when Z aliases V,
    // 1 when the preconditioner was given v_i itself)
    std::vector<double> cw, sz;
    double r0norm = -1, relres = 1;
    bool breakdown = false, converged = false;
    bool nonfinite = false;  // a NaN or Inf reached a residual norm or a Hessenberg column
    bool x_zero = false;     // x is still the zero initial guess, so D x (or S x) is zero without an application
    long long applies = 0, inner_applies = 0, restarts = 0;
    std::vector<double> hist;
};

struct Ctx {
    const dirac_op *op;
    const fgmres_params *p;
    hipStream_t st;
    long long N;  // complex numbers per field of the solved system
    int V;        // its sites (V/2 for the even-odd reduced system)
    int apbc;
    bool schur;   // solve S x_e = bhat (even-odd reduction) instead of D x = b
    double2 *pinned;  // host staging for scalar reads (hipHostMalloc)
    size_t pinned_n;
};

// instantiated inner-cycle graphs of one solve, keyed by the right-hand sides they cover
struct GraphCache {
    hipStream_t cap = nullptr;     // private capture stream
    hipStream_t launch = nullptr;  // stream the graphs are launched on
    std::map<std::vector<int>, hipGraphExec_t> exec;
    ~GraphCache() {
        // an error return may leave launched graphs running: wait for them first
        if (!exec.empty()) (void)hipStreamSynchronize(launch);
        for (auto &e : exec) (void)hipGraphExecDestroy(e.second);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

// operator applications of the solved system: one batched stencil launch for D, or two parity launches for S
// over all listed right-hand sides (tmp: each one's odd scratch)
struct ApplyItem {
    void *out;
    const void *in;
    void *tmp;
};

hipError_t apply_many(const Ctx &c, int prec, const std::vector<ApplyItem> &items, hipStream_t s) {
    if (items.empty()) return hipSuccess;
    if (c.schur) {
        std::vector<SchurItem> list;
        for (const ApplyItem &it : items) list.push_back({it.out, it.in, it.tmp});
        return schur_apply_list(prec, false, c.op, list, s);
    }
    std::vector<dirac_batch> b;
    for (const ApplyItem &it : items) b.push_back({it.out, it.in, 1});
    return dslash_launch_batches(b.data(), (int)b.size(), prec, false, c.op->data(prec), c.op->g, c.apbc, false, s);
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

hipError_t launch_state(void (*kern)(InnerList), const std::vector<Rhs *> &rs, int mi, hipStream_t s) {
    for (size_t a = 0; a < rs.size(); a += kListMax) {
        InnerList L;
        L.n = (int)std::min<size_t>(kListMax, rs.size() - a);
        L.mi = mi;
        for (int q = 0; q < L.n; q++) L.d[q] = rs[a + q]->in;
        hipLaunchKernelGGL(kern, dim3(1), dim3(64), 0, s, L);
    }
    return hipGetLastError();
}

template <typename F> hipError_t launch_state_k(const std::vector<Rhs *> &rs, int mi, hipStream_t s, F launch) {
    for (size_t a = 0; a < rs.size(); a += kListMax) {
        InnerList L;
        L.n = (int)std::min<size_t>(kListMax, rs.size() - a);
        L.mi = mi;
        for (int q = 0; q < L.n; q++) L.d[q] = rs[a + q]->in;
        launch(L);
    }
    return hipGetLastError();
}

// Issue the body of one inner GMRES cycle (start, steps, triangular solve)
// for every listed right-hand side on stream s; W_0 must hold v = V[j].
// host_steps: read the active flags after every step (one synchronisation)
// and drop finished right-hand sides from later launches; otherwise every
// step is issued for all of them and finished ones are skipped on the device
// (graph capture).  The body does not depend on the outer slot j.
int issue_inner_body(const Ctx &c, const std::vector<Rhs *> &list, bool host_steps, hipStream_t s) {
    const fgmres_params &p = *c.p;
    const int prec = inner_prec(p.mode);
    const int mi = p.inner_restart;
    const int maxit = p.inner_maxit < mi ? p.inner_maxit : mi;
    WD_TRY(launch_state(k_inner_init, list, mi, s));
    std::vector<Rhs *> act = list;
    for (int k = 0; k < maxit && !act.empty(); k++) {
        // W_{k+1} = D W_k, one batched launch for the right-hand sides still iterating
        std::vector<ApplyItem> b;
        for (Rhs *r : act) b.push_back({r->Vi[k + 1], r->Vi[k], r->ti});
        WD_TRY(apply_many(c, prec, b, s));
        for (Rhs *r : act)
            WD_TRY(site_mdot(prec, r->Vi.data(), k + 1, r->Vi[k + 1], c.V, r->partial, r->hcol, r->in.hdr, s));
        WD_TRY(launch_state_k(act, mi, s, [&](const InnerList &L) {
            hipLaunchKernelGGL(k_inner_prep, dim3(1), dim3(64), 0, s, L, k);
        }));
        for (Rhs *r : act)
            WD_TRY(site_axpy(prec, r->Vi.data(), k + 1, r->in.coef, r->Vi[k + 1], c.V, r->partial, r->hcol + k + 1,
                             r->in.hdr, s));
        WD_TRY(launch_state_k(act, mi, s, [&](const InnerList &L) {
            hipLaunchKernelGGL(k_inner_givens, dim3(1), dim3(64), 0, s, L, k, p.inner_tol, maxit);
        }));
        if (!host_steps) continue;
        std::vector<std::pair<const double2 *, int>> src;
        for (Rhs *r : act) src.emplace_back(r->in.hdr, 1);
        std::vector<std::vector<zc>> h;
        int rc = fetch(c, src, h);
        if (rc) return rc;
        std::vector<Rhs *> next;
        for (size_t q = 0; q < act.size(); q++)
            if (h[q][0].imag() != 0.0) next.push_back(act[q]);
        act.swap(next);
    }
    WD_TRY(launch_state(k_inner_solve, list, mi, s));
    return WDIRAC_OK;
}

// Inner solves z = M^{-1} v_j of the listed right-hand sides (v_j = V[j],
// z = Z[j], j each one's outer step).  The cycle body runs step by step, or
// as a graph captured on first use for this set of right-hand sides.
int inner_solve(const Ctx &c, const std::vector<Rhs *> &list, GraphCache *gc, const std::vector<Rhs> &all) {
    const int prec = inner_prec(c.p->mode);
    const int mi = c.p->inner_restart;
    const int maxit = c.p->inner_maxit < mi ? c.p->inner_maxit : mi;
    for (Rhs *r : list)
        WD_TRY(site_scale(WDIRAC_F64, prec, r->V[r->outer.j], r->Vi[0], 1.0 / r->cw[r->outer.j], c.V, c.st));
    if (!gc) {
        int rc = issue_inner_body(c, list, true, c.st);
        if (rc) return rc;
    } else {
        std::vector<int> key;
        for (Rhs *r : list) key.push_back((int)(r - all.data()));
        auto it = gc->exec.find(key);
        if (it == gc->exec.end()) {
            if (!gc->cap) WD_TRY(hipStreamCreateWithFlags(&gc->cap, hipStreamNonBlocking));
            WD_TRY(hipStreamBeginCapture(gc->cap, hipStreamCaptureModeThreadLocal));
            const int rc = issue_inner_body(c, list, false, gc->cap);
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(gc->cap, &graph);
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (e != hipSuccess) return fail(WDIRAC_EHIP, std::string("inner-cycle capture: ") + hipGetErrorString(e));
            hipGraphExec_t exec = nullptr;
            const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) return fail(WDIRAC_EHIP, std::string("inner-cycle graph: ") + hipGetErrorString(ei));
            it = gc->exec.emplace(key, exec).first;
        }
        WD_TRY(hipGraphLaunch(it->second, c.st));
    }
    for (Rhs *r : list)
        WD_TRY(site_combine(prec, r->Vi.data(), maxit, r->in.coef, r->in.hdr, static_cast<double2 *>(r->Z[r->outer.j]),
                            c.V, c.st));
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
        hipStream_t st;
        ~PinnedGuard() {
            (void)hipStreamSynchronize(st);  // no copy into the staging buffer may still be pending
            (void)hipHostFree(p);
        }
    } guard{pinned, stream};
    const long long Vs = system_sites(op, p);
    Ctx c{op, p, stream, 12LL * Vs, (int)Vs, (op->flags & WDIRAC_ANTIPERIODIC_T) ? 1 : 0, p->schur != 0, pinned,
          pinned_n};
    const bool mixed = is_mixed(p->mode);          // preconditioner = inner GMRES
    const bool sapm = p->mode == FGMRES_SAP;       // preconditioner = SAP
    const bool amgm = p->mode == FGMRES_AMG;       // preconditioner = two-level multigrid
    SapGeom sg{};
    if (sapm) {
        const int rc = sap_geometry(op, &p->sap, sg);
        if (rc) return rc;
    }
    const int m = p->restart;
    GraphCache graphs;
    graphs.launch = stream;
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
        r.xu = reinterpret_cast<double2 *>(x) + (size_t)k * 12 * op->g.V;
        r.bu = reinterpret_cast<const double2 *>(b) + (size_t)k * 12 * op->g.V;
        r.x = r.xu;
        r.b = r.bu;
        if (c.schur) {
            r.x = reinterpret_cast<double2 *>(take(L.f64));
            r.bh = reinterpret_cast<double2 *>(take(L.f64));
            r.b = r.bh;
            r.t64 = take(L.f64);
            if (mixed) r.ti = take(p->mode == FGMRES_MIXED_F32 ? L.f32 : L.f16);
        }
        for (int i = 0; i <= m; i++) r.V.push_back(take(L.f64));
        r.w = reinterpret_cast<double2 *>(take(L.f64));
        if (mixed || sapm || amgm) {
            for (int i = 0; i < m; i++) r.Z.push_back(take(L.f64));
            const size_t fi = p->mode == FGMRES_MIXED_F32 ? L.f32 : L.f16;
            if (mixed)
                for (int i = 0; i <= p->inner_restart; i++) r.Vi.push_back(take(fi));
            if (sapm) r.sapw = reinterpret_cast<double2 *>(take(align256(sap_workspace(op, &p->sap, 1))));
        } else {
            r.Z = std::vector<void *>(r.V.begin(), r.V.begin() + m);  // M = I: z_j = v_j
        }
        char *s = take(L.scal);
        r.partial = reinterpret_cast<double2 *>(s);
        r.hcol = r.partial + partial_entries(p);
        r.coef = r.hcol + kmax;
        r.hcol2 = r.coef + kmax;
        r.nrm = r.hcol2 + kmax;
        char *end = reinterpret_cast<char *>(r.nrm + 1);
        if (mixed) {
            char *ib = s + align256(sizeof(double2) * (partial_entries(p) + 3 * (size_t)kmax + 8));
            r.in = carve_inner(ib, p->inner_restart, r.hcol);
            end = ib + inner_state_bytes(p->inner_restart);
        }
        if (end > s + L.scal) return fail(WDIRAC_EINVAL, "internal: scalar block overflow");
    }
    if ((size_t)(wp - static_cast<char *>(work)) > work_bytes) return fail(WDIRAC_EINVAL, "workspace too small");

    // phase timing: events around the preconditioner, the FP64 apply and the
    // orthogonalisation of every step (read after the step's synchronisation)
    struct Events {
        hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
        ~Events() {
            for (hipEvent_t &x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev;
    for (hipEvent_t &x : ev.e) WD_TRY(hipEventCreate(&x));
    // |x0|^2 of every right-hand side, in one synchronisation: with the usual zero initial guess the products
    // D x0 of the set-up and of the first residual are zero, so they are counted without being launched (an x0
    // whose entries all lie below ~1e-162 in magnitude also reads as zero; its product is far below the FP64
    // resolution of any residual)
    {
        std::vector<std::pair<const double2 *, int>> xs;
        const void *none = nullptr;
        for (Rhs &r : R) {
            WD_TRY(mdot_all<double2>(&none, 0, r.xu, 12LL * op->g.V, r.partial, r.nrm, c.st));
            xs.emplace_back(r.nrm, 1);
        }
        std::vector<std::vector<zc>> got;
        const int rc = fetch(c, xs, got);
        if (rc) return rc;
        for (size_t k = 0; k < R.size(); k++) R[k].x_zero = got[k][0].real() == 0.0;
    }
    if (c.schur) {
        // |b - D x0| over both parities (the tolerance's reference, so that tol means the same as for D x = b),
        // then the reduced right-hand side bhat = b_e - H_eo A_oo^{-1} b_o
        std::vector<std::pair<const double2 *, int>> src;
        for (Rhs &r : R) {
            double2 *xo = static_cast<double2 *>(r.V[0]), *bo = static_cast<double2 *>(r.V[1]);
            WD_TRY(parity_split_launch(op, WDIRAC_F64, r.x, xo, r.xu, 1, c.st));
            WD_TRY(parity_split_launch(op, WDIRAC_F64, r.bh, bo, r.bu, 1, c.st));
            // with x0 = 0 its zero halves stand for the zero halves of D x0
            if (!r.x_zero) WD_TRY(parity_launch(kParApply, WDIRAC_F64, false, op, 0, r.w, r.x, xo, 1, c.st));
            WD_TRY(residual(r.bh, r.x_zero ? xo : r.w, static_cast<double2 *>(r.t64), c.N, r.partial, r.nrm, c.st));
            if (!r.x_zero) WD_TRY(parity_launch(kParApply, WDIRAC_F64, false, op, 1, r.w, xo, r.x, 1, c.st));
            WD_TRY(residual(bo, r.x_zero ? r.x : r.w, static_cast<double2 *>(r.t64), c.N, r.partial, r.hcol2,
                            c.st));
            WD_TRY(parity_launch(kParInvSelf, WDIRAC_F64, false, op, 1, r.t64, bo, nullptr, 1, c.st));
            WD_TRY(parity_launch(kParSelfSub, WDIRAC_F64, false, op, 0, r.bh, r.bh, r.t64, 1, c.st));
            src.emplace_back(r.nrm, 1);
            src.emplace_back(r.hcol2, 1);
        }
        std::vector<std::vector<zc>> got;
        int rc = fetch(c, src, got);
        if (rc) return rc;
        for (size_t k = 0; k < R.size(); k++) {
            const double ne = got[2 * k][0].real(), no = got[2 * k + 1][0].real();
            if (!std::isfinite(ne) || !std::isfinite(no)) {
                // non-finite b or x0: no iteration can mean anything, the caller's x stays as it is
                R[k].nonfinite = true;
                R[k].phase = Phase::Done;
                continue;
            }
            R[k].r0norm = std::sqrt(std::max(ne, 0.0) + std::max(no, 0.0));
        }
    }
    double t_apply = 0, t_precond = 0, t_ortho = 0;
    bool any = true;
    while (any) {
        // preconditioning of the right-hand sides inside a cycle
        std::vector<Rhs *> arn, res;
        for (Rhs &r : R) {
            if (r.phase == Phase::Arnoldi) arn.push_back(&r);
            if (r.phase == Phase::Residual) res.push_back(&r);
        }
        WD_TRY(hipEventRecord(ev.e[0], c.st));
        if (mixed && !arn.empty()) {
            int rc = inner_solve(c, arn, p->graph ? &graphs : nullptr, R);
            if (rc) return rc;
        }
        if (sapm)
            for (Rhs *r : arn)
                WD_TRY(sap_apply(op, p->sap, sg, static_cast<double2 *>(r->Z[r->outer.j]),
                                 static_cast<const double2 *>(r->V[r->outer.j]), 1, r->sapw,
                                 1.0 / r->cw[r->outer.j], c.st));
        if (amgm)
            for (Rhs *r : arn) {
                const int rc = amg_precond_one(p->amg, static_cast<double2 *>(r->Z[r->outer.j]),
                                               static_cast<const double2 *>(r->V[r->outer.j]),
                                               1.0 / r->cw[r->outer.j], c.st);
                if (rc) return rc;
            }
        WD_TRY(hipEventRecord(ev.e[1], c.st));
        // one batched FP64 application for all of them (restart residuals and Arnoldi products)
        std::vector<ApplyItem> bat;
        for (Rhs *r : res)
            if (!r->x_zero) bat.push_back({r->w, r->x, r->t64});
        for (Rhs *r : arn) bat.push_back({r->V[r->outer.j + 1], r->Z[r->outer.j], r->t64});
        WD_TRY(apply_many(c, WDIRAC_F64, bat, c.st));
        WD_TRY(hipEventRecord(ev.e[2], c.st));
        for (Rhs *r : res) {
            r->applies++;  // counted also when x is still zero and x itself stands for the zero product
            WD_TRY(residual(r->b, r->x_zero ? r->x : r->w, static_cast<double2 *>(r->V[0]), c.N, r->partial,
                            r->nrm, c.st));
            r->x_zero = false;  // the cycle's update changes x
        }
        for (Rhs *r : arn) {
            // classical Gram-Schmidt of w = V[j+1] = D Z[j] against V[0..j]: one launch of inner products (w read
            // about once), then one update pass that also measures |w_new|^2; coefficients <V_i, w> / cw_i^2
            r->applies++;
            const int j = r->outer.j;
            std::vector<double> ic2(j + 1);
            for (int i = 0; i <= j; i++) ic2[i] = 1.0 / (r->cw[i] * r->cw[i]);
            WD_TRY(mdot_all<double2>(r->V.data(), j + 1, r->V[j + 1], c.N, r->partial, r->hcol, c.st));
            WD_TRY(axpy_multi<double2>(r->V.data(), j + 1, r->hcol, ic2.data(), r->V[j + 1], c.N, r->partial,
                                       r->hcol + j + 1, c.st));
        }
        WD_TRY(hipEventRecord(ev.e[3], c.st));
        std::vector<std::pair<const double2 *, int>> src;
        for (Rhs *r : res) src.emplace_back(r->nrm, 1);
        for (Rhs *r : arn) src.emplace_back(r->hcol, r->outer.j + 2);
        if (mixed)
            for (Rhs *r : arn) src.emplace_back(r->in.hdr, 1);  // inner steps taken
        std::vector<std::vector<zc>> got;
        if (!src.empty()) {
            int rc = fetch(c, src, got);
            if (rc) return rc;
        } else {
            WD_TRY(hipStreamSynchronize(c.st));
        }
        {
            float ms[3] = {0, 0, 0};
            for (int k = 0; k < 3; k++) WD_TRY(hipEventElapsedTime(&ms[k], ev.e[k], ev.e[k + 1]));
            t_precond += ms[0] * 1e-3;
            t_apply += ms[1] * 1e-3;
            t_ortho += ms[2] * 1e-3;
        }
        // restarts: convergence test on the true residual
        for (size_t k = 0; k < res.size(); k++) {
            Rhs &r = *res[k];
            const double n2 = got[k][0].real();
            if (!std::isfinite(n2)) {
                // NaN/Inf in b, x0 or the iterate: reported as its own outcome, never as convergence
                r.nonfinite = true;
                r.phase = Phase::Done;
                continue;
            }
            const double beta = std::sqrt(std::max(n2, 0.0));
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
            if (log_level() >= 2)
                std::fprintf(stderr, "[wdirac] fgmres rhs %d: restart %lld after %lld applies, relres %.3e\n",
                             (int)(&r - R.data()), r.restarts, r.applies, r.relres);
            r.cw.assign(m + 1, 0.0);
            r.sz.assign(m, 1.0);
            r.cw[0] = beta;  // V[0] = r = beta v_0
            if (!mixed && !sapm && !amgm) r.sz[0] = beta;  // M = I: Z aliases V
            r.outer.reset(m, beta);
            r.phase = Phase::Arnoldi;
        }
        // Arnoldi steps: Hessenberg column, Givens, continue or end the cycle
        for (size_t k = 0; k < arn.size(); k++) {
            Rhs &r = *arn[k];
            const int j = r.outer.j;
            const std::vector<zc> &hk = got[res.size() + k];
            if (mixed) r.inner_applies += (long long)got[res.size() + arn.size() + k][0].real();
            bool finite = true;
            for (int i = 0; i <= j + 1; i++) finite = finite && std::isfinite(hk[i].real()) && std::isfinite(hk[i].imag());
            if (!finite) {
                // the cycle is abandoned without its update: x keeps the iterate of the last completed cycle
                r.nonfinite = true;
                r.phase = Phase::Done;
                continue;
            }
            // Z[j] = sz_j z_j: h_ij = <V_i, V[j+1]> / (cw_i sz_j), |V[j+1]| = sz_j h_{j+1,j}
            const double szj = r.sz[j];
            std::vector<zc> col(j + 2);
            for (int i = 0; i <= j; i++) col[i] = hk[i] / (r.cw[i] * szj);
            const double cn = std::sqrt(std::max(hk[j + 1].real(), 0.0));
            const double hn = cn / szj;
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
                const int jn = r.outer.j;  // = j + 1
                r.cw[jn] = cn;
                if (!(cn > 1e-100 && cn < 1e100)) {
                    // keep the stored magnitudes representable: normalise explicitly (rare)
                    WD_TRY((scale<double2, double2>(r.V[jn], r.V[jn], nullptr, false, 1.0 / cn, c.N, c.st)));
                    r.cw[jn] = 1.0;
                }
                if (!mixed && !sapm && !amgm) r.sz[jn] = r.cw[jn];  // Z aliases V
                continue;
            }
            std::vector<zc> yz = r.outer.solve();
            for (size_t i = 0; i < yz.size(); i++) yz[i] /= r.sz[i];
            const std::vector<double2> y = to_d2(yz);
            WD_TRY(update<double2>(r.Z.data(), (int)y.size(), y.data(), r.x, c.N, c.st));
            r.phase = Phase::Residual;
        }
        any = false;
        for (Rhs &r : R)
            if (r.phase != Phase::Done) any = true;
    }
    if (c.schur) {
        // x_o = A_oo^{-1} (b_o - H_oe x_e), x = (x_e, x_o), and the true residual |b - D x| over both parities
        std::vector<std::pair<const double2 *, int>> src;
        std::vector<Rhs *> fin;
        for (Rhs &r : R) {
            if (r.nonfinite) continue;  // the caller's x is left untouched
            fin.push_back(&r);
            double2 *xo = static_cast<double2 *>(r.V[0]), *be = static_cast<double2 *>(r.V[1]);
            double2 *bo = static_cast<double2 *>(r.t64);
            WD_TRY(parity_split_launch(op, WDIRAC_F64, be, bo, r.bu, 1, c.st));
            WD_TRY(parity_launch(kParInvSelfSub, WDIRAC_F64, false, op, 1, xo, bo, r.x, 1, c.st));
            WD_TRY(parity_launch(kParApply, WDIRAC_F64, false, op, 0, r.w, r.x, xo, 1, c.st));
            WD_TRY(residual(be, r.w, r.bh, c.N, r.partial, r.nrm, c.st));
            WD_TRY(parity_launch(kParApply, WDIRAC_F64, false, op, 1, r.w, xo, r.x, 1, c.st));
            WD_TRY(residual(bo, r.w, r.bh, c.N, r.partial, r.hcol2, c.st));
            WD_TRY(parity_merge_launch(op, WDIRAC_F64, r.xu, r.x, xo, 1, c.st));
            src.emplace_back(r.nrm, 1);
            src.emplace_back(r.hcol2, 1);
        }
        std::vector<std::vector<zc>> got;
        if (!src.empty()) {
            int rc = fetch(c, src, got);
            if (rc) return rc;
        }
        for (size_t k = 0; k < fin.size(); k++) {
            const double ne = got[2 * k][0].real(), no = got[2 * k + 1][0].real();
            if (!std::isfinite(ne) || !std::isfinite(no)) {
                fin[k]->nonfinite = true;
                fin[k]->converged = false;
                continue;
            }
            const double rn = std::sqrt(std::max(ne, 0.0) + std::max(no, 0.0));
            fin[k]->relres = fin[k]->r0norm > 0 ? rn / fin[k]->r0norm : 0.0;
        }
    }
    WD_TRY(hipStreamSynchronize(stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool all = true, bad = false;
    for (int k = 0; k < nrhs; k++) {
        Rhs &r = R[k];
        all = all && r.converged;
        bad = bad || r.nonfinite;
        if (!st) continue;
        fgmres_stats &s = st[k];
        s.applies = r.applies;
        s.inner_applies = r.inner_applies;
        s.restarts = r.restarts;
        s.converged = r.converged ? 1 : 0;
        s.breakdown = r.breakdown ? 1 : 0;
        s.nonfinite = r.nonfinite ? 1 : 0;
        s.wave = nrhs;
        s.true_residual = r.nonfinite ? std::numeric_limits<double>::quiet_NaN() : r.relres;
        s.seconds = secs;
        s.seconds_apply = t_apply;
        s.seconds_precond = t_precond;
        s.seconds_ortho = t_ortho;
        s.nhist = (int)std::min<size_t>(r.hist.size(), FGMRES_HIST_MAX);
        for (int i = 0; i < s.nhist; i++) s.hist[i] = r.hist[i];
    }
    if (bad) return WDIRAC_ENONFINITE;
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
    if (p->mode != FGMRES_F64 && p->mode != FGMRES_MIXED_F32 && p->mode != FGMRES_MIXED_F16S &&
        p->mode != FGMRES_SAP && p->mode != FGMRES_AMG)
        return fail(WDIRAC_EINVAL, "unknown solver mode");
    if (p->mode == FGMRES_AMG) {
        if (!p->amg) return fail(WDIRAC_EINVAL, "FGMRES_AMG needs fgmres_params.amg");
        if (p->amg->op != op) return fail(WDIRAC_EINVAL, "the AMG was made for another operator");
        if (p->schur) return fail(WDIRAC_EUNSUPPORTED, "the AMG preconditioner works on the full system only");
    }
    if (p->mode == FGMRES_SAP) {
        if (p->schur) return fail(WDIRAC_EUNSUPPORTED, "the SAP preconditioner works on the full system only");
        SapGeom sg;
        const int rc = sap_geometry(op, &p->sap, sg);
        if (rc) return rc;
    }
    if (p->wave < 0) return fail(WDIRAC_EINVAL, "wave must be >= 0");
    if (p->schur != 0 && p->schur != 1) return fail(WDIRAC_EINVAL, "schur must be 0 or 1");
    if (p->schur) {
        if (!(op->flags & WDIRAC_EVEN_ODD)) return fail(WDIRAC_EUNSUPPORTED, "schur needs WDIRAC_EVEN_ODD at create");
        if (p->mode != FGMRES_F64 && !op->cinv(inner_prec(p->mode)))
            return fail(WDIRAC_EUNSUPPORTED, "inner precision not materialised at create");
    }
    if (is_mixed(p->mode)) {
        if (p->inner_restart < 1 || p->inner_restart > 1000) return fail(WDIRAC_EINVAL, "inner_restart in [1, 1000]");
        if (p->inner_maxit < 1) return fail(WDIRAC_EINVAL, "inner_maxit must be >= 1");
        if (!(p->inner_tol > 0.0)) return fail(WDIRAC_EINVAL, "inner_tol must be > 0");
        if (!op->data(inner_prec(p->mode)).links)
            return fail(WDIRAC_EUNSUPPORTED, "inner precision not materialised at create");
    }
    return WDIRAC_OK;
}

// Right-hand sides per wave.  An explicit p->wave is used as given (capped at
// nrhs).  With p->wave == 0 the library chooses: fgmres_workspace_bytes sizes
// the wave from the device memory free at that moment (keeping a reserve for
// the caller), and fgmres_solve takes as many right-hand sides per wave as the
// workspace it is handed can hold, so the two calls agree whenever the caller
// allocates what fgmres_workspace_bytes asked for.
static int wave_explicit(const fgmres_params *p, int nrhs) { return p->wave < nrhs ? p->wave : nrhs; }

static int wave_from_free_memory(const dirac_op *op, const fgmres_params *p, int nrhs) {
    const size_t per = solver_workspace(op, p, 1);
    size_t free_b = 0, total_b = 0;
    if (hipSetDevice(op->device) != hipSuccess || hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    // headroom for the caller's own fields and the runtime: 1/16 of the device, at least 4 GiB
    const size_t reserve = std::max(total_b / 16, (size_t)4 << 30);
    const size_t avail = free_b > reserve ? free_b - reserve : 0;
    const size_t w = per ? avail / per : (size_t)nrhs;
    return (int)std::max<size_t>(1, std::min<size_t>(w, (size_t)nrhs));
}

size_t fgmres_workspace_bytes(const dirac_op *op, const fgmres_params *p, int nrhs) {
    if (nrhs < 1 || check_params(op, p)) return 0;
    const int w = p->wave > 0 ? wave_explicit(p, nrhs) : wave_from_free_memory(op, p, nrhs);
    return solver_workspace(op, p, w);
}

int fgmres_solve(const dirac_op *op, double *x, const double *b, int nrhs, const fgmres_params *p,
                 fgmres_stats *st, void *work, size_t work_bytes, void *stream) {
    int rc = check_params(op, p);
    if (rc) return rc;
    if (!x || !b || !work) return fail(WDIRAC_EINVAL, "null x, b or workspace");
    if (nrhs < 1) return fail(WDIRAC_EINVAL, "nrhs must be >= 1");
    rc = check_apply(op, x, b, nrhs, WDIRAC_F64);
    if (rc) return rc;
    int w = 0;
    if (p->wave > 0) {
        w = wave_explicit(p, nrhs);
    } else {
        const size_t per = solver_workspace(op, p, 1);
        w = (int)std::min<size_t>(per ? work_bytes / per : (size_t)nrhs, (size_t)nrhs);
        if (w < 1) w = 1;  // rejected just below
    }
    if (work_bytes < solver_workspace(op, p, w)) return fail(WDIRAC_EINVAL, "workspace too small");
    if (reinterpret_cast<uintptr_t>(work) & 255) return fail(WDIRAC_EINVAL, "workspace must be 256-byte aligned");
    const size_t field = (size_t)24 * op->g.V;  // doubles per right-hand side
    bool notconv = false, nonfinite = false;
    for (int k0 = 0; k0 < nrhs; k0 += w) {
        const int nw = nrhs - k0 < w ? nrhs - k0 : w;
        rc = solve(op, x + k0 * field, b + k0 * field, nw, p, st ? st + k0 : nullptr, work, work_bytes,
                   (hipStream_t)stream);
        if (rc < 0) return rc;
        notconv = notconv || rc == WDIRAC_ENOTCONV;
        nonfinite = nonfinite || rc == WDIRAC_ENONFINITE;
        if (st)
            for (int k = k0; k < k0 + nw; k++) st[k].wave = w;
    }
    if (nonfinite) return WDIRAC_ENONFINITE;
    return notconv ? WDIRAC_ENOTCONV : WDIRAC_OK;
}

}  // extern "C"
