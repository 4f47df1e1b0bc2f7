/*
 * wdirac: Wilson-clover Dirac operator and FGMRES on one AMD Instinct MI355X
 * (gfx950).  C ABI.
 *
 * The operator (arXiv 2407.00041, Eq. (1.13) with lattice spacing a = 1, i.e.
 * D = D_sc - D_nc of Eqs. (2.5)-(2.7)):
 *
 *   (D psi)(x) = A(x) psi(x)
 *              - 1/2 sum_mu (I_4 - gamma_mu) (x) U_mu(x)       psi(x+mu)
 *              - 1/2 sum_mu (I_4 + gamma_mu) (x) U_mu(x-mu)^H  psi(x-mu)
 *   A(x)       = (4 + m0) I_12 + c_sw C(x),
 *   C(x)       = -(1/32) sum_{mu,nu} (gamma_mu gamma_nu) (x) (Q_mu,nu(x) - Q_nu,mu(x))
 *
 * with the clover leaves Q of Eq. (1.12) (Eq. (1.11) for C).  Lattice
 * directions T,Z,Y,X and (anti-)periodic neighbours follow Sec. 1.1,
 * Eqs. (1.7)-(1.9).  The paper does not print its gamma basis; this library
 * uses the chiral Euclidean basis gamma_mu = [[0, B_mu], [B_mu^H, 0]] with
 * B_T = 1, B_Z = -i sigma_3, B_Y = -i sigma_2, B_X = -i sigma_1, so
 * gamma_5 = diag(1, 1, -1, -1) and C(x) is block-diagonal in chirality.
 *
 * ---------------------------------------------------------------------------
 * Canonical (host-facing) layouts.  A complex number is two consecutive
 * doubles (re, im); the site index is lexicographic
 * i = ((t*nZ + z)*nY + y)*nX + x (x fastest); dims[] = {nT, nZ, nY, nX}.
 *   spinor : [nrhs][V][12] complex128, component 3*sigma + colour
 *            (Eqs. (1.1)-(1.3): colour fastest).
 *   links  : [V][4][3][3]  complex128, mu = T,Z,Y,X, U_mu(x) = link x -> x+mu,
 *            row-major ((U v)_a = sum_b U[3a+b] v_b).
 *   clover : [V][42]       complex128, the unit-c_sw term C(x): chirality
 *            block + (spins 0,1) then block - (spins 2,3); each block = its
 *            6 diagonal entries then its 15 strict-upper entries in row-major
 *            pair order (0,1),(0,2),...,(4,5); block-local index
 *            3*(sigma mod 2) + colour.  Diagonal imaginary parts are ignored.
 *
 * Native (device) field layouts, per right-hand side, one 16-byte vector of
 * consecutive spinor components per (block, site):
 *   WDIRAC_F64  : [12][V] complex128                       192 B/site
 *   WDIRAC_F32  : [ 6][V] (2 x complex64)                    96 B/site
 *   WDIRAC_F16S : [ 3][V] (4 x complex fp16), then [V] fp32 per-site scales;
 *                 stored value = scale * fp16 value, scale = max |real part or
 *                 imaginary part| over the site's 24 reals (0 -> all zero).
 * Consecutive right-hand sides are dirac_field_bytes(op, prec, 1) apart.
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by every entry point.
 *   Return value : WDIRAC_OK (0); negative = error; positive = warning.
 *                  dirac_last_error() gives a thread-local message.
 *   Streams      : `stream` is a hipStream_t (NULL = the null stream).
 *                  Entry points documented "asynchronous" only enqueue work.
 *   Ownership    : the handle owns every device buffer it allocates;
 *                  dirac_destroy frees them.  Caller buffers stay the caller's.
 *   Threads      : a handle is immutable after dirac_create, so applies of
 *                  one handle may be issued from several host threads onto
 *                  different streams.  The process-wide launch knobs
 *                  (dirac_tune_set) and the autotuner's table are guarded by
 *                  locks; a launch uses the values current when it is
 *                  issued.  Calls that share caller-owned buffers (outputs,
 *                  workspaces) must not overlap.
 */
#ifndef WDIRAC_H
#define WDIRAC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define WDIRAC_OK 0
#define WDIRAC_EINVAL (-1)       /* bad argument (null, alias, size, enum)  */
#define WDIRAC_ENOMEM (-2)       /* device allocation failed                */
#define WDIRAC_EHIP (-3)         /* a HIP runtime call or launch failed     */
#define WDIRAC_EUNSUPPORTED (-4) /* precision not materialised, no device   */
#define WDIRAC_ENOTCONV 1        /* solver hit maxit; result still valid    */
#define WDIRAC_ENONFINITE 2      /* solver met NaN/Inf in some right-hand   */
                                 /* side's b, x0 or residuals; see stats    */

/* precisions */
#define WDIRAC_F64 0
#define WDIRAC_F32 1
#define WDIRAC_F16S 2

/* dirac_create flags */
#define WDIRAC_ANTIPERIODIC_T 1u /* hops across the T boundary get sign -1 */
#define WDIRAC_WITH_F32 2u       /* also materialise FP32 links + clover    */
#define WDIRAC_WITH_F16 4u       /* also materialise FP16 links + clover    */
#define WDIRAC_COMPRESS_LINKS 8u /* store two rows per link; the third is
                                    rebuilt as conj(row0 x row1) (SU(3) only) */
#define WDIRAC_COMPRESS_CLOVER 16u /* store each chirality block of C as its
                                    spin-diagonal difference and off-diagonal
                                    3x3 blocks (27 of 36 reals) */
#define WDIRAC_EVEN_ODD 32u      /* also store A(x)^{-1} for the even-odd
                                    (red-black) reduced system; every extent
                                    must be even */

typedef struct dirac_op dirac_op;

/* Message of the last error raised on the calling thread ("" if none). */
const char *dirac_last_error(void);

/* Library version string. */
const char *dirac_version(void);

/*
 * Create an operator (Sec. 2.3: the operator data are the links and the
 * per-site self-coupling matrices; the clover part is computed once, not per
 * application).
 *   dims   : {nT, nZ, nY, nX}, each >= 2.
 *   links  : HOST canonical links (see above).
 *   clover : HOST canonical packed unit-c_sw term C(x), or NULL to build it
 *            from the links on the device (Eqs. (1.11)-(1.12)).
 *   m0,csw : mass and clover coefficient; A(x) = (4 + m0) I + csw C(x).
 *   flags  : WDIRAC_* flags above.  FP64 data are always materialised.
 *            WDIRAC_COMPRESS_LINKS keeps 2 of the 3 rows of every link (the
 *            third row of an SU(3) matrix is conj(row0 x row1)); it needs
 *            |U U^H - 1| and |det U - 1| <= 1e-12 for every link.
 *            WDIRAC_COMPRESS_CLOVER uses that each 6x6 chirality block of
 *            the clover term of Eq. (1.11) is sum_k sigma_k (x) G_k (Pauli
 *            matrices in the block's two spins, since gamma_mu gamma_nu is
 *            block diagonal with traceless 2x2 blocks for mu != nu): its two
 *            spin-diagonal 3x3 blocks are opposite, so A's block is stored as
 *            H = (A_00 - A_11)/2 (Hermitian, 9 reals) and A_01 (18 reals),
 *            with A_00 = (4+m0) + H, A_11 = (4+m0) - H.  It needs
 *            |C_00 + C_11| <= 1e-10 max(1, |C|) at every site (always true for
 *            a clover built from the links).
 *            WDIRAC_EVEN_ODD additionally stores the inverse of each 6x6
 *            chirality block of A(x) (FP64 Gauss-Jordan with partial
 *            pivoting, packed like the clover, at every materialised
 *            precision) for the even-odd functions below.
 * Synchronous.  Copies everything into device memory owned by the handle;
 * the caller may free its arrays on return.  Errors: EINVAL (null pointer,
 * dims < 2, a NaN or Inf entry in the links or in the clover passed in,
 * non-SU(3) links with WDIRAC_COMPRESS_LINKS, a clover without the
 * structure above with WDIRAC_COMPRESS_CLOVER, an odd extent or a (nearly)
 * singular block of A with WDIRAC_EVEN_ODD), ENOMEM, EHIP, EUNSUPPORTED
 * (no HIP device).
 */
int dirac_create(dirac_op **op, const int dims[4], const double *links, const double *clover,
                 double m0, double csw, unsigned flags);

/* Free the handle and its device memory.  NULL is accepted. */
int dirac_destroy(dirac_op *op);

/* Number of lattice sites V of the handle (0 for NULL). */
long long dirac_volume(const dirac_op *op);

/* Bytes of a native field of `nrhs` right-hand sides at precision `prec`
 * (0 on bad arguments). */
size_t dirac_field_bytes(const dirac_op *op, int prec, int nrhs);

/*
 * out = D in (Eq. (1.13)), for nrhs right-hand sides in native layout at
 * precision prec, on device buffers of dirac_field_bytes(op, prec, nrhs)
 * bytes each.  Each lane loads the links and clover entries its site needs
 * once per block of right-hand sides; a link or neighbour spinor that
 * several sites use is loaded by each of them, and the caches absorb only
 * part of those repeats (at 48^3 x 96 the FP64 apply reads about 1.6x its
 * algorithmic bytes from the memory side of the L2).  Asynchronous on
 * `stream`; no allocation, no host sync.
 * Errors: EINVAL (null, nrhs < 1, out overlapping in, unknown prec),
 * EUNSUPPORTED (prec not materialised by dirac_create), EHIP (launch).
 */
int dirac_apply(const dirac_op *op, void *out, const void *in, int nrhs, int prec, void *stream);

/*
 * out = D^H in.  The adjoint swaps the projectors of Eq. (1.13):
 * -1/2 (I + gamma_mu) (x) U_mu(x) psi(x+mu) - 1/2 (I - gamma_mu) (x)
 * U_mu(x-mu)^H psi(x-mu), with A(x) Hermitian; equivalently gamma_5 D gamma_5.
 * Same arguments, behaviour and errors as dirac_apply.
 */
int dirac_apply_adjoint(const dirac_op *op, void *out, const void *in, int nrhs, int prec,
                        void *stream);

/*
 * Several independent batches of right-hand sides (possibly of different
 * sizes) through ONE launch over a work list of (site tile, register block of
 * right-hand sides) items spanning all batches: out_b = D in_b (or D^H when
 * dagger != 0) for every batch.  Each link and clover entry is read once per
 * site tile and register block (tile orders 0-4), or once per site for all
 * right-hand sides of the launch (order 5).  Work-groups are handed out by
 * the hardware in item order, or, with the "persistent_blocks" knob set, a
 * persistent grid of that many resident work-groups strides through the list.
 */
typedef struct {
    void *out;       /* native, nrhs fields                                 */
    const void *in;  /* native, nrhs fields, must not overlap out           */
    int nrhs;        /* >= 1                                                */
} dirac_batch;

int dirac_apply_batched(const dirac_op *op, const dirac_batch *batches, int nbatch, int prec,
                        int dagger, void *stream);

/*
 * Process-wide launch parameters of the stencil kernels (the autotuner's
 * knobs).  Keys: "block" (threads per work-group: 64, 128, 192, 256),
 * "order" (0 linear, 1 one contiguous 1/8 of the lattice per XCD, 2 every
 * XCD takes 1/8 of each T-slice and the slices are swept in order, 3 lanes
 * walk columns along T carrying the T neighbours in registers, 4 as 3 with
 * each work-group's columns forming a 16 (X) x 4 (Y) x block/64 (Z) patch,
 * 5 link-stationary: FP32/FP16S with two-row links, each lane keeps its links
 * and clover on chip for all right-hand sides of the launch, 128-lane
 * work-groups over the tiles of order 6; other precisions and link formats
 * fall back to order 2, 6 XCD k takes the (t, z) planes with z = k mod 8,
 * z-block by z-block and each block's planes in T order),
 * "tchunk" (orders 3 and 4: sites per lane along T, >= 1; order 5:
 * right-hand sides per launch, the launch split into groups of that many,
 * 1 or >= 64 for all in one launch),
 * "persistent_blocks" (0, the default: dirac_apply_batched launches one
 * work-group per work item; > 0: a persistent grid of at most that many and
 * at most the co-resident work-groups, each walking the item list),
 * "nr_f64", "nr_f32", "nr_f16s" (right-hand sides per register block: 1, 2
 * or 4; for order 5 the tile shape instead: 1 for tiles of 128 consecutive
 * sites of one (t, z) plane, 2 for the same 64 (y, x) sites of two
 * consecutive z-planes, one wave each, 4 for those walked along T in (y, x)
 * blocks of about eight x-rows).  Setting any of these launch knobs makes them override autotuned
 * choices; "explicit" = 0 returns to the autotuned ones (1 forces the knobs).
 * Not synchronised with launches in flight; set before applying.
 * Errors: EINVAL (unknown key or value out of range).
 */
int dirac_tune_set(const char *key, int value);
int dirac_tune_get(const char *key, int *value);

/*
 * Autotuner: time candidate launch configurations of the stencil (tile order,
 * work-group size, T-chunk, register block) for this operator, precision and
 * nrhs right-hand sides in one launch, on temporary device buffers, and keep
 * the fastest for every later launch with the same lattice extents,
 * precision, right-hand-side bucket (1, 2, 3-4, 5-8, ...), link format and
 * clover format.  Candidates: tile orders 0, 2, 3, 4 (and, for several
 * right-hand sides, 6, and 5 for FP32/FP16S with two-row links, in one
 * launch or groups of 4, 6, 8, 12 or 16 right-hand sides, over plane or
 * z-pair tiles), work-groups of 128/256,
 * T-chunks 2/4/8, register blocks 1/2/4 and, for several right-hand sides, a
 * persistent grid.  The choice is appended to the JSON-lines file named by
 * the environment variable WDIRAC_TUNE_CACHE when it is set; that file is
 * read back the first time a configuration is looked up.  Synchronous;
 * allocates.
 *   cfg_out (optional): {order, block, tchunk, nr, persistent} chosen;
 *   us_out (optional): its time per launch in microseconds.
 * Errors: EINVAL, EUNSUPPORTED (precision not materialised), ENOMEM, EHIP.
 */
int dirac_autotune(const dirac_op *op, int prec, int nrhs, int cfg_out[5], double *us_out, void *stream);

/* Forget every autotuned configuration of this process. */
int dirac_tune_clear(void);

/*
 * Canonical <-> native conversion of device fields: the reordering of a
 * site's consecutive components into component-major arrays of the paper's
 * componentwise storage (Sec. 4.5, Eq. (4.1), and the reordering step of
 * Listing 4.4), here with one 16-, 8- or 4-byte vector per (block, site).
 *   dirac_pack   : native[prec] <- canonical complex128 [nrhs][V][12]
 *                  (F32: round to nearest even; F16S: per-site scale as
 *                  documented above, round to nearest even).
 *   dirac_unpack : canonical complex128 <- native[prec].
 * Both buffers on the device.  Asynchronous.  Errors: EINVAL.
 */
int dirac_pack(const dirac_op *op, void *native, const double *canonical, int nrhs, int prec,
               void *stream);
int dirac_unpack(const dirac_op *op, double *canonical, const void *native, int nrhs, int prec,
                 void *stream);

/*
 * Unit-c_sw clover term from device canonical links (Eqs. (1.11)-(1.12)):
 * clover_out = C(x), canonical packed [V][42] complex128, device buffers.
 * Independent of any handle.  Asynchronous.  Errors: EINVAL, EHIP.
 */
int dirac_clover_term(const int dims[4], const double *links_dev, double *clover_dev, void *stream);

/* ------------------------------------------------------------------------ */
/*
 * Schwarz alternating procedure (SAP), the block smoother Sec. 1.3 names for
 * the preconditioner of FGMRES (additive and red-black multiplicative
 * Schwarz over non-overlapping lattice blocks; the paper gives no further
 * detail, the method follows its textbook definition):
 *   - blocks of block[0] x ... x block[3] sites (T, Z, Y, X); each extent
 *     divides the lattice extent, every direction holds an even number of
 *     blocks or exactly one (a block spanning a direction keeps its hops in
 *     that direction, periodically), and a block has at most 256 sites.  A
 *     block's colour is the sum of its block coordinates mod 2.
 *   - D_B, the block operator, is D with the hops that leave the block
 *     dropped; the local solve is mr_iters minimal-residual steps from 0:
 *     q = D_B rho, alpha = <q, rho> / <q, q>, e += alpha rho, rho -= alpha q.
 *   - a red-black cycle: for colour 0 then 1, r = b - D x and x_B += e_B on
 *     every block of that colour; an additive cycle: one r = b - D x, then
 *     x_B += e_B on every block.
 * The block arithmetic runs at `prec` (FP64, or FP32 with the FP32 operator
 * data); x and b are FP64 and the dot products accumulate in FP64.
 */
typedef struct {
    int block[4];  /* block extents {bT, bZ, bY, bX}                        */
    int cycles;    /* Schwarz cycles (>= 1), from x = 0                       */
    int mr_iters;  /* minimal-residual steps per block solve (>= 1)          */
    int additive;  /* 0 = red-black multiplicative, 1 = additive             */
    int prec;      /* WDIRAC_F64 or WDIRAC_F32                               */
} sap_params;

/* Device workspace dirac_sap needs: nrhs FP64 fields for additive SAP with
 * cycles > 1 (two iterates alternate), else 0.  0 also on bad arguments. */
size_t dirac_sap_workspace_bytes(const dirac_op *op, const sap_params *p, int nrhs);

/*
 * x = SAP(b): `cycles` Schwarz cycles on D x = b from x = 0, for nrhs
 * right-hand sides.  x, b: device native FP64 fields (x overwritten, must not
 * overlap b); work: device workspace of dirac_sap_workspace_bytes bytes (may
 * be NULL when that is 0), must not overlap x or b.  Asynchronous; no
 * allocation.  One work-group per block and pass.  Errors: EINVAL (null
 * pointer, overlap, a blocking that breaks the rules above, cycles or
 * mr_iters < 1, workspace too small), EUNSUPPORTED (prec not materialised),
 * EHIP.
 */
int dirac_sap(const dirac_op *op, double *x, const double *b, int nrhs, const sap_params *p, void *work,
              size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/*
 * Two-level aggregation multigrid (AMG), the preconditioner Sec. 1.3
 * outlines: a coarse operator D_c that acts like D on the near kernel (the
 * eigenvectors of small |eigenvalue|, which the Schwarz smoother reduces
 * poorly) and keeps D's nearest-neighbour structure, a restriction R and a
 * prolongation P, and the subspace correction z <- z + P D_c^{-1} R r,
 * which with the smoother approximates D z = v; the setup approximates
 * right eigenvectors of small eigenvalues (Sec. 5.1 / Table 5.2: the
 * coarse lattice, 24 test vectors, 4 setup iterations in the paper's runs).
 * The paper gives no formulas; this library reads the outline as:
 *   - aggregates of agg[0] x ... x agg[3] sites (T, Z, Y, X; each extent
 *     divides the lattice extent); one coarse site per aggregate, coarse
 *     sites lexicographic in the aggregate coordinates (x fastest);
 *   - P from the N = ntv test vectors: on every (aggregate, chirality) --
 *     chirality 0 = spins 0, 1 (gamma_5 = +1), 1 = spins 2, 3 -- the test
 *     vectors restricted there are orthonormalised in order (Gram-Schmidt:
 *     the Q of a QR factorisation with positive real diag(R)); column
 *     (a, s, k) of P is the k-th of them.  R = P^H, D_c = P^H D P;
 *   - coarse vectors: device complex128 [Vc][2][N] (coarse site, chirality,
 *     test vector), Vc = product of the coarse extents; nrhs of them back
 *     to back;
 *   - M r = e + SAP(r - D e) with e = P D_c^{-1} P^H r, D_c^{-1} by GMRES
 *     (restart coarse_restart, from 0, to |b - D_c x| <= coarse_tol |b| or
 *     coarse_maxit applications of D_c), SAP as in dirac_sap;
 *   - setup: init_iters passes of v_k <- SAP(v_k) / |SAP(v_k)| over the
 *     caller's test vectors, build P and D_c; then setup_iters passes of
 *     v_k <- M v_k / |M v_k| with the current two-level method, each
 *     followed by a rebuild.
 * Everything runs in FP64 except the smoother (its own precision) and,
 * with prec = WDIRAC_F32, the storage of P.
 */
typedef struct {
    int agg[4];            /* aggregate extents {aT, aZ, aY, aX}              */
    int ntv;               /* test vectors N, 1..32 (2N unknowns per coarse   */
                           /* site); at most 6 x the sites of an aggregate    */
    int init_iters;        /* smoother passes over the test vectors (>= 0)    */
    int setup_iters;       /* two-level passes over the test vectors (>= 0)   */
    sap_params smoother;   /* post-smoother of M and smoother of the setup    */
    int coarse_restart;    /* GMRES restart on D_c, 1..1000                   */
    long long coarse_maxit;/* D_c applications per coarse solve (>= 1)        */
    double coarse_tol;     /* relative residual of a coarse solve, (0, 1)     */
    int prec;              /* storage of P: WDIRAC_F64 or WDIRAC_F32 (FP32    */
                           /* rounds the orthonormal columns; restriction,    */
                           /* prolongation and the coarse build still         */
                           /* accumulate in FP64)                             */
} amg_params;

typedef struct dirac_amg dirac_amg;

/* what dirac_amg_export copies */
#define WDIRAC_AMG_TEST_VECTORS 0    /* the N test vectors: N native FP64 fields          */
#define WDIRAC_AMG_INTERPOLATION 1   /* P as N native FP64 fields q_k (q_k on (a, s) =    */
                                     /* column (a, s, k))                                 */
#define WDIRAC_AMG_COARSE_OPERATOR 2 /* D_c blocks: complex128 [Vc][5][2N][2N], per       */
                                     /* coarse site its block with itself, then with its  */
                                     /* +T, +Z, +Y, +X neighbour (rows = output unknowns  */
                                     /* s N + k; hops gathered by direction, so a block   */
                                     /* to a neighbour that is also the -mu neighbour     */
                                     /* holds the +mu hops only; zero where one aggregate */
                                     /* spans the direction); the -mu blocks follow from  */
                                     /* D_c[a, a - mu] = G5 D_c[a - mu, a]^H G5, G5 = +1  */
                                     /* on chirality 0 and -1 on chirality 1              */

/*
 * Run the setup and create the two-level method for `op` (which must hold
 * the FP64 operator and the smoother's precision).  testvecs: device, N
 * native FP64 fields, the initial test vectors (drawn by the caller, e.g.
 * Gaussian); copied, the caller keeps ownership.  The handle owns its
 * device memory (2N fields for test vectors and P, D_c, the coarse GMRES
 * basis and two fine temporaries) and a small pinned staging buffer, and
 * keeps a pointer to `op`, which must outlive it.  Blocks until the setup
 * is done.  Calls that use one handle must not overlap (they share its
 * workspace).  Errors: EINVAL (parameters, test vectors dependent on some
 * aggregate), ENOMEM, EUNSUPPORTED (precision not materialised), EHIP.
 */
int dirac_amg_create(dirac_amg **amg, const dirac_op *op, const amg_params *p, const double *testvecs,
                     void *stream);
int dirac_amg_destroy(dirac_amg *amg);
/* Coarse extents, unknowns per coarse site (2N) and, in coarse_stats when not
 * NULL, {coarse solves, D_c applications} since create. */
int dirac_amg_sizes(const dirac_amg *amg, int coarse_dims[4], int *unknowns_per_site, long long *coarse_stats);
/* coarse = P^H fine (nrhs native FP64 fields -> nrhs coarse vectors).  Asynchronous. */
int dirac_amg_restrict(const dirac_amg *amg, double *coarse, const double *fine, int nrhs, void *stream);
/* fine = P coarse.  Asynchronous. */
int dirac_amg_prolong(const dirac_amg *amg, double *fine, const double *coarse, int nrhs, void *stream);
/* out = D_c in (coarse vectors; out must not overlap in).  Asynchronous. */
int dirac_amg_coarse_apply(const dirac_amg *amg, double *out, const double *in, int nrhs, void *stream);
/* x = D_c^{-1} b by the coarse GMRES of M (one coarse vector); iters (may be
 * NULL) = D_c applications.  Blocking. */
int dirac_amg_coarse_solve(const dirac_amg *amg, double *x, const double *b, long long *iters, void *stream);
/* z = M r for nrhs native FP64 fields (z must not overlap r).  Blocking. */
int dirac_amg_precond(const dirac_amg *amg, double *z, const double *r, int nrhs, void *stream);
/* Copy the test vectors, P or D_c (WDIRAC_AMG_*) into device memory at out. */
int dirac_amg_export(const dirac_amg *amg, int what, double *out, void *stream);

/* ------------------------------------------------------------------------ */
/* FGMRES (Algorithm 2, Sec. 1.2) for D x = b.                               */

#define FGMRES_F64 0        /* plain FP64 FGMRES(restart), no preconditioner */
#define FGMRES_MIXED_F32 1  /* FP64 outer FGMRES, inner GMRES on FP32 D     */
#define FGMRES_MIXED_F16S 2 /* FP64 outer FGMRES, inner GMRES on FP16S D    */
#define FGMRES_SAP 3        /* FP64 FGMRES, M_j^{-1} = SAP (fgmres_params.sap) */
#define FGMRES_AMG 4        /* FP64 FGMRES, M_j^{-1} = the two-level method   */
                            /* of fgmres_params.amg                            */

typedef struct {
    int restart;        /* outer Krylov dimension m (>= 1)                   */
    double tol;         /* stop when ||b - D x|| < tol ||b - D x0||          */
    long long maxit;    /* maximum FP64 operator applications                */
    int mode;           /* FGMRES_F64 / FGMRES_MIXED_F32 / FGMRES_MIXED_F16S */
    int inner_restart;  /* inner GMRES dimension (mixed modes)               */
    double inner_tol;   /* inner relative residual target (mixed modes)      */
    int inner_maxit;    /* inner operator applications per outer step        */
    int graph;          /* mixed modes: 1 = run each inner cycle as a HIP     */
                        /* graph, captured once per set of right-hand sides  */
                        /* and replayed (no host step per inner iteration);  */
                        /* 0 = issue it step by step                         */
    int wave;           /* right-hand sides solved together (lockstep, one   */
                        /* batched apply per step); nrhs is processed in     */
                        /* consecutive waves of this size.  0 = chosen by    */
                        /* the library: fgmres_workspace_bytes sizes the     */
                        /* wave from the free device memory (minus a reserve */
                        /* of max(1/16 of the device, 4 GiB)), fgmres_solve  */
                        /* fits as many right-hand sides per wave as its     */
                        /* workspace holds; the wave used is in the stats    */
    int schur;          /* 1 = solve the even-odd reduced system S x_e = bhat */
                        /* (operator created with WDIRAC_EVEN_ODD) and       */
                        /* reconstruct x_o; tol stays relative to the full   */
                        /* |b - D x0|; only the even sites of x0 start the   */
                        /* iteration; applies count applications of S       */
                        /* (not with FGMRES_SAP)                             */
    sap_params sap;     /* FGMRES_SAP: the preconditioner's SAP; its work is */
                        /* part of the solver's workspace                    */
    const dirac_amg *amg; /* FGMRES_AMG: the two-level preconditioner (made  */
                        /* by dirac_amg_create for the same operator; its    */
                        /* own workspace is used, one right-hand side at a   */
                        /* time; full system only)                           */
} fgmres_params;

#define FGMRES_HIST_MAX 4096

typedef struct {
    long long applies;          /* FP64 operator applications (a product   */
                                /* with the zero initial guess is counted  */
                                /* but, being zero, not launched)          */
    long long inner_applies;    /* low-precision applications (mixed)        */
    long long restarts;         /* outer cycles                              */
    int converged;              /* 1 if the tolerance was met                */
    int breakdown;              /* 1 if |h_{j+1,j}| < tol/10 ended a cycle   */
    int nonfinite;              /* 1 if a NaN/Inf appeared in ||b - D x0||,  */
                                /* a restart residual or a Hessenberg column */
                                /* (b, x0 or the operator data not finite):  */
                                /* the right-hand side stops, converged = 0, */
                                /* true_residual = NaN, and x holds x0 or    */
                                /* the iterate of its last completed cycle   */
    int wave;                   /* right-hand sides of the wave it ran in    */
    double true_residual;       /* final ||b - D x|| / ||b - D x0||, FP64    */
    double seconds;             /* wall time of the solve (of its wave)      */
    double seconds_apply;       /* of which FP64 operator applications,      */
    double seconds_precond;     /* inner (low-precision) solves, and          */
    double seconds_ortho;       /* outer Gram-Schmidt and residuals (GPU     */
                                /* time of the wave, from HIP events)         */
    int nhist;                  /* entries in hist[]                         */
    double hist[FGMRES_HIST_MAX]; /* relative residual estimate per step    */
} fgmres_stats;

/* Workspace bytes fgmres_solve needs for `nrhs` right-hand sides: for one
 * wave of min(p->wave, nrhs) of them when p->wave > 0, or for a wave sized
 * from the free device memory when p->wave == 0 (at least one right-hand
 * side).  0 on bad arguments. */
size_t fgmres_workspace_bytes(const dirac_op *op, const fgmres_params *p, int nrhs);

/*
 * Solve D x_r = b_r for nrhs right-hand sides.  Every right-hand side runs
 * its own FGMRES (its own Krylov space, residuals and convergence test); the
 * operator applications of the right-hand sides still iterating are issued
 * together as one batched launch.
 *   x, b : device, native FP64, nrhs fields each.  x is the initial guess on
 *          entry (x0) and the solution on return.
 *   st   : host array of nrhs stats records (may be NULL); `seconds` is the
 *          wall time of the wave that solved the right-hand side.
 *   work : device workspace (256-byte aligned) of at least
 *          fgmres_workspace_bytes(op, p, nrhs) bytes for p->wave > 0; with
 *          p->wave == 0 every wave takes as many right-hand sides as
 *          work_bytes can hold (at least one).  Reused by every wave.
 * Blocks until done (one host synchronisation per outer Arnoldi step to read
 * the residual estimates, plus one per inner step unless p->graph is set).
 * Each call also allocates a small pinned host staging buffer (a few KB) and
 * four HIP events for the phase timers, and, with p->graph, its graphs; all
 * are released before it returns.
 * Returns WDIRAC_ENONFINITE (> 0) when some right-hand side met a NaN or Inf
 * (its stats record has nonfinite = 1; the other right-hand sides are solved
 * as if it were absent), else WDIRAC_ENOTCONV (> 0) when some right-hand side
 * reached maxit (x still holds its last iterate); errors: EINVAL,
 * EUNSUPPORTED (mixed-mode precision not materialised), EHIP.
 */
int fgmres_solve(const dirac_op *op, double *x, const double *b, int nrhs,
                 const fgmres_params *p, fgmres_stats *st, void *work, size_t work_bytes,
                 void *stream);

/* ------------------------------------------------------------------------ */
/*
 * Even-odd (red-black) reduction.  Red-black ordering is one of the
 * splittings the paper's solver library uses in its Schwarz smoothers
 * (Sec. 1.3); here it is applied to the whole system as a Schur complement
 * (sites coloured by (t + z + y + x) mod 2, the odd sites eliminated).
 * With D = A + H (A(x) the site-local term,
 * H the hopping sum of Eq. (1.13), which only couples sites of opposite
 * parity (t + z + y + x) mod 2), eliminating the odd sites gives
 *     S x_e = b_e - H_eo A_oo^{-1} b_o,   S = A_ee - H_eo A_oo^{-1} H_oe,
 *     x_o   = A_oo^{-1} (b_o - H_oe x_e).
 * A parity field holds the V/2 sites of one parity in lexicographic order
 * (half-lattice index s >> 1 of full-lattice site s), in the native layout
 * of its precision with V/2 in place of V (dirac_field_bytes of a lattice of
 * V/2 sites; nrhs fields back to back).  All need an operator created with
 * WDIRAC_EVEN_ODD and the precision materialised; all are asynchronous on
 * `stream`.  Errors: EINVAL (null or misaligned pointer, overlapping buffers
 * as stated, nrhs < 1, unknown precision), EUNSUPPORTED (no WDIRAC_EVEN_ODD
 * or precision not materialised), EHIP.
 */
/* Bytes of nrhs parity fields at a precision (0 for a null operator). */
size_t dirac_parity_field_bytes(const dirac_op *op, int prec, int nrhs);
/* full field -> even and odd parity fields (no overlap among the three). */
int dirac_parity_split(const dirac_op *op, void *even, void *odd, const void *full, int nrhs, int prec,
                       void *stream);
/* even and odd parity fields -> full field (full overlaps neither). */
int dirac_parity_merge(const dirac_op *op, void *full, const void *even, const void *odd, int nrhs, int prec,
                       void *stream);
/* out = S in (dagger != 0: S^H in = A_ee in - (H^H)_eo A_oo^{-1} (H^H)_oe in);
 * in, out even fields; tmp: nrhs odd fields of scratch (receives
 * A_oo^{-1} H_oe in).  out, tmp and in must not overlap. */
int dirac_apply_schur(const dirac_op *op, void *out, const void *in, void *tmp, int nrhs, int prec, int dagger,
                      void *stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * out = S in (or S^H in) as dirac_apply_schur, with the odd-parity
 * intermediate A_oo^{-1} H_oe in kept in a static device array of the
 * library (128 MiB per device, held until the process ends) instead of a
 * caller's tmp.  nrhs odd fields must fit in it: at most 134217728 bytes of
 * dirac_parity_field_bytes(op, prec, nrhs), i.e. about 1.4 M lattice sites
 * per FP64 right-hand side; larger requests fail with EINVAL.  Calls no
 * allocating routine (device, pinned or host).  Every call on one device
 * shares that scratch, so calls that overlap on a device (concurrent
 * streams or threads) race; the scratch keeps the last call's values.
 * Results are bit-identical to dirac_apply_schur.  Errors as for
 * dirac_apply_schur, plus EHIP when the scratch was not set up (the
 * operator's create resolves it on its device). */
int dirac_apply_schur_noalloc(const dirac_op *op, void *out, const void *in, int nrhs, int prec, int dagger,
                              void *stream);
/* bhat = b_even - H_eo A_oo^{-1} b_odd (the reduced right-hand side); tmp:
 * nrhs odd fields receiving A_oo^{-1} b_odd (may be b_odd itself, must not
 * overlap b_even); bhat may be b_even itself and must not overlap tmp. */
int dirac_schur_prepare(const dirac_op *op, void *bhat, const void *b_even, const void *b_odd, void *tmp, int nrhs,
                        int prec, void *stream);
/* x_odd = A_oo^{-1} (b_odd - H_oe x_even); x_odd may be b_odd itself and
 * must not overlap x_even. */
int dirac_schur_reconstruct(const dirac_op *op, void *x_odd, const void *x_even, const void *b_odd, int nrhs,
                            int prec, void *stream);

/* ------------------------------------------------------------------------ */
/*
 * Link derivative ("force") of L = Re sum_r <eta_r, D(U) x_r> (FP64):
 * the hopping term of Eq. (1.13) and the clover leaves of Eqs. (1.11)-(1.12)
 * differentiated with respect to each link.
 *   dU  : device [V][4][3][3] complex128 (canonical link layout), written:
 *         F_mu(x) = P_TA(G_mu(x) U_mu(x)^H), P_TA(M) = (M - M^H)/2 -
 *         tr(M - M^H)/6, with G = dL/dRe U + i dL/dIm U, summed over the
 *         nrhs pairs; with raw != 0, G itself is written instead.
 *   eta, x : device native FP64, nrhs fields each.
 *   work : device workspace of at least dirac_force_workspace_bytes(op)
 *          bytes (may be NULL when that is 0); it holds the clover
 *          insertion matrices between the kernel's two passes, so calls that
 *          overlap must not share it.
 * Includes the clover contribution when csw != 0 and the clover term was
 * built from the links.  Asynchronous.  Errors: EINVAL (null pointer,
 * nrhs < 1, workspace too small), EHIP.
 */
size_t dirac_force_workspace_bytes(const dirac_op *op);
int dirac_force(const dirac_op *op, double *dU, const double *eta, const double *x, int nrhs,
                int raw, void *work, size_t work_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* WDIRAC_H */
