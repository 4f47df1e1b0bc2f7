/*
 * FP64 CPU oracle for the Wilson-clover Dirac operator (arXiv 2407.00041).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
 * reference that the GPU library is checked against.  It shares no code,
 * header, table or helper with the GPU library, and only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Everything here is the definition written out, in double precision, one
 * lattice site at a time:
 *   - lattice, directions T,Z,Y,X and (anti-)periodic neighbours: Sec. 1.1,
 *     Eqs. (1.7)-(1.9);
 *   - spinor component order, colour fastest (index 3*sigma + c): Eqs. (1.1)-(1.3);
 *   - clover leaves Q_{mu nu}(x): Eq. (1.12), every ordered pair (mu,nu)
 *     evaluated from the four products as printed (Q_{nu mu} is NOT taken
 *     as the conjugate of Q_{mu nu});
 *   - clover term -(1/32) sum_{mu,nu} (gamma_mu gamma_nu) (x) (Q_{mu nu} - Q_{nu mu})
 *     over all 16 ordered pairs: Eq. (1.11);
 *   - the operator in its rearranged form, Eq. (1.13) with a = 1, i.e.
 *     D psi = D_sc psi - D_nc psi of Eqs. (2.5)-(2.7).  The hopping blocks are
 *     applied as the full 12x12 Kronecker products (I_4 -/+ gamma_mu) (x) U,
 *     without half-spinor projection.
 *
 * Readings of points the paper leaves open (gamma basis, packed clover
 * order, link entry order, site order, boundary sign) are stated next to the
 * code that implements them.
 *
 * Canonical layouts (all complex numbers are two consecutive doubles re, im):
 *   spinor : [V][12]          component 3*sigma + c
 *   links  : [V][4][3][3]     mu = T,Z,Y,X; U_mu(x) is the link x -> x+mu,
 *                             row-major, (U v)_a = sum_b U[3a+b] v_b
 *   clover : [V][42]          unit-c_sw clover term C(x), packed:
 *                             chirality block + (spins 0,1) then block -
 *                             (spins 2,3); each block = 6 diagonal entries,
 *                             then the 15 strict-upper entries in row-major
 *                             pair order (0,1),(0,2),...,(4,5); block-local
 *                             index 3*(sigma mod 2) + c.  Imaginary parts of
 *                             the diagonal entries are ignored on input.
 *   site   : lexicographic i = ((t*nZ + z)*nY + y)*nX + x, x fastest.
 *
 * parity pinned: see the oracle tests (free-field and constant-U(1) plane
 * waves in closed form, gamma_5-hermiticity, the adjoint identity, gauge
 * covariance, constant abelian field strength, dense brute force from the
 * covariant differences of Eq. (1.10)).
 */
#include <complex.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* gamma matrices.  The paper does not print its basis; we use the
 * chiral Euclidean basis gamma_mu = [[0, B_mu], [B_mu^H, 0]] (2x2 blocks
 * in spin space) with B_T = 1, B_Z = -i sigma_3, B_Y = -i sigma_2,
 * B_X = -i sigma_1, which gives gamma_5 = diag(1,1,-1,-1) and therefore a
 * clover term that is block-diagonal in chirality (2 x 21 = 42 independent
 * complex entries, matching the 42 stored per site in Sec. 2.3).
 * Written out entry by entry below.                                     */
static void gamma_matrix(int mu, cplx g[4][4])
{
    memset(g, 0, sizeof(cplx) * 16);
    switch (mu) {
    case 0: /* T */
        g[0][2] = 1; g[1][3] = 1; g[2][0] = 1; g[3][1] = 1;
        break;
    case 1: /* Z */
        g[0][2] = -I; g[1][3] = I; g[2][0] = I; g[3][1] = -I;
        break;
    case 2: /* Y */
        g[0][3] = -1; g[1][2] = 1; g[2][1] = 1; g[3][0] = -1;
        break;
    default: /* X */
        g[0][3] = -I; g[1][2] = -I; g[2][1] = I; g[3][0] = I;
        break;
    }
}

void oracle_gamma(int mu, double *out /* [4][4] complex */)
{
    cplx g[4][4];
    gamma_matrix(mu, g);
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) {
            out[2 * (4 * a + b)] = creal(g[a][b]);
            out[2 * (4 * a + b) + 1] = cimag(g[a][b]);
        }
}

/* ------------------------------------------------------------------ */
/* lattice geometry, Eqs. (1.7)-(1.9): coordinates (t,z,y,x)           */
static long site_of(const int dims[4], const int c[4])
{
    return (((long)c[0] * dims[1] + c[1]) * dims[2] + c[2]) * dims[3] + c[3];
}

static void coords_of(const int dims[4], long i, int c[4])
{
    c[3] = (int)(i % dims[3]); i /= dims[3];
    c[2] = (int)(i % dims[2]); i /= dims[2];
    c[1] = (int)(i % dims[1]); i /= dims[1];
    c[0] = (int)i;
}

/* site x + step*mu with periodic wrap; *crossed is set when the hop passes
 * the lattice boundary in direction mu.                                  */
static long shifted(const int dims[4], long i, int mu, int step, int *crossed)
{
    int c[4];
    coords_of(dims, i, c);
    int v = c[mu] + step;
    int cr = 0;
    if (v < 0) { v += dims[mu]; cr = 1; }
    if (v >= dims[mu]) { v -= dims[mu]; cr = 1; }
    c[mu] = v;
    if (crossed) *crossed = cr;
    return site_of(dims, c);
}

/* ------------------------------------------------------------------ */
/* 3x3 complex helpers (plain loops)                                    */
static void load_link(const double *links, long site, int mu, cplx U[3][3])
{
    const double *p = links + 2 * (36 * site + 9 * mu);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            U[a][b] = p[2 * (3 * a + b)] + I * p[2 * (3 * a + b) + 1];
}

static void dagger3(cplx A[3][3], cplx out[3][3])
{
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            out[a][b] = conj(A[b][a]);
}

static void mul3(cplx A[3][3], cplx B[3][3], cplx out[3][3])
{
    cplx t[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++) s += A[a][k] * B[k][b];
            t[a][b] = s;
        }
    memcpy(out, t, sizeof(t));
}

/* product of four link matrices, each optionally daggered */
typedef struct { long site; int mu; int dag; } linkref;

static void path4(const double *links, const linkref r[4], cplx out[3][3])
{
    cplx acc[3][3], M[3][3], Md[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) acc[a][b] = (a == b);
    for (int k = 0; k < 4; k++) {
        load_link(links, r[k].site, r[k].mu, M);
        if (r[k].dag) { dagger3(M, Md); mul3(acc, Md, acc); }
        else mul3(acc, M, acc);
    }
    memcpy(out, acc, sizeof(acc));
}

/* Q_{mu nu}(x) of Eq. (1.12): the four plaquettes around x in the mu-nu
 * plane, each term copied factor by factor from the equation.           */
static void leaves(const int dims[4], const double *links, long x, int mu, int nu,
                   cplx Q[3][3])
{
    long xpm = shifted(dims, x, mu, +1, NULL);        /* x+mu        */
    long xpn = shifted(dims, x, nu, +1, NULL);        /* x+nu        */
    long xmm = shifted(dims, x, mu, -1, NULL);        /* x-mu        */
    long xmn = shifted(dims, x, nu, -1, NULL);        /* x-nu        */
    long xmm_pn = shifted(dims, xmm, nu, +1, NULL);   /* x-mu+nu     */
    long xmm_mn = shifted(dims, xmm, nu, -1, NULL);   /* x-mu-nu     */
    long xmn_pm = shifted(dims, xmn, mu, +1, NULL);   /* x-nu+mu     */
    cplx P[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) Q[a][b] = 0;

    /* U_mu(x) U_nu(x+mu) U_mu(x+nu)^H U_nu(x)^H */
    linkref l1[4] = {{x, mu, 0}, {xpm, nu, 0}, {xpn, mu, 1}, {x, nu, 1}};
    /* U_nu(x) U_mu(x-mu+nu)^H U_nu(x-mu)^H U_mu(x-mu) */
    linkref l2[4] = {{x, nu, 0}, {xmm_pn, mu, 1}, {xmm, nu, 1}, {xmm, mu, 0}};
    /* U_mu(x-mu)^H U_nu(x-mu-nu)^H U_mu(x-mu-nu) U_nu(x-nu) */
    linkref l3[4] = {{xmm, mu, 1}, {xmm_mn, nu, 1}, {xmm_mn, mu, 0}, {xmn, nu, 0}};
    /* U_nu(x-nu)^H U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^H */
    linkref l4[4] = {{xmn, nu, 1}, {xmn, mu, 0}, {xmn_pm, nu, 0}, {x, mu, 1}};
    const linkref *all[4] = {l1, l2, l3, l4};
    for (int k = 0; k < 4; k++) {
        path4(links, all[k], P);
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Q[a][b] += P[a][b];
    }
}

void oracle_leaves(const int dims[4], const double *links, long x, int mu, int nu,
                   double *out /* [3][3] complex */)
{
    cplx Q[3][3];
    leaves(dims, links, x, mu, nu, Q);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            out[2 * (3 * a + b)] = creal(Q[a][b]);
            out[2 * (3 * a + b) + 1] = cimag(Q[a][b]);
        }
}

/* full 12x12 unit-c_sw clover term at one site, Eq. (1.11):
 * C(x) = -(1/32) sum over all ordered (mu,nu) of
 *        (gamma_mu gamma_nu) (x) (Q_{mu nu}(x) - Q_{nu mu}(x))           */
static void clover_full(const int dims[4], const double *links, long x, cplx C[12][12])
{
    for (int r = 0; r < 12; r++)
        for (int s = 0; s < 12; s++) C[r][s] = 0;
    for (int mu = 0; mu < 4; mu++)
        for (int nu = 0; nu < 4; nu++) {
            cplx gm[4][4], gn[4][4], gg[4][4], Qmn[3][3], Qnm[3][3];
            gamma_matrix(mu, gm);
            gamma_matrix(nu, gn);
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    cplx s = 0;
                    for (int k = 0; k < 4; k++) s += gm[a][k] * gn[k][b];
                    gg[a][b] = s;
                }
            leaves(dims, links, x, mu, nu, Qmn);
            leaves(dims, links, x, nu, mu, Qnm);
            for (int al = 0; al < 4; al++)
                for (int be = 0; be < 4; be++)
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++)
                            C[3 * al + a][3 * be + b] +=
                                -(1.0 / 32.0) * gg[al][be] * (Qmn[a][b] - Qnm[a][b]);
        }
}

/* pack order of the 42 entries (see header) */
static void pack_pair(int k, int *r, int *s)
{
    /* k in 0..20 inside one block: 0..5 diagonal, 6..20 strict upper */
    *r = 0; *s = 0;
    if (k < 6) { *r = k; *s = k; return; }
    int n = 6;
    for (int i = 0; i < 6; i++)
        for (int j = i + 1; j < 6; j++) {
            if (n == k) { *r = i; *s = j; return; }
            n++;
        }
}

/* Unit-c_sw clover term for every site, packed as [V][42].  Returns the
 * largest modulus of an entry outside the two chirality blocks and of the
 * anti-Hermitian part inside them (both vanish for exact arithmetic), so a
 * caller can confirm the block structure the packing relies on.          */
double oracle_clover_term(const int dims[4], const double *links, double *clover)
{
    long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
    double worst = 0.0;
#pragma omp parallel for reduction(max : worst) schedule(static)
    for (long x = 0; x < V; x++) {
        cplx C[12][12];
        clover_full(dims, links, x, C);
        for (int r = 0; r < 12; r++)
            for (int s = 0; s < 12; s++) {
                double d = (r / 6 != s / 6) ? cabs(C[r][s]) : cabs(C[r][s] - conj(C[s][r]));
                if (d > worst) worst = d;
            }
        double *out = clover + 2 * 42 * x;
        for (int blk = 0; blk < 2; blk++)
            for (int k = 0; k < 21; k++) {
                int r, s;
                pack_pair(k, &r, &s);
                cplx v = C[6 * blk + r][6 * blk + s];
                out[2 * (21 * blk + k)] = creal(v);
                out[2 * (21 * blk + k) + 1] = cimag(v);
            }
    }
    return worst;
}

/* A(x) = (4 + m0) I_12 + csw * C(x), from the packed C(x)                */
static void self_matrix(const double *p /* 42 complex of one site, or NULL */, double m0,
                        double csw, cplx A[12][12])
{
    for (int r = 0; r < 12; r++)
        for (int s = 0; s < 12; s++) A[r][s] = (r == s) ? (4.0 + m0) : 0.0;
    if (!p) return;
    for (int blk = 0; blk < 2; blk++)
        for (int k = 0; k < 21; k++) {
            int r, s;
            pack_pair(k, &r, &s);
            cplx v = p[2 * (21 * blk + k)] + I * p[2 * (21 * blk + k) + 1];
            if (r == s) {
                A[6 * blk + r][6 * blk + r] += csw * creal(v);
            } else {
                A[6 * blk + r][6 * blk + s] += csw * v;
                A[6 * blk + s][6 * blk + r] += csw * conj(v);
            }
        }
}

/* (D psi)(x) at one site, Eq. (1.13) with a = 1.  dagger != 0 gives the
 * adjoint operator D^H, whose hopping blocks are the conjugate transposes
 * of D's: -1/2 (I + gamma_mu) (x) U_mu(x) psi(x+mu) and
 * -1/2 (I - gamma_mu) (x) U_mu(x-mu)^H psi(x-mu); A(x) is Hermitian.
 * antiperiodic_t != 0 multiplies every hop that crosses the T boundary
 * by -1 (anti-periodic boundary in time, Sec. 1.1).                      */
static void apply_site(const int dims[4], const double *links, const double *clover_x,
                       double m0, double csw, int antiperiodic_t, int dagger,
                       const double *in, long x, cplx out[12])
{
    cplx A[12][12];
    self_matrix(clover_x, m0, csw, A);
    const double *px = in + 2 * 12 * x;
    for (int r = 0; r < 12; r++) {
        cplx s = 0;
        for (int c = 0; c < 12; c++) s += A[r][c] * (px[2 * c] + I * px[2 * c + 1]);
        out[r] = s;
    }
    double pm = dagger ? -1.0 : 1.0;
    for (int mu = 0; mu < 4; mu++) {
        cplx g[4][4], U[3][3], W[3][3];
        gamma_matrix(mu, g);
        int cr;
        /* forward: -1/2 ((I - pm*gamma) (x) U_mu(x)) psi(x+mu) */
        long y = shifted(dims, x, mu, +1, &cr);
        double sgn = (antiperiodic_t && mu == 0 && cr) ? -1.0 : 1.0;
        load_link(links, x, mu, U);
        const double *py = in + 2 * 12 * y;
        for (int al = 0; al < 4; al++)
            for (int a = 0; a < 3; a++) {
                cplx s = 0;
                for (int be = 0; be < 4; be++)
                    for (int b = 0; b < 3; b++) {
                        cplx spin = (al == be ? 1.0 : 0.0) - pm * g[al][be];
                        s += spin * U[a][b] * (py[2 * (3 * be + b)] + I * py[2 * (3 * be + b) + 1]);
                    }
                out[3 * al + a] -= 0.5 * sgn * s;
            }
        /* backward: -1/2 ((I + pm*gamma) (x) U_mu(x-mu)^H) psi(x-mu) */
        y = shifted(dims, x, mu, -1, &cr);
        sgn = (antiperiodic_t && mu == 0 && cr) ? -1.0 : 1.0;
        load_link(links, y, mu, U);
        dagger3(U, W);
        py = in + 2 * 12 * y;
        for (int al = 0; al < 4; al++)
            for (int a = 0; a < 3; a++) {
                cplx s = 0;
                for (int be = 0; be < 4; be++)
                    for (int b = 0; b < 3; b++) {
                        cplx spin = (al == be ? 1.0 : 0.0) + pm * g[al][be];
                        s += spin * W[a][b] * (py[2 * (3 * be + b)] + I * py[2 * (3 * be + b) + 1]);
                    }
                out[3 * al + a] -= 0.5 * sgn * s;
            }
    }
}

/* out = D in (dagger = 0) or D^H in (dagger = 1) on the whole lattice.
 * clover may be NULL (c_sw term absent).  in and out must not overlap.  */
void oracle_dirac_apply(const int dims[4], const double *links, const double *clover,
                        double m0, double csw, int antiperiodic_t, int dagger,
                        const double *in, double *out)
{
    long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; x++) {
        cplx r[12];
        apply_site(dims, links, clover ? clover + 2 * 42 * x : NULL, m0, csw, antiperiodic_t,
                   dagger, in, x, r);
        for (int k = 0; k < 12; k++) {
            out[2 * (12 * x + k)] = creal(r[k]);
            out[2 * (12 * x + k) + 1] = cimag(r[k]);
        }
    }
}

/* (D in) at a list of sites only: out is [nsites][12] complex and
 * clover_at is the packed clover term of the listed sites, [nsites][42]
 * (or NULL).                                                              */
void oracle_dirac_apply_sites(const int dims[4], const double *links, const double *clover_at,
                              double m0, double csw, int antiperiodic_t, int dagger,
                              const double *in, const long *sites, long nsites, double *out)
{
#pragma omp parallel for schedule(static)
    for (long n = 0; n < nsites; n++) {
        cplx r[12];
        apply_site(dims, links, clover_at ? clover_at + 2 * 42 * n : NULL, m0, csw,
                   antiperiodic_t, dagger, in, sites[n], r);
        for (int k = 0; k < 12; k++) {
            out[2 * (12 * n + k)] = creal(r[k]);
            out[2 * (12 * n + k) + 1] = cimag(r[k]);
        }
    }
}

/* Unit-c_sw clover term at a list of sites, packed [nsites][42].        */
void oracle_clover_term_sites(const int dims[4], const double *links, const long *sites,
                              long nsites, double *clover)
{
#pragma omp parallel for schedule(static)
    for (long n = 0; n < nsites; n++) {
        cplx C[12][12];
        clover_full(dims, links, sites[n], C);
        double *out = clover + 2 * 42 * n;
        for (int blk = 0; blk < 2; blk++)
            for (int k = 0; k < 21; k++) {
                int r, s;
                pack_pair(k, &r, &s);
                cplx v = C[6 * blk + r][6 * blk + s];
                out[2 * (21 * blk + k)] = creal(v);
                out[2 * (21 * blk + k) + 1] = cimag(v);
            }
    }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* thread count of the site loops (n >= 1); for timing runs pinned to a CPU set */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Link derivative of L = Re sum_x eta(x)^H (D psi)(x) (a new quantity; the
 * paper has no force).  For a link U = U_rho(y) the derivative is
 * G = dL/dRe U + i dL/dIm U, a 3x3 complex matrix.  L is real-linear in
 * the entries of every single link, so G follows from the definition of D
 * term by term:
 *   - hopping, Eq. (1.13): U_rho(y) appears once forward (site y) and once
 *     backward (site y+rho), giving
 *       G = -1/2 sum_s eta(y)_s [(I - gamma) psi(y+rho)]_s^H
 *           -1/2 sum_s [(I + gamma) psi(y)]_s eta(y+rho)_s^H;
 *   - clover, Eqs. (1.11)-(1.12): every leaf product P = A U B containing
 *     the link contributes coef (B K A)^H, and every P = A U^H B contributes
 *     coef (B K A), with coef = -c_sw/32 (or +c_sw/32 for the Q_{nu mu}
 *     leaves) and K_{ba} = sum (gamma_mu gamma_nu)_{al,be} psi_{be b}
 *     conj(eta_{al a}) at the leaf's base site.  The leaves are enumerated
 *     literally over the sites that can contain the link.
 * F = P_TA(G U^H), P_TA(M) = (M - M^H)/2 - tr(M - M^H)/6 I.
 * Only when with_clover != 0 is the clover part added.                  */
static void clover_link_grad(const int dims[4], const double *links, double csw,
                             const double *eta, const double *psi, long y, int rho,
                             cplx G[3][3])
{
    /* candidate base sites: the 3^4 box around y (deduplicated) */
    long cand[81];
    int ncand = 0;
    for (int d0 = -1; d0 <= 1; d0++)
        for (int d1 = -1; d1 <= 1; d1++)
            for (int d2 = -1; d2 <= 1; d2++)
                for (int d3 = -1; d3 <= 1; d3++) {
                    int c[4], d[4] = {d0, d1, d2, d3};
                    coords_of(dims, y, c);
                    for (int k = 0; k < 4; k++) c[k] = ((c[k] + d[k]) % dims[k] + dims[k]) % dims[k];
                    long s = site_of(dims, c);
                    int dup = 0;
                    for (int k = 0; k < ncand; k++) if (cand[k] == s) dup = 1;
                    if (!dup) cand[ncand++] = s;
                }
    for (int ci = 0; ci < ncand; ci++) {
        long x = cand[ci];
        const double *pe = eta + 2 * 12 * x, *pp = psi + 2 * 12 * x;
        for (int mu = 0; mu < 4; mu++)
            for (int nu = 0; nu < 4; nu++) {
                if (mu == nu) continue;
                cplx gm[4][4], gn[4][4], gg[4][4], K[3][3];
                gamma_matrix(mu, gm);
                gamma_matrix(nu, gn);
                for (int a = 0; a < 4; a++)
                    for (int b = 0; b < 4; b++) {
                        cplx s = 0;
                        for (int k = 0; k < 4; k++) s += gm[a][k] * gn[k][b];
                        gg[a][b] = s;
                    }
                for (int b = 0; b < 3; b++)
                    for (int a = 0; a < 3; a++) {
                        cplx s = 0;
                        for (int al = 0; al < 4; al++)
                            for (int be = 0; be < 4; be++)
                                s += gg[al][be] * (pp[2 * (3 * be + b)] + I * pp[2 * (3 * be + b) + 1]) *
                                     conj(pe[2 * (3 * al + a)] + I * pe[2 * (3 * al + a) + 1]);
                        K[b][a] = s;
                    }
                for (int which = 0; which < 2; which++) {
                    /* which = 0: leaves of Q_{mu nu}, +; which = 1: Q_{nu mu}, - */
                    int m1 = which ? nu : mu, n1 = which ? mu : nu;
                    double coef = (which ? 1.0 : -1.0) * csw / 32.0;
                    long xpm = shifted(dims, x, m1, +1, NULL);
                    long xpn = shifted(dims, x, n1, +1, NULL);
                    long xmm = shifted(dims, x, m1, -1, NULL);
                    long xmn = shifted(dims, x, n1, -1, NULL);
                    long xmm_pn = shifted(dims, xmm, n1, +1, NULL);
                    long xmm_mn = shifted(dims, xmm, n1, -1, NULL);
                    long xmn_pm = shifted(dims, xmn, m1, +1, NULL);
                    linkref lv[4][4] = {
                        {{x, m1, 0}, {xpm, n1, 0}, {xpn, m1, 1}, {x, n1, 1}},
                        {{x, n1, 0}, {xmm_pn, m1, 1}, {xmm, n1, 1}, {xmm, m1, 0}},
                        {{xmm, m1, 1}, {xmm_mn, n1, 1}, {xmm_mn, m1, 0}, {xmn, n1, 0}},
                        {{xmn, n1, 1}, {xmn, m1, 0}, {xmn_pm, n1, 0}, {x, m1, 1}}};
                    for (int l = 0; l < 4; l++)
                        for (int pos = 0; pos < 4; pos++) {
                            if (lv[l][pos].site != y || lv[l][pos].mu != rho) continue;
                            cplx Am[3][3], Bm[3][3], M[3][3], Md[3][3], BKA[3][3];
                            for (int a = 0; a < 3; a++)
                                for (int b = 0; b < 3; b++) Am[a][b] = Bm[a][b] = (a == b);
                            for (int k = 0; k < 4; k++) {
                                if (k == pos) continue;
                                load_link(links, lv[l][k].site, lv[l][k].mu, M);
                                if (lv[l][k].dag) dagger3(M, Md); else memcpy(Md, M, sizeof(M));
                                if (k < pos) mul3(Am, Md, Am); else mul3(Bm, Md, Bm);
                            }
                            mul3(Bm, K, BKA);
                            mul3(BKA, Am, BKA);
                            for (int a = 0; a < 3; a++)
                                for (int b = 0; b < 3; b++)
                                    G[a][b] += lv[l][pos].dag ? coef * BKA[a][b] : coef * conj(BKA[b][a]);
                        }
                }
            }
    }
}

void oracle_force_links(const int dims[4], const double *links, double csw, int with_clover,
                        int antiperiodic_t, int nrhs, const double *eta, const double *psi,
                        const long *link_sites, const int *link_dirs, long nlinks,
                        double *G_out /* [nlinks][3][3] */, double *F_out /* [nlinks][3][3] */)
{
    long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
#pragma omp parallel for schedule(dynamic, 16)
    for (long n = 0; n < nlinks; n++) {
        long y = link_sites[n];
        int rho = link_dirs[n];
        cplx G[3][3], g[4][4], U[3][3], Ud[3][3], M[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) G[a][b] = 0;
        gamma_matrix(rho, g);
        int cr;
        long yp = shifted(dims, y, rho, +1, &cr);
        double sgn = (antiperiodic_t && rho == 0 && cr) ? -1.0 : 1.0;
        for (int r = 0; r < nrhs; r++) {
            const double *e = eta + 2 * 12 * V * r, *p = psi + 2 * 12 * V * r;
            for (int al = 0; al < 4; al++) {
                cplx q[3], pr[3];
                for (int b = 0; b < 3; b++) {
                    cplx s1 = 0, s2 = 0;
                    for (int be = 0; be < 4; be++) {
                        cplx m_ = (al == be ? 1.0 : 0.0) - g[al][be];
                        cplx p_ = (al == be ? 1.0 : 0.0) + g[al][be];
                        s1 += m_ * (p[2 * (12 * yp + 3 * be + b)] + I * p[2 * (12 * yp + 3 * be + b) + 1]);
                        s2 += p_ * (p[2 * (12 * y + 3 * be + b)] + I * p[2 * (12 * y + 3 * be + b) + 1]);
                    }
                    q[b] = s1;
                    pr[b] = s2;
                }
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) {
                        cplx ey = e[2 * (12 * y + 3 * al + a)] + I * e[2 * (12 * y + 3 * al + a) + 1];
                        cplx eyp = e[2 * (12 * yp + 3 * al + b)] + I * e[2 * (12 * yp + 3 * al + b) + 1];
                        G[a][b] += -0.5 * sgn * ey * conj(q[b]);
                        G[a][b] += -0.5 * sgn * pr[a] * conj(eyp);
                    }
            }
            if (with_clover) clover_link_grad(dims, links, csw, e, p, y, rho, G);
        }
        load_link(links, y, rho, U);
        dagger3(U, Ud);
        mul3(G, Ud, M);
        cplx tr = 0;
        for (int a = 0; a < 3; a++) tr += M[a][a] - conj(M[a][a]);
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                cplx f = 0.5 * (M[a][b] - conj(M[b][a])) - (a == b ? tr / 6.0 : 0.0);
                G_out[2 * (9 * n + 3 * a + b)] = creal(G[a][b]);
                G_out[2 * (9 * n + 3 * a + b) + 1] = cimag(G[a][b]);
                F_out[2 * (9 * n + 3 * a + b)] = creal(f);
                F_out[2 * (9 * n + 3 * a + b) + 1] = cimag(f);
            }
    }
}
