"""Two-level aggregation multigrid preconditioner for D x = b, FP64 NumPy.
TEST INFRASTRUCTURE ONLY (the test-suite, the smoke check and the benchmark's
CPU-baseline leg); nothing here is shared with the GPU library.

Sec. 1.3 describes the method only in outline: a coarse operator D_c that
acts like D on the near kernel (the span of eigenvectors with small
|eigenvalue|, which the Schwarz smoother reduces poorly) and keeps D's
nearest-neighbour structure; a restriction R and a prolongation P between
the lattice and the coarse lattice; the subspace correction
z <- z + P D_c^{-1} R r, which together with the smoother approximates the
solution of D z = v; and a setup phase that approximates right eigenvectors
of small eigenvalues to build P and R.  Sec. 5.1 (Table 5.2) fixes the
remaining knobs of the paper's runs: the depth-1 (coarse) lattice size, 24
test vectors and 4 setup iterations.  The readings below make that outline a
definite algorithm (each is also listed in the design notes):

  * Aggregates are lattice blocks of a_T x a_Z x a_Y x a_X sites (each extent
    divides the lattice's); the coarse lattice has one site per aggregate,
    in lexicographic order of the block coordinates (x fastest).
  * Chirality: spins 0, 1 (gamma_5 = +1, components 0..5 of a site's 12) and
    spins 2, 3 (gamma_5 = -1, components 6..11).
  * P from N test vectors v_1..v_N: for every aggregate a and chirality s the
    restrictions of v_1..v_N to (a, s) are orthonormalised in order (plain
    Gram-Schmidt: the Q factor whose R has a positive real diagonal).  Column
    (a, s, k) of P is the k-th of them; its support is (a, s).  R = P^H and
    D_c = P^H D P (Galerkin).  P is kept as N fine fields q_k (q_k restricted
    to (a, s) is column (a, s, k)).
  * Coarse vectors are [V_c, 2, N]: coarse site, chirality, test vector.
  * Two-level preconditioner M r: coarse-grid correction e = P D_c^{-1} P^H r
    (D_c^{-1} exact, or GMRES to a relative tolerance), then post-smoothing
    z = e + SAP(r - D e) (SAP from zero as in ``oracle.sap``).
  * Setup: the caller draws the initial test vectors (Gaussian); then
    ``init_iters`` times v_k <- SAP(v_k) / |SAP(v_k)| (inverse iteration with
    the smoother as approximate inverse), build P and D_c; then
    ``setup_iters`` times v_k <- M v_k / |M v_k| with the current two-level
    method, rebuilding P and D_c after each pass over the test vectors.
"""
from __future__ import annotations

import numpy as np

from . import dirac_apply, volume
from .fgmres import fgmres
from .sap import Schwarz

CHI = (np.arange(6), np.arange(6, 12))    # components of chirality + and -


def coarse_dims(dims, agg):
    d = np.asarray(dims, np.int64)
    a = np.asarray(agg, np.int64)
    if a.shape != (4,) or np.any(a < 1) or np.any(d % a):
        raise ValueError(f"aggregate extents {tuple(a)} must divide the lattice {tuple(d)}")
    return tuple(int(v) for v in d // a)


def aggregate_of(dims, agg) -> np.ndarray:
    """Coarse site (aggregate index) of every lexicographic fine site."""
    nc = coarse_dims(dims, agg)
    n = [int(v) for v in dims]
    t, z, y, x = np.meshgrid(*[np.arange(k) for k in n], indexing="ij")
    a = [int(v) for v in agg]
    ct, cz, cy, cx = t // a[0], z // a[1], y // a[2], x // a[3]
    return (((ct * nc[1] + cz) * nc[2] + cy) * nc[3] + cx).reshape(-1)


def orthonormalise(W: np.ndarray) -> np.ndarray:
    """Gram-Schmidt of the columns of W in order (each new column made
    orthogonal to the previous ones, then normalised): the Q of W = QR with a
    positive real diagonal of R.  Raises when a column is (numerically)
    dependent on the previous ones."""
    Q = np.array(W, np.complex128)
    for k in range(Q.shape[1]):
        for j in range(k):
            Q[:, k] -= np.vdot(Q[:, j], Q[:, k]) * Q[:, j]
        nk = np.linalg.norm(Q[:, k])
        if not nk > 1e-12 * max(np.linalg.norm(W[:, k]), 1e-300):
            raise ValueError(f"test vector {k} is linearly dependent on the previous ones on an aggregate")
        Q[:, k] /= nk
    return Q


class TwoLevel:
    """P, R = P^H and D_c for one operator D(U, m0, csw), aggregation and set of
    test vectors, and the two-level preconditioner built from them."""

    def __init__(self, dims, links, m0: float, csw: float, agg, testvecs, clover=None, antiperiodic_t: bool = False,
                 sap_block=(2, 2, 2, 2), sap_cycles: int = 1, sap_mr: int = 4, sap_additive: bool = False):
        self.dims = tuple(int(d) for d in dims)
        self.V = volume(self.dims)
        self.U = links
        self.m0, self.csw = float(m0), float(csw)
        self.clover = clover
        self.ap = bool(antiperiodic_t)
        self.agg = tuple(int(a) for a in agg)
        self.cdims = coarse_dims(self.dims, self.agg)
        self.Vc = volume(self.cdims)
        self.amap = aggregate_of(self.dims, self.agg)
        self.members = [np.nonzero(self.amap == a)[0] for a in range(self.Vc)]   # increasing site order
        self.sap_block = tuple(int(b) for b in sap_block)
        self.sap = None       # built on first use (the blocking is only checked when smoothing)
        self.sap_kw = dict(cycles=int(sap_cycles), mr_iters=int(sap_mr), additive=bool(sap_additive))
        self.build(testvecs)

    # -- operators on fine fields [V, 12] -----------------------------------
    def D(self, psi):
        return dirac_apply(self.dims, self.U, psi, self.m0, self.csw, clover=self.clover, antiperiodic_t=self.ap)

    def smooth(self, r):
        if self.sap is None:
            self.sap = Schwarz(self.dims, self.U, self.m0, self.csw, self.sap_block, clover=self.clover,
                               antiperiodic_t=self.ap)
        return self.sap.apply(r, **self.sap_kw)

    # -- interpolation ------------------------------------------------------
    def build(self, testvecs):
        """P (as N fine fields) and the dense D_c from test vectors [N, V, 12]."""
        T = np.asarray(testvecs, np.complex128).reshape(-1, self.V, 12)
        self.N = T.shape[0]
        if self.N > 6 * min(len(m) for m in self.members):
            raise ValueError("more test vectors than an aggregate's chirality block has components")
        self.test = T.copy()
        q = np.zeros_like(T)
        for sites in self.members:
            for comps in CHI:
                W = T[:, sites][:, :, comps].reshape(self.N, -1).T        # (sites x 6) rows, N columns
                Q = orthonormalise(W)
                q[:, sites[:, None], comps[None, :]] = Q.T.reshape(self.N, len(sites), 6)
        self.q = q
        self.Dc = None

    def restrict(self, f):
        """c = P^H f: c[a, s, k] = sum over sites x of a and components of s of conj(q_k(x)) f(x)."""
        f = np.asarray(f, np.complex128).reshape(self.V, 12)
        c = np.zeros((self.Vc, 2, self.N), np.complex128)
        for a, sites in enumerate(self.members):
            for s, comps in enumerate(CHI):
                qa = self.q[:, sites][:, :, comps].reshape(self.N, -1)
                c[a, s] = qa.conj() @ f[sites][:, comps].reshape(-1)
        return c

    def prolong(self, c):
        """f = P c: f(x) on the components of s = sum_k q_k(x) c[a(x), s, k]."""
        c = np.asarray(c, np.complex128).reshape(self.Vc, 2, self.N)
        f = np.zeros((self.V, 12), np.complex128)
        for a, sites in enumerate(self.members):
            for s, comps in enumerate(CHI):
                qa = self.q[:, sites][:, :, comps]                         # [N, n_a, 6]
                f[sites[:, None], comps[None, :]] = np.einsum("kis,k->is", qa, c[a, s])
        return f

    def coarse_matrix(self):
        """Dense D_c = P^H D P, column by column: column j = P^H D (P e_j)."""
        if self.Dc is None:
            nc = self.Vc * 2 * self.N
            cols = np.zeros((nc, nc), np.complex128)
            E = np.eye(nc, dtype=np.complex128)
            for j in range(nc):
                cols[:, j] = self.restrict(self.D(self.prolong(E[j]))).ravel()
            self.Dc = cols
        return self.Dc

    def coarse_apply(self, c):
        return (self.coarse_matrix() @ np.asarray(c, np.complex128).ravel()).reshape(self.Vc, 2, self.N)

    def coarse_solve(self, rc, tol=None, restart: int = 30, maxit: int = 10000):
        """D_c^{-1} rc exactly (tol None), or FGMRES(restart) without preconditioner to the relative tolerance."""
        rc = np.asarray(rc, np.complex128).reshape(-1)
        if tol is None:
            return np.linalg.solve(self.coarse_matrix(), rc).reshape(self.Vc, 2, self.N)
        Dc = self.coarse_matrix()
        x, _ = fgmres(lambda v: Dc @ v, rc, m=restart, tol=tol, maxit=maxit)
        return x.reshape(self.Vc, 2, self.N)

    # -- the two-level method -----------------------------------------------
    def coarse_correction(self, r, tol=None):
        return self.prolong(self.coarse_solve(self.restrict(r), tol))

    def precond(self, r, tol=None):
        """M r: e = P D_c^{-1} P^H r, then z = e + SAP(r - D e)."""
        r = np.asarray(r, np.complex128).reshape(self.V, 12)
        e = self.coarse_correction(r, tol)
        return e + self.smooth(r - self.D(e))


def setup(dims, links, m0, csw, agg, initial, init_iters: int = 2, setup_iters: int = 1, coarse_tol=None,
          **kw) -> TwoLevel:
    """The setup phase: smoothed initial test vectors, then two-level setup iterations (see the module text)."""
    T = np.array(initial, np.complex128).reshape(-1, volume(dims), 12)
    tl = TwoLevel(dims, links, m0, csw, agg, T, **kw)
    for _ in range(init_iters):
        for k in range(T.shape[0]):
            v = tl.smooth(T[k])
            T[k] = v / np.linalg.norm(v)
    tl.build(T)
    for _ in range(setup_iters):
        for k in range(T.shape[0]):
            v = tl.precond(T[k], coarse_tol)
            T[k] = v / np.linalg.norm(v)
        tl.build(T)
    return tl
