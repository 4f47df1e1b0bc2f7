"""Schwarz alternating procedure (SAP) for D x = b, in plain NumPy (FP64).
TEST INFRASTRUCTURE ONLY (the test-suite, the smoke check and the benchmark's
CPU-baseline leg); nothing here is shared with the GPU library.

Sec. 1.3 names the smoothers of the paper's solver library: additive,
red-black and 16-colour multiplicative Schwarz methods over non-overlapping
lattice blocks, used inside the (F)GMRES preconditioner.  The paper gives no
further detail, so the method is taken from its textbook definition (domain
decomposition with non-overlapping subdomains and local solves):

  * The lattice is cut into blocks of b_T x b_Z x b_Y x b_X sites (every
    extent divides the lattice's).  Block coordinates are the site coordinates
    divided by the block extents; a block's colour is the sum of its
    coordinates mod 2 (red-black).  For the colouring to separate the blocks
    every direction holds an even number of blocks, or exactly one (the block
    then spans that direction, and its hops in it stay inside the block).
  * D_B, the block operator, is D restricted to the block's sites: the hops
    of Eq. (1.13) whose neighbour lies outside the block are dropped
    (homogeneous Dirichlet boundary).  D_B rho for rho on the block equals
    (D rho_ext) at the block's sites, rho_ext being rho extended by zero.
  * Local solve M_B ~ D_B^{-1}: ``mr_iters`` steps of the minimal-residual
    iteration from e = 0, or an exact dense solve (tiny blocks only):
        rho = r_B, e = 0;  repeat:  q = D_B rho;  alpha = <q, rho> / <q, q>;
        e += alpha rho;  rho -= alpha q          (<a, b> = a^H b)
    alpha minimises |rho - alpha q|.
  * One multiplicative (red-black) cycle: for colour c = 0, 1 in turn,
    r = b - D x, then x_B += M_B r_B on every block B of colour c.
    One additive cycle: r = b - D x once, then x_B += M_B r_B on every block.
  * The preconditioner of FGMRES applies ``cycles`` cycles from x = 0.

A block's sites are listed in lexicographic order of its local coordinates
(local x fastest), which is also the order of the full lattice.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import clover_term_sites, dirac_apply, dirac_apply_sites, volume


def check_blocking(dims, bdims) -> np.ndarray:
    """Number of blocks per direction; raises unless every extent divides and
    each direction holds an even number of blocks or exactly one."""
    dims = np.asarray(dims, np.int64)
    b = np.asarray(bdims, np.int64)
    if b.shape != (4,) or np.any(b < 1) or np.any(dims % b):
        raise ValueError(f"block extents {tuple(b)} must divide the lattice {tuple(dims)}")
    nb = dims // b
    if np.any((nb % 2 == 1) & (nb != 1)):
        raise ValueError(f"{tuple(nb)} blocks per direction: each count must be even or 1 for red-black colouring")
    return nb


def block_list(dims, bdims):
    """[(colour, sites)] for every block, block coordinates in lexicographic order."""
    nb = check_blocking(dims, bdims)
    n = np.asarray(dims, np.int64)
    b = np.asarray(bdims, np.int64)
    local = np.array(list(itertools.product(*[range(int(k)) for k in b])), np.int64)  # local x fastest
    out = []
    for bc in itertools.product(*[range(int(k)) for k in nb]):
        c = local + np.asarray(bc, np.int64) * b
        sites = ((c[:, 0] * n[1] + c[:, 1]) * n[2] + c[:, 2]) * n[3] + c[:, 3]
        out.append((int(sum(bc)) % 2, sites))
    return out


class Schwarz:
    """SAP for one operator D(U, m0, csw) and one blocking."""

    def __init__(self, dims, links, m0: float, csw: float, bdims, clover=None, antiperiodic_t: bool = False):
        self.dims = tuple(int(d) for d in dims)
        self.V = volume(self.dims)
        self.U = links
        self.m0, self.csw = float(m0), float(csw)
        self.ap = bool(antiperiodic_t)
        self.clover = clover
        self.blocks = block_list(self.dims, bdims)
        self._rows = {}

    def _clover_rows(self, k, sites):
        if self.csw == 0.0:
            return None
        if k not in self._rows:
            self._rows[k] = (clover_term_sites(self.dims, self.U, sites) if self.clover is None
                             else np.asarray(self.clover).reshape(self.V, 42)[sites])
        return self._rows[k]

    def residual(self, b, x):
        return b - dirac_apply(self.dims, self.U, x, self.m0, self.csw, clover=self.clover, antiperiodic_t=self.ap)

    def block_apply(self, k, rho):
        """D_B rho for block k (rho: [n_B, 12])."""
        sites = self.blocks[k][1]
        ext = np.zeros((self.V, 12), np.complex128)
        ext[sites] = rho
        return dirac_apply_sites(self.dims, self.U, ext, sites, self.m0, self.csw, antiperiodic_t=self.ap,
                                 clover_rows=self._clover_rows(k, sites))

    def block_dense(self, k):
        """D_B as a dense matrix (columns = D_B applied to unit vectors)."""
        n = 12 * len(self.blocks[k][1])
        cols = [self.block_apply(k, e.reshape(-1, 12)).ravel() for e in np.eye(n, dtype=np.complex128)]
        return np.stack(cols, axis=1)

    def mr(self, k, r, iters: int):
        """Minimal-residual iterations on D_B e = r from e = 0."""
        e = np.zeros_like(r)
        rho = r.copy()
        for _ in range(iters):
            q = self.block_apply(k, rho)
            qq = np.vdot(q.ravel(), q.ravel()).real
            alpha = np.vdot(q.ravel(), rho.ravel()) / qq if qq > 0 else 0.0
            e = e + alpha * rho
            rho = rho - alpha * q
        return e

    def local_solve(self, k, r, mr_iters: int, exact: bool):
        if exact:
            return np.linalg.solve(self.block_dense(k), r.ravel()).reshape(r.shape)
        return self.mr(k, r, mr_iters)

    def apply(self, b, cycles: int = 1, mr_iters: int = 4, additive: bool = False, exact: bool = False,
              x0=None):
        """x after `cycles` Schwarz cycles on D x = b from x0 (default 0); b: [V, 12]."""
        b = np.asarray(b, np.complex128).reshape(self.V, 12)
        x = np.zeros_like(b) if x0 is None else np.array(x0, np.complex128).reshape(self.V, 12)
        for _ in range(cycles):
            if additive:
                r = self.residual(b, x)
                upd = [(self.blocks[k][1], self.local_solve(k, r[self.blocks[k][1]], mr_iters, exact))
                       for k in range(len(self.blocks))]
                for sites, e in upd:
                    x[sites] += e
                continue
            for colour in (0, 1):
                r = self.residual(b, x)
                for k, (c, sites) in enumerate(self.blocks):
                    if c == colour:
                        x[sites] += self.local_solve(k, r[sites], mr_iters, exact)
        return x

    def first_pass_at(self, k, b, mr_iters: int):
        """x on block k after the colour-0 pass of the first cycle from x = 0
        (block k of colour 0): M_B b_B, which needs only the block's data."""
        assert self.blocks[k][0] == 0
        return self.mr(k, np.asarray(b)[self.blocks[k][1]], mr_iters)

    def second_pass_at(self, k, b, x_colour0, mr_iters: int):
        """x on block k (colour 1) after the first cycle, given x after the
        colour-0 pass (zero on colour-1 blocks): M_B (b - D x)_B, with D x
        evaluated at the block's sites only."""
        assert self.blocks[k][0] == 1
        sites = self.blocks[k][1]
        dx = dirac_apply_sites(self.dims, self.U, x_colour0, sites, self.m0, self.csw, antiperiodic_t=self.ap,
                               clover_rows=self._clover_rows(k, sites))
        return self.mr(k, np.asarray(b)[sites] - dx, mr_iters)
