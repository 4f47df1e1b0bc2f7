"""Even-odd (red-black) reduction of the Wilson-clover system, FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Red-black ordering is one of the site splittings the paper's solver library
offers for its Schwarz smoothers (Sec. 1.3); here it is applied to the whole
operator.  Sites of parity p = (t + z + y + x) mod 2 are listed in increasing
lexicographic order; a parity field has shape [..., V/2, 12].  Writing
D = A + H with A(x) the site-local term of Eq. (1.13) (mass plus the clover
term of Eqs. (1.11)-(1.12)) and H the hopping sum, which only couples sites of
opposite parity, block elimination of the odd sites gives

    S x_e = b_e - H_eo A_oo^{-1} b_o,    S = A_ee - H_eo A_oo^{-1} H_oe,
    x_o   = A_oo^{-1} (b_o - H_oe x_e),

and S^H = A_ee - (H^H)_eo A_oo^{-1} (H^H)_oe (A is Hermitian).

Every step is a plain definition: H is the oracle operator with 4 + m0 = 0 and
no clover term, A(x) is unpacked from the packed clover term, and A^{-1} is a
dense 12 x 12 solve per site.
"""
from __future__ import annotations

import numpy as np

from . import clover_term, clover_term_sites, dirac_apply, dirac_apply_sites, volume


def parity(dims) -> np.ndarray:
    """(t + z + y + x) mod 2 for every lexicographic site."""
    nT, nZ, nY, nX = (int(d) for d in dims)
    t, z, y, x = np.meshgrid(np.arange(nT), np.arange(nZ), np.arange(nY), np.arange(nX), indexing="ij")
    return ((t + z + y + x) % 2).reshape(-1)


def sites_of(dims, p: int) -> np.ndarray:
    """Lexicographic sites of parity p in increasing order (the parity-field order)."""
    return np.nonzero(parity(dims) == p)[0]


def split(dims, psi):
    """Full field [..., V, 12] -> (even, odd) parity fields."""
    return psi[..., sites_of(dims, 0), :], psi[..., sites_of(dims, 1), :]


def merge(dims, even, odd):
    """(even, odd) parity fields -> full field."""
    V = volume(dims)
    out = np.zeros(even.shape[:-2] + (V, 12), np.complex128)
    out[..., sites_of(dims, 0), :] = even
    out[..., sites_of(dims, 1), :] = odd
    return out


def site_matrices(dims, links, m0: float, csw: float, clover=None) -> np.ndarray:
    """A(x) = (4 + m0) I_12 + csw C(x) for every site, [V, 12, 12].

    C(x) is the packed unit-c_sw term (chirality block + on spins 0, 1, then
    block - on spins 2, 3; 6 real diagonal entries, then the 15 strict-upper
    entries in row-major pair order; block-local index 3 (sigma mod 2) + c).
    """
    V = volume(dims)
    if clover is None:
        clover = clover_term(dims, links) if csw != 0.0 else np.zeros((V, 42), np.complex128)
    return _matrices_from_rows(np.asarray(clover, np.complex128).reshape(V, 42), m0, csw)


def _matrices_from_rows(C, m0: float, csw: float) -> np.ndarray:
    V = C.shape[0]
    A = np.zeros((V, 12, 12), np.complex128)
    iu = np.triu_indices(6, 1)
    for blk in range(2):
        B = np.zeros((V, 6, 6), np.complex128)
        packed = C[:, 21 * blk:21 * (blk + 1)]
        B[:, np.arange(6), np.arange(6)] = packed[:, :6].real
        B[:, iu[0], iu[1]] = packed[:, 6:]
        B[:, iu[1], iu[0]] = np.conj(packed[:, 6:])
        A[:, 6 * blk:6 * blk + 6, 6 * blk:6 * blk + 6] = csw * B
    A += (4.0 + m0) * np.eye(12)
    return A


class EvenOdd:
    """The reduced system of one operator D(U, m0, csw)."""

    def __init__(self, dims, links, m0: float, csw: float = 0.0, clover=None, antiperiodic_t: bool = False):
        self.dims = tuple(int(d) for d in dims)
        if any(d % 2 for d in self.dims):
            raise ValueError("even-odd splitting needs every lattice extent even")
        self.V = volume(self.dims)
        self.U = links
        self.ap = bool(antiperiodic_t)
        if clover is None and csw != 0.0:
            clover = clover_term(self.dims, links)
        self.A = site_matrices(self.dims, links, m0, csw, clover)
        self.e, self.o = sites_of(self.dims, 0), sites_of(self.dims, 1)
        self.Ainv_o = np.linalg.inv(self.A[self.o])

    def hop(self, psi, dagger=False):
        """H psi (or H^H psi) on full fields: D with 4 + m0 = 0 and no clover term."""
        return dirac_apply(self.dims, self.U, psi, -4.0, 0.0, None, self.ap, dagger)

    def _to_full(self, f, sites):
        out = np.zeros(f.shape[:-2] + (self.V, 12), np.complex128)
        out[..., sites, :] = f
        return out

    def hop_oe(self, xe, dagger=False):
        """(H x)_o for x supported on even sites."""
        return self.hop(self._to_full(xe, self.e), dagger)[..., self.o, :]

    def hop_eo(self, xo, dagger=False):
        """(H x)_e for x supported on odd sites."""
        return self.hop(self._to_full(xo, self.o), dagger)[..., self.e, :]

    def ainv_o(self, fo):
        return np.einsum("sij,...sj->...si", self.Ainv_o, fo)

    def a_e(self, fe):
        return np.einsum("sij,...sj->...si", self.A[self.e], fe)

    def schur(self, xe, dagger=False):
        """S x_e, S = A_ee - H_eo A_oo^{-1} H_oe (or S^H)."""
        return self.a_e(xe) - self.hop_eo(self.ainv_o(self.hop_oe(xe, dagger)), dagger)

    def prepare(self, be, bo):
        """Right-hand side of the reduced system: b_e - H_eo A_oo^{-1} b_o."""
        return be - self.hop_eo(self.ainv_o(bo))

    def reconstruct(self, xe, bo):
        """x_o = A_oo^{-1} (b_o - H_oe x_e)."""
        return self.ainv_o(bo - self.hop_oe(xe))


def neighbours(dims, sites) -> np.ndarray:
    """[n, 8] lexicographic neighbours (x + mu, x - mu for mu = T, Z, Y, X) of the listed sites."""
    n = np.asarray(dims, np.int64)
    s = np.asarray(sites, np.int64)
    c = np.stack([s // (n[1] * n[2] * n[3]), (s // (n[2] * n[3])) % n[1], (s // n[3]) % n[2], s % n[3]], -1)
    out = []
    for mu in range(4):
        for d in (1, -1):
            cc = c.copy()
            cc[:, mu] = (cc[:, mu] + d) % n[mu]
            out.append(((cc[:, 0] * n[1] + cc[:, 1]) * n[2] + cc[:, 2]) * n[3] + cc[:, 3])
    return np.stack(out, -1)


def schur_sites(dims, links, xe, sites, m0: float, csw: float, antiperiodic_t: bool = False) -> np.ndarray:
    """(S x_e) at the listed even sites (full-lattice indices), [n, 12], computed
    from their neighbourhood only: t_o = A_oo^{-1} (H x_e) at the odd
    neighbours, then A(x) x_e(x) - (H t_o)(x).  For lattices too large for the
    whole-lattice class above."""
    V = volume(dims)
    sites = np.asarray(sites, np.int64)
    assert np.all(parity(dims)[sites] == 0)
    full = np.zeros((V, 12), np.complex128)
    full[sites_of(dims, 0)] = xe
    odd = np.unique(neighbours(dims, sites))
    h = dirac_apply_sites(dims, links, full, odd, -4.0, 0.0, antiperiodic_t=antiperiodic_t)
    Co = clover_term_sites(dims, links, odd) if csw != 0.0 else np.zeros((len(odd), 42), np.complex128)
    t = np.linalg.solve(_matrices_from_rows(Co, m0, csw), h[..., None])[..., 0]
    tf = np.zeros((V, 12), np.complex128)
    tf[odd] = t
    ht = dirac_apply_sites(dims, links, tf, sites, -4.0, 0.0, antiperiodic_t=antiperiodic_t)
    Ce = clover_term_sites(dims, links, sites) if csw != 0.0 else np.zeros((len(sites), 42), np.complex128)
    return np.einsum("sij,sj->si", _matrices_from_rows(Ce, m0, csw), full[sites]) - ht
