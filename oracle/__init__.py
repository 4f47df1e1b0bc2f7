"""FP64 CPU oracle for the Wilson-clover Dirac operator and FGMRES.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here is shared with the GPU
library (no code, header, table or helper), and this package never imports it.

- ``oracle.c`` (plain C, OpenMP over sites): the operator of Eq. (1.13) with
  the clover term of Eqs. (1.11)-(1.12), its adjoint, and the exact link
  derivative of L = Re<eta, D(U) psi>.
- ``fgmres.py`` (NumPy): Algorithm 2 (FGMRES) of Sec. 1.2.
- ``evenodd.py`` (NumPy): the even-odd (red-black) reduction of D x = b to
  the even sites (Schur complement, right-hand side, odd-site reconstruction).
- ``sap.py`` (NumPy): the Schwarz alternating procedure over non-overlapping
  lattice blocks (red-black multiplicative and additive; minimal-residual or
  exact block solves), the preconditioner of Sec. 1.3.
- ``amg.py`` (NumPy): the two-level aggregation multigrid of Sec. 1.3
  (test-vector setup, interpolation P, Galerkin coarse operator D_c = P^H D P,
  coarse-grid correction followed by SAP post-smoothing).

All arrays use the canonical host layouts documented in ``oracle.c``:
spinors [..., V, 12] complex128, links [V, 4, 3, 3] complex128, packed clover
[V, 42] complex128.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (in-tree)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", _SO + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        L.oracle_dirac_apply.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, P, P]
        L.oracle_dirac_apply.restype = None
        L.oracle_dirac_apply_sites.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_int, ctypes.c_int, P, P,
                                               ctypes.c_long, P]
        L.oracle_dirac_apply_sites.restype = None
        L.oracle_clover_term.argtypes = [P, P, P]
        L.oracle_clover_term.restype = ctypes.c_double
        L.oracle_clover_term_sites.argtypes = [P, P, P, ctypes.c_long, P]
        L.oracle_clover_term_sites.restype = None
        L.oracle_leaves.argtypes = [P, P, ctypes.c_long, ctypes.c_int, ctypes.c_int, P]
        L.oracle_leaves.restype = None
        L.oracle_gamma.argtypes = [ctypes.c_int, P]
        L.oracle_gamma.restype = None
        L.oracle_force_links.argtypes = [P, P, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, P, P, P, P, ctypes.c_long, P, P]
        L.oracle_force_links.restype = None
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(dims) -> np.ndarray:
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    assert d.shape == (4,) and (d >= 1).all()
    return d


def _c128(a, shape_tail) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    assert a.shape[-len(shape_tail):] == tuple(shape_tail), (a.shape, shape_tail)
    return a


def volume(dims) -> int:
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def gamma(mu: int) -> np.ndarray:
    """4x4 gamma_mu (mu = 0..3 for T,Z,Y,X) in the oracle's basis."""
    out = np.zeros((4, 4), np.complex128)
    lib().oracle_gamma(int(mu), _p(out))
    return out


def clover_term(dims, links) -> np.ndarray:
    """Unit-c_sw clover term C(x) of Eq. (1.11), packed [V, 42]."""
    d = _dims(dims)
    V = volume(d)
    U = _c128(links, (4, 3, 3)).reshape(V, 4, 3, 3)
    out = np.zeros((V, 42), np.complex128)
    worst = lib().oracle_clover_term(_p(d), _p(U), _p(out))
    # the packing keeps two Hermitian chirality blocks; anything else must vanish
    assert worst < 1e-10, f"clover term not block-diagonal Hermitian: {worst}"
    return out


def clover_term_sites(dims, links, sites) -> np.ndarray:
    d = _dims(dims)
    V = volume(d)
    U = _c128(links, (4, 3, 3)).reshape(V, 4, 3, 3)
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    out = np.zeros((len(s), 42), np.complex128)
    lib().oracle_clover_term_sites(_p(d), _p(U), _p(s), len(s), _p(out))
    return out


def leaves(dims, links, site: int, mu: int, nu: int) -> np.ndarray:
    d = _dims(dims)
    V = volume(d)
    U = _c128(links, (4, 3, 3)).reshape(V, 4, 3, 3)
    out = np.zeros((3, 3), np.complex128)
    lib().oracle_leaves(_p(d), _p(U), int(site), int(mu), int(nu), _p(out))
    return out


def dirac_apply(dims, links, psi, m0: float, csw: float = 0.0, clover=None,
                antiperiodic_t: bool = False, dagger: bool = False) -> np.ndarray:
    """D psi (or D^H psi) for psi of shape [V, 12] or [nrhs, V, 12].

    ``clover`` is the packed unit-c_sw term [V, 42]; if None and csw != 0 it is
    built from the links first (Eqs. 1.11-1.12).
    """
    d = _dims(dims)
    V = volume(d)
    U = _c128(links, (4, 3, 3)).reshape(V, 4, 3, 3)
    if clover is None and csw != 0.0:
        clover = clover_term(d, U)
    C = None if clover is None else _c128(clover, (42,)).reshape(V, 42)
    x = _c128(psi, (V, 12))
    batch = x.reshape(-1, V, 12)
    out = np.empty_like(batch)
    for r in range(batch.shape[0]):
        xr = np.ascontiguousarray(batch[r])
        lib().oracle_dirac_apply(_p(d), _p(U), None if C is None else _p(C), float(m0),
                                 float(csw), int(bool(antiperiodic_t)), int(bool(dagger)),
                                 _p(xr), _p(out[r]))
    return out.reshape(x.shape)


def dirac_apply_sites(dims, links, psi, sites, m0: float, csw: float = 0.0, clover=None,
                      antiperiodic_t: bool = False, dagger: bool = False,
                      clover_rows=None) -> np.ndarray:
    """(D psi)(x) at the listed sites only; returns [len(sites), 12].

    ``clover`` may be the full packed [V, 42] array or None (then, if csw != 0,
    the clover term is built at the listed sites only); ``clover_rows`` may
    instead give the packed term of the listed sites, [len(sites), 42].
    """
    d = _dims(dims)
    V = volume(d)
    U = _c128(links, (4, 3, 3)).reshape(V, 4, 3, 3)
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    x = _c128(psi, (V, 12)).reshape(V, 12)
    out = np.zeros((len(s), 12), np.complex128)
    if clover_rows is not None:
        C = _c128(clover_rows, (42,)).reshape(len(s), 42)
    elif clover is None:
        # A(x) enters at the output site only: build C there and nowhere else
        C = clover_term_sites(d, U, s) if csw != 0.0 else None
    else:
        C = np.ascontiguousarray(_c128(clover, (42,)).reshape(V, 42)[s])
    lib().oracle_dirac_apply_sites(_p(d), _p(U), None if C is None else _p(C), float(m0),
                                   float(csw), int(bool(antiperiodic_t)), int(bool(dagger)),
                                   _p(x), _p(s), len(s), _p(out))
    return out


def force_links(dims, links, eta, psi, link_sites, link_dirs, csw: float = 0.0,
                with_clover: bool = True, antiperiodic_t: bool = False):
    """Exact link derivative of L = Re sum_r <eta_r, D(U) psi_r>.

    Returns (G, F) of shape [n, 3, 3]: G = dL/dRe U + i dL/dIm U and the
    su(3) projection F = P_TA(G U^H).
    """
    d = _dims(dims)
    V = volume(d)
    U = _c128(links, (4, 3, 3)).reshape(V, 4, 3, 3)
    e = _c128(eta, (V, 12)).reshape(-1, V, 12)
    p = _c128(psi, (V, 12)).reshape(-1, V, 12)
    assert e.shape == p.shape
    s = np.ascontiguousarray(np.asarray(link_sites, dtype=np.int64))
    m = np.ascontiguousarray(np.asarray(link_dirs, dtype=np.int32))
    assert s.shape == m.shape
    G = np.zeros((len(s), 3, 3), np.complex128)
    F = np.zeros((len(s), 3, 3), np.complex128)
    lib().oracle_force_links(_p(d), _p(U), float(csw), int(bool(with_clover) and csw != 0.0),
                             int(bool(antiperiodic_t)), e.shape[0], _p(e), _p(p), _p(s), _p(m),
                             len(s), _p(G), _p(F))
    return G, F


from .fgmres import fgmres  # noqa: E402,F401
