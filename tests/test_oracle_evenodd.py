"""Pins of the oracle's even-odd reduction (oracle/evenodd.py) against facts
fixed by linear algebra and by the free field, not by its own code.

* dense block elimination: S = D_ee - D_eo D_oo^{-1} D_oe from the dense
  matrix assembled out of the covariant differences of Eq. (1.10) plus
  Eq. (1.11) (the brute force of the operator pins), and the solution of
  D x = b from a dense solve;
* free field: a plane wave restricted to the even sites is an eigenvector of S
  with the 4 x 4 spin matrix (4 + m0) - H(p)^2 / (4 + m0), H(p) the hopping
  symbol of Eq. (1.13);
* the site-local matrices A(x) against the oracle operator minus its hopping
  part, A_oo^{-1} A_oo = 1, and the half-lattice order (index s >> 1).
"""
import numpy as np
import pytest

import oracle
from oracle import evenodd
from paper_2407_00041_amd import synth
from test_oracle_operator import G, coords, dense_brute_force, rel


def perm(dims):
    e, o = evenodd.sites_of(dims, 0), evenodd.sites_of(dims, 1)
    idx = lambda s: (12 * s[:, None] + np.arange(12)[None, :]).reshape(-1)
    return idx(e), idx(o)


@pytest.mark.parametrize("dims,antiperiodic", [((2, 2, 2, 4), False), ((4, 2, 2, 2), True)])
def test_schur_equals_dense_block_elimination(dims, antiperiodic):
    rng = np.random.default_rng(11)
    U = synth.haar_links(dims, 31)
    m0, csw = -0.2, 1.1
    D = dense_brute_force(dims, U, m0, csw, antiperiodic)
    ie, io = perm(dims)
    Dee, Deo, Doe, Doo = D[np.ix_(ie, ie)], D[np.ix_(ie, io)], D[np.ix_(io, ie)], D[np.ix_(io, io)]
    S = Dee - Deo @ np.linalg.solve(Doo, Doe)
    eo = evenodd.EvenOdd(dims, U, m0, csw, antiperiodic_t=antiperiodic)
    Vh = synth.volume(dims) // 2
    xe = rng.standard_normal((2, Vh, 12)) + 1j * rng.standard_normal((2, Vh, 12))
    for r in range(2):
        assert rel(eo.schur(xe[r]).reshape(-1), S @ xe[r].reshape(-1)) < 1e-13
        assert rel(eo.schur(xe[r], dagger=True).reshape(-1), S.conj().T @ xe[r].reshape(-1)) < 1e-13
    # the reduced system and the reconstruction reproduce the dense solve
    b = rng.standard_normal((synth.volume(dims), 12)) + 1j * rng.standard_normal((synth.volume(dims), 12))
    x = np.linalg.solve(D, b.reshape(-1)).reshape(-1, 12)
    be, bo = evenodd.split(dims, b)
    xe_ref, xo_ref = evenodd.split(dims, x)
    rhs = eo.prepare(be, bo)
    assert rel(rhs.reshape(-1), (S @ xe_ref.reshape(-1))) < 1e-12
    xe_s = np.linalg.solve(S, rhs.reshape(-1)).reshape(-1, 12)
    assert rel(xe_s, xe_ref) < 1e-12
    assert rel(eo.reconstruct(xe_s, bo), xo_ref) < 1e-12
    assert rel(evenodd.merge(dims, xe_s, eo.reconstruct(xe_s, bo)), x) < 1e-12


def test_free_field_plane_wave_is_schur_eigenvector():
    dims = (4, 6, 2, 4)
    V = synth.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3)).copy()
    m0 = -0.3
    a = 4.0 + m0
    eo = evenodd.EvenOdd(dims, U, m0, 0.0)
    rng = np.random.default_rng(5)
    c = coords(dims)
    for n in [(1, 0, 0, 0), (1, 2, 1, 3), (0, 5, 1, 1), (2, 3, 0, 2)]:
        p = 2 * np.pi * np.asarray(n) / np.asarray(dims)
        H = -np.sum(np.cos(p)) * np.eye(4, dtype=complex)
        for mu in range(4):
            H = H + 1j * np.sin(p[mu]) * G[mu]
        M = a * np.eye(4) - H @ H / a
        u = rng.standard_normal(12) + 1j * rng.standard_normal(12)
        wave = np.exp(1j * (c @ p))[:, None] * u[None, :]
        want = np.exp(1j * (c @ p))[:, None] * (M @ u.reshape(4, 3)).reshape(1, 12)
        we, _ = evenodd.split(dims, wave)
        ve, _ = evenodd.split(dims, want)
        assert rel(eo.schur(we), ve) < 1e-13


def test_site_matrices_inverse_and_order():
    dims = (4, 4, 2, 6)
    V = synth.volume(dims)
    U = synth.smooth_links(dims, 8).numpy()
    m0, csw = -0.35, 1.0
    rng = np.random.default_rng(2)
    psi = rng.standard_normal((V, 12)) + 1j * rng.standard_normal((V, 12))
    A = evenodd.site_matrices(dims, U, m0, csw)
    local = oracle.dirac_apply(dims, U, psi, m0, csw) - oracle.dirac_apply(dims, U, psi, -4.0, 0.0)
    assert rel(np.einsum("sij,sj->si", A, psi), local) < 1e-13
    eo = evenodd.EvenOdd(dims, U, m0, csw)
    assert np.max(np.abs(eo.Ainv_o @ A[eo.o] - np.eye(12))) < 1e-13
    # the parity-field order is index s >> 1 within each parity (nX even)
    for p in range(2):
        s = evenodd.sites_of(dims, p)
        assert np.array_equal(s >> 1, np.arange(V // 2))
        assert np.all(evenodd.parity(dims)[s] == p)
    with pytest.raises(ValueError):
        evenodd.EvenOdd((4, 4, 3, 2), synth.haar_links((4, 4, 3, 2), 1), m0, 0.0)


def test_reduced_fgmres_solves_the_full_system():
    dims = (4, 4, 4, 4)
    U = synth.smooth_links(dims, 21).numpy()
    m0, csw = -0.3, 1.0
    eo = evenodd.EvenOdd(dims, U, m0, csw)
    b = synth.gaussian_spinor(dims, 22)
    be, bo = evenodd.split(dims, b)
    rhs = eo.prepare(be, bo)
    xe, info = oracle.fgmres(eo.schur, rhs, 20, 1e-11, 400)
    x = evenodd.merge(dims, xe, eo.reconstruct(xe, bo))
    r = b - oracle.dirac_apply(dims, U, x, m0, csw)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-10


def test_schur_at_sites_equals_whole_lattice():
    """The neighbourhood-only evaluation used at full size agrees with the
    whole-lattice definition (also anti-periodic, and with extent 2)."""
    for dims, ap in [((4, 6, 2, 4), True), ((2, 4, 4, 2), False)]:
        U = synth.smooth_links(dims, 3).numpy()
        eo = evenodd.EvenOdd(dims, U, -0.3, 1.0, antiperiodic_t=ap)
        Vh = synth.volume(dims) // 2
        rng = np.random.default_rng(1)
        xe = rng.standard_normal((Vh, 12)) + 1j * rng.standard_normal((Vh, 12))
        want = eo.schur(xe)
        pick = np.array([0, 5, Vh // 2, Vh - 1])
        got = evenodd.schur_sites(dims, U, xe, evenodd.sites_of(dims, 0)[pick], -0.3, 1.0, antiperiodic_t=ap)
        assert rel(got, want[pick]) < 1e-14
