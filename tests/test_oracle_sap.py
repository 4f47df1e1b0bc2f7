"""Pins of the oracle's Schwarz alternating procedure (oracle/sap.py) to facts
that do not come from the oracle itself: the textbook multiplicative and
additive Schwarz iterations written with dense matrices of the brute-force
operator (Eq. (1.10) from covariant differences), the whole-lattice block
(one cycle = D^{-1}), single-site blocks (the site-local term and the
even-odd block Gauss-Seidel), the minimal-residual step's orthogonality, and
the vanishing residual on the last-solved colour."""
import numpy as np
import pytest

import oracle
from oracle import evenodd, sap
from paper_2407_00041_amd import synth
from test_oracle_operator import dense_brute_force


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def inputs(dims, seed):
    U = synth.smooth_links(dims, seed).numpy()
    b = synth.gaussian_spinor(dims, seed + 1)
    return U, b


def colour_dofs(dims, bdims, colour):
    idx = []
    for c, sites in sap.block_list(dims, bdims):
        if c == colour:
            idx.extend((12 * sites[:, None] + np.arange(12)[None, :]).ravel())
    return np.sort(np.array(idx))


@pytest.mark.parametrize("dims,bdims,ap", [((2, 2, 2, 4), (2, 2, 2, 2), False),
                                           ((4, 2, 2, 4), (2, 2, 2, 2), True),
                                           ((4, 2, 2, 2), (2, 2, 1, 2), False)])
def test_multiplicative_and_additive_equal_dense_definition(dims, bdims, ap):
    """x <- x + R_c^T D_cc^{-1} R_c (b - D x) for c = 0, 1 (and the additive
    form with one shared residual), with dense D from the brute-force builder
    and D_cc its restriction to the colour's sites, equals the oracle's
    block-by-block SAP with exact local solves, over two cycles."""
    m0, csw = -0.3, 1.0
    U, b = inputs(dims, 31)
    D = dense_brute_force(dims, U, m0, csw, antiperiodic=ap)
    bv = b.ravel()
    xm = np.zeros_like(bv)
    xa = np.zeros_like(bv)
    idx = [colour_dofs(dims, bdims, c) for c in (0, 1)]
    for _ in range(2):
        for c in (0, 1):
            r = bv - D @ xm
            xm[idx[c]] += np.linalg.solve(D[np.ix_(idx[c], idx[c])], r[idx[c]])
        r = bv - D @ xa
        upd = np.zeros_like(xa)
        for c in (0, 1):
            upd[idx[c]] = np.linalg.solve(D[np.ix_(idx[c], idx[c])], r[idx[c]])
        xa += upd
    S = sap.Schwarz(dims, U, m0, csw, bdims, antiperiodic_t=ap)
    assert rel(S.apply(b, cycles=2, exact=True).ravel(), xm) < 1e-12
    assert rel(S.apply(b, cycles=2, exact=True, additive=True).ravel(), xa) < 1e-12


def test_whole_lattice_block_is_the_inverse():
    dims = (2, 2, 2, 4)
    m0, csw = -0.3, 1.0
    U, b = inputs(dims, 33)
    D = dense_brute_force(dims, U, m0, csw)
    S = sap.Schwarz(dims, U, m0, csw, dims)
    x = S.apply(b, cycles=1, exact=True)
    assert rel(x.ravel(), np.linalg.solve(D, b.ravel())) < 1e-12


def test_single_site_blocks_reduce_to_site_local_solves():
    """Blocks of one site: D_B = A(x).  Red-black: x_e = A_ee^{-1} b_e, then
    x_o = A_oo^{-1} (b_o - H_oe x_e) (the even-odd oracle's pieces); additive:
    x = A^{-1} b.  Many MR steps on an HPD A(x) reach the same."""
    dims = (2, 2, 4, 2)
    m0, csw = -0.3, 1.0
    U, b = inputs(dims, 35)
    eo = evenodd.EvenOdd(dims, U, m0, csw)
    be, bo = evenodd.split(dims, b)
    xe = np.linalg.solve(eo.A[eo.e], be[..., None])[..., 0]
    xo = eo.ainv_o(bo - eo.hop_oe(xe))
    want = evenodd.merge(dims, xe, xo)
    S = sap.Schwarz(dims, U, m0, csw, (1, 1, 1, 1))
    assert rel(S.apply(b, cycles=1, exact=True), want) < 1e-13
    assert rel(S.apply(b, cycles=1, mr_iters=40), want) < 1e-9
    xa = np.linalg.solve(eo.A, b[..., None])[..., 0]
    assert rel(S.apply(b, cycles=1, exact=True, additive=True), xa) < 1e-13


def test_minimal_residual_step():
    """Each MR step leaves the new block residual orthogonal to q = D_B rho
    (alpha minimises |rho - alpha q|), so the residual norm never grows."""
    dims = (4, 4, 4, 4)
    m0, csw = -0.3, 1.0
    U, b = inputs(dims, 37)
    S = sap.Schwarz(dims, U, m0, csw, (2, 2, 2, 2))
    k = 3
    sites = S.blocks[k][1]
    rho = b[sites]
    e = np.zeros_like(rho)
    norms = [np.linalg.norm(rho)]
    for _ in range(6):
        q = S.block_apply(k, rho)
        alpha = np.vdot(q, rho) / np.vdot(q, q).real
        e, rho = e + alpha * rho, rho - alpha * q
        assert abs(np.vdot(q, rho)) < 1e-12 * np.linalg.norm(q) * np.linalg.norm(rho) + 1e-14
        norms.append(np.linalg.norm(rho))
    assert all(n1 <= n0 * (1 + 1e-14) for n0, n1 in zip(norms, norms[1:]))
    assert rel(S.mr(k, b[sites], 6), e) < 1e-14
    # e solves D_B e = r_B up to the final residual rho
    assert rel(S.block_apply(k, e), b[sites] - rho) < 1e-13


def test_exact_cycle_clears_the_last_colour():
    dims = (4, 4, 2, 4)
    m0, csw = -0.3, 1.0
    U, b = inputs(dims, 39)
    S = sap.Schwarz(dims, U, m0, csw, (2, 2, 2, 2))
    x = S.apply(b, cycles=1, exact=True)
    r = S.residual(b, x)
    last = np.concatenate([s for c, s in S.blocks if c == 1])
    first = np.concatenate([s for c, s in S.blocks if c == 0])
    assert np.linalg.norm(r[last]) < 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(r[first]) > 1e-3 * np.linalg.norm(b)


def test_blocking_rules():
    with pytest.raises(ValueError):
        sap.check_blocking((8, 8, 8, 8), (3, 4, 4, 4))
    with pytest.raises(ValueError):
        sap.check_blocking((12, 8, 8, 8), (4, 4, 4, 4))  # three blocks along T
    assert tuple(sap.check_blocking((8, 4, 4, 8), (4, 4, 4, 4))) == (2, 1, 1, 2)
    blocks = sap.block_list((4, 2, 2, 4), (2, 2, 2, 2))
    assert [c for c, _ in blocks] == [0, 1, 1, 0]
    assert sorted(np.concatenate([s for _, s in blocks])) == list(range(64))


def test_fgmres_with_sap_preconditioner():
    """FGMRES with one red-black SAP cycle (4^4 blocks, 4 MR steps) as M_j^{-1}
    reaches 1e-10 by the true residual, with far fewer operator applications
    than without a preconditioner."""
    dims = (8, 8, 8, 8)
    m0, csw = -0.3, 1.0
    U, b = inputs(dims, 41)
    S = sap.Schwarz(dims, U, m0, csw, (4, 4, 4, 4))
    C = oracle.clover_term(dims, U)
    A = lambda v: oracle.dirac_apply(dims, U, v, m0, csw, clover=C)
    x, info = oracle.fgmres(A, b, m=10, tol=1e-10, maxit=500, precond=lambda v, j: S.apply(v, 1, 4))
    _, plain = oracle.fgmres(A, b, m=10, tol=1e-10, maxit=1000)
    assert info["converged"]
    assert np.linalg.norm(b - A(x)) / np.linalg.norm(b) <= 1e-10 * 1.01
    assert info["applies"] * 3 < plain["applies"], (info["applies"], plain["applies"])
