"""Pins of the oracle's two-level multigrid (oracle/amg.py) to facts that do
not come from the oracle itself:

* Gram-Schmidt equals the Householder QR of a library routine (phases fixed
  so that R has a positive real diagonal);
* P has orthonormal columns, commutes with gamma_5 and reproduces every test
  vector (P P^H v_k = v_k), and restriction is the adjoint of prolongation;
* free field and constant U(1) backgrounds with constant test vectors: D_c in
  closed form (a coarse Wilson operator with hop weights 1/a_mu and mass
  4 + m0 - sum_mu (a_mu - 1)/a_mu), periodic and anti-periodic, with coarse
  extents 1 and 2 where neighbours coincide;
* D_c = P^H D P with D the brute-force matrix of Eq. (1.10) plus Eq. (1.11),
  and the coarse gamma_5-hermiticity D_c^H = G5c D_c G5c;
* single-site aggregates with 6 test vectors: P is unitary, so the two-level
  method is D^{-1} and FGMRES stops after one Arnoldi step (the optimal
  preconditioner of Sec. 1.3);
* the setup moves the interpolation towards the near kernel (Sec. 1.3): the
  part of D's smallest-|eigenvalue| eigenvector outside range(P) shrinks;
* FGMRES with the two-level preconditioner reaches 1e-10 in fewer operator
  applications than with SAP alone or with no preconditioner."""
import numpy as np
import pytest

import oracle
from oracle import amg
from paper_2407_00041_amd import synth
from test_oracle_operator import G, coords, dense_brute_force


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def gaussian(n, V, seed):
    return synth.gaussian_spinor((1, 1, 1, V), seed, nrhs=n).reshape(n, V, 12)


def dense_P(tl):
    nc = tl.Vc * 2 * tl.N
    E = np.eye(nc, dtype=np.complex128)
    return np.stack([tl.prolong(E[j]).ravel() for j in range(nc)], axis=1)


def test_gram_schmidt_equals_householder_qr():
    rng = np.random.default_rng(5)
    W = rng.normal(size=(60, 9)) + 1j * rng.normal(size=(60, 9))
    Q = amg.orthonormalise(W)
    Qh, Rh = np.linalg.qr(W)
    ph = np.diag(Rh) / np.abs(np.diag(Rh))
    assert np.allclose(Q, Qh * ph[None, :].conj(), atol=1e-13)
    R = Q.conj().T @ W
    assert np.allclose(np.tril(R, -1), 0, atol=1e-12)
    assert np.all(np.diag(R).real > 0) and np.allclose(np.diag(R).imag, 0, atol=1e-12)
    with pytest.raises(ValueError):
        amg.orthonormalise(np.stack([W[:, 0], 2 * W[:, 0]], 1))


@pytest.mark.parametrize("dims,agg,N", [((4, 4, 4, 4), (2, 2, 2, 2), 8), ((2, 4, 2, 6), (2, 1, 2, 3), 5)])
def test_interpolation_properties(dims, agg, N):
    U = synth.smooth_links(dims, 40).numpy()
    V = synth.volume(dims)
    T = gaussian(N, V, 41)
    tl = amg.TwoLevel(dims, U, -0.3, 1.0, agg, T)
    P = dense_P(tl)
    assert np.allclose(P.conj().T @ P, np.eye(P.shape[1]), atol=1e-13)
    for k in range(N):
        v = T[k].ravel()
        assert rel(P @ (P.conj().T @ v), v) < 1e-13
    f = gaussian(1, V, 42)[0]
    g5 = np.r_[np.ones(6), -np.ones(6)]
    c = tl.restrict(f)
    assert np.allclose(tl.restrict(f * g5), c * np.array([1, -1])[None, :, None], atol=1e-13)
    assert np.allclose(c.ravel(), P.conj().T @ f.ravel(), atol=1e-13)
    cr = gaussian(1, tl.Vc * 2 * N, 43).ravel()[:tl.Vc * 2 * N]
    assert np.allclose(tl.prolong(cr).ravel(), P @ cr, atol=1e-13)


def closed_form_coarse(dims, agg, m0, theta, antiperiodic):
    """Coarse operator of the free field with constant U(1) links e^{i theta_mu} and the constant test vectors
    e_k + e_{6+k}: hops of D from Eq. (1.13) counted per aggregate pair."""
    nc = amg.coarse_dims(dims, agg)
    Vc = int(np.prod(nc))
    cc = coords(nc)
    M = np.zeros((Vc, 12, Vc, 12), np.complex128)
    I4 = np.eye(4)
    for a in range(Vc):
        M[a, :, a, :] += (4.0 + m0) * np.eye(12)
        for mu in range(4):
            for d in (1, -1):
                hop = -0.5 * np.kron(I4 - d * G[mu], np.eye(3)) * np.exp(1j * d * theta[mu])
                # hops that stay inside the aggregate without wrapping: (a_mu - 1) of every a_mu
                M[a, :, a, :] += hop * (agg[mu] - 1) / agg[mu]
                # the hop leaving the aggregate: 1 of every a_mu, to the neighbouring coarse site
                e = np.zeros(4, int)
                e[mu] = d
                nb = cc[a] + e
                wraps = nb[mu] < 0 or nb[mu] >= nc[mu]
                sign = -1.0 if (antiperiodic and mu == 0 and wraps) else 1.0
                b = ((nb[0] % nc[0] * nc[1] + nb[1] % nc[1]) * nc[2] + nb[2] % nc[2]) * nc[3] + nb[3] % nc[3]
                M[a, :, b, :] += sign * hop / agg[mu]
    return M.reshape(Vc * 12, Vc * 12)


@pytest.mark.parametrize("dims,agg,theta,ap", [
    ((4, 6, 4, 8), (2, 3, 2, 2), (0.0, 0.0, 0.0, 0.0), False),
    ((4, 6, 4, 8), (2, 3, 2, 2), (0.3, -0.7, 1.1, 0.2), True),
    ((6, 2, 4, 4), (3, 2, 1, 2), (0.5, 0.1, -0.4, 0.9), False),
    ((4, 2, 4, 6), (4, 1, 2, 2), (0.2, 0.6, 0.0, -0.3), True)])
def test_free_field_coarse_operator_closed_form(dims, agg, theta, ap):
    V = synth.volume(dims)
    m0 = -0.3
    U = np.zeros((V, 4, 3, 3), np.complex128)
    for mu in range(4):
        U[:, mu] = np.exp(1j * theta[mu]) * np.eye(3)
    T = np.zeros((6, V, 12), np.complex128)
    for k in range(6):
        T[k, :, k] = 1.0
        T[k, :, 6 + k] = 1.0
    tl = amg.TwoLevel(dims, U, m0, 1.0, agg, T, antiperiodic_t=ap)
    Dc = tl.coarse_matrix()
    assert np.allclose(Dc, closed_form_coarse(dims, agg, m0, theta, ap), atol=1e-13)


@pytest.mark.parametrize("dims,agg,N,ap", [((2, 2, 2, 4), (1, 2, 1, 2), 4, False),
                                           ((2, 2, 2, 4), (2, 1, 2, 2), 3, True)])
def test_galerkin_product_of_brute_force_operator(dims, agg, N, ap):
    m0, csw = -0.3, 1.0
    U = synth.smooth_links(dims, 44).numpy()
    V = synth.volume(dims)
    tl = amg.TwoLevel(dims, U, m0, csw, agg, gaussian(N, V, 45), antiperiodic_t=ap)
    P = dense_P(tl)
    Dc_ref = P.conj().T @ dense_brute_force(dims, U, m0, csw, antiperiodic=ap) @ P
    Dc = tl.coarse_matrix()
    assert rel(Dc, Dc_ref) < 1e-12
    g5c = np.tile(np.r_[np.ones(N), -np.ones(N)], tl.Vc)
    assert np.allclose(Dc.conj().T, g5c[:, None] * Dc * g5c[None, :], atol=1e-12)


def test_single_site_aggregates_give_exact_inverse():
    """Aggregates of one site and 6 test vectors: P is square and unitary, D_c is similar to D, and the
    coarse correction alone solves D z = r (the smoother then sees a zero residual)."""
    dims = (2, 2, 2, 4)
    m0, csw = -0.3, 1.0
    U = synth.smooth_links(dims, 46).numpy()
    V = synth.volume(dims)
    tl = amg.TwoLevel(dims, U, m0, csw, (1, 1, 1, 1), gaussian(6, V, 47))
    P = dense_P(tl)
    assert np.allclose(P.conj().T @ P, np.eye(12 * V), atol=1e-12)
    D = dense_brute_force(dims, U, m0, csw)
    r = gaussian(1, V, 48)[0]
    z = tl.precond(r)
    assert rel(z.ravel(), np.linalg.solve(D, r.ravel())) < 1e-11
    x, info = oracle.fgmres(lambda v: tl.D(v), r, m=10, tol=1e-10, maxit=50, precond=lambda v, j: tl.precond(v))
    assert info["converged"] and info["applies"] == 3, info
    assert rel(tl.D(x), r) < 1e-10


def test_coarse_gmres_reaches_the_exact_coarse_solution():
    dims = (4, 4, 2, 4)
    U = synth.smooth_links(dims, 49).numpy()
    V = synth.volume(dims)
    tl = amg.TwoLevel(dims, U, -0.3, 1.0, (2, 2, 2, 2), gaussian(4, V, 50))
    rc = gaussian(1, V, 51).ravel()[:tl.Vc * 2 * tl.N]
    assert rel(tl.coarse_solve(rc, tol=1e-13), tl.coarse_solve(rc)) < 1e-11


def test_setup_approaches_the_near_kernel():
    """Sec. 1.3: the setup approximates eigenvectors of small |eigenvalue|.  After it, the smallest mode's part
    outside range(P) is smaller than with the raw random test vectors."""
    dims = (2, 2, 4, 4)
    m0, csw = -0.4, 1.0
    U = synth.smooth_links(dims, 52).numpy()
    V = synth.volume(dims)
    D = dense_brute_force(dims, U, m0, csw)
    w, X = np.linalg.eig(D)
    vmin = X[:, np.argmin(np.abs(w))]
    T0 = gaussian(8, V, 53)

    def outside(t):
        P = dense_P(t)
        return np.linalg.norm(vmin - P @ (P.conj().T @ vmin)) / np.linalg.norm(vmin)

    seq = [outside(amg.TwoLevel(dims, U, m0, csw, (2, 2, 2, 2), T0))]
    for si in range(3):
        seq.append(outside(amg.setup(dims, U, m0, csw, (2, 2, 2, 2), T0, init_iters=3, setup_iters=si)))
    assert all(b < a for a, b in zip(seq, seq[1:])), seq
    assert seq[-1] < 0.5 * seq[0], seq


def test_two_level_fgmres_needs_fewer_applies():
    dims = (4, 4, 4, 4)
    m0, csw = -0.4, 1.0
    U = synth.smooth_links(dims, 54).numpy()
    V = synth.volume(dims)
    b = gaussian(1, V, 55)[0]
    tl = amg.setup(dims, U, m0, csw, (2, 2, 2, 2), gaussian(6, V, 56), init_iters=3, setup_iters=1)
    kw = dict(m=20, tol=1e-10, maxit=3000)
    x, info = oracle.fgmres(tl.D, b, precond=lambda v, j: tl.precond(v), **kw)
    assert info["converged"] and rel(tl.D(x), b) < 1.01e-10
    _, info_sap = oracle.fgmres(tl.D, b, precond=lambda v, j: tl.smooth(v), **kw)
    _, info_none = oracle.fgmres(tl.D, b, **kw)
    assert info["applies"] < info_sap["applies"] < info_none["applies"], (info, info_sap, info_none)
