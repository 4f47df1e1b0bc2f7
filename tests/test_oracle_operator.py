"""Pins of the CPU oracle's operator against facts fixed by the paper and by the
mathematics, independent of the oracle's own code.

* gamma algebra: Hermitian, anticommuting, gamma_5 diagonal (the property the
  42-entry clover storage of Sec. 2.3 relies on).
* free field (U = 1) and constant U(1) backgrounds: the plane-wave action of
  Eq. (1.13) in closed form, m0 + sum(1 - cos q) + i sum gamma sin q with
  q = p + theta (p shifted by pi/L_T under the anti-periodic time boundary).
* adjoint identity <y, D x> = <D^H y, x> and gamma_5-hermiticity.
* gauge covariance of Eq. (1.13) with the clover term of Eqs. (1.11)-(1.12).
* constant abelian field strength: the clover term in closed form.
* dense brute force: D assembled from the covariant differences of Eq. (1.10)
  plus Eq. (1.11), compared column by column on tiny lattices (including
  L = 2 where x + mu and x - mu coincide).
"""
import numpy as np
import pytest

import oracle
from paper_2407_00041_amd import synth

G = [oracle.gamma(mu) for mu in range(4)]
G5 = G[3] @ G[2] @ G[1] @ G[0]   # gamma_X gamma_Y gamma_Z gamma_T


def coords(dims):
    """[V, 4] integer coordinates (t, z, y, x) in lexicographic site order."""
    return np.stack(np.meshgrid(*[np.arange(n) for n in dims], indexing="ij"), -1).reshape(-1, 4)


def site_index(dims, c):
    c = np.asarray(c) % np.asarray(dims)
    return ((c[..., 0] * dims[1] + c[..., 1]) * dims[2] + c[..., 2]) * dims[3] + c[..., 3]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# --------------------------------------------------------------------------
def test_gamma_algebra():
    for mu in range(4):
        assert np.allclose(G[mu], G[mu].conj().T, atol=0)
        for nu in range(4):
            anti = G[mu] @ G[nu] + G[nu] @ G[mu]
            assert np.allclose(anti, 2 * np.eye(4) * (mu == nu), atol=1e-15)
    assert np.allclose(G5, np.diag([1, 1, -1, -1]), atol=1e-15)


# --------------------------------------------------------------------------
def plane_wave_expected(dims, u, p, theta, m0):
    """e^{i p.x} u under D with U_mu = e^{i theta_mu} I: closed form."""
    q = np.asarray(p) + np.asarray(theta)
    M = (m0 + np.sum(1 - np.cos(q))) * np.eye(4, dtype=complex)
    for mu in range(4):
        M = M + 1j * np.sin(q[mu]) * G[mu]
    c = coords(dims)
    phase = np.exp(1j * (c @ np.asarray(p)))
    spin = (M @ u.reshape(4, 3))                        # [4 spins, 3 colours]
    return phase[:, None] * spin.reshape(1, 12)


@pytest.mark.parametrize("dims", [(4, 6, 8, 10), (3, 5, 2, 4)])
@pytest.mark.parametrize("antiperiodic", [False, True])
@pytest.mark.parametrize("abelian", [False, True])
def test_plane_waves_closed_form(dims, antiperiodic, abelian):
    rng = np.random.default_rng(11)
    V = synth.volume(dims)
    m0 = -0.37
    theta = rng.uniform(-np.pi, np.pi, 4) if abelian else np.zeros(4)
    U = np.zeros((V, 4, 3, 3), complex)
    for mu in range(4):
        U[:, mu] = np.exp(1j * theta[mu]) * np.eye(3)
    c = coords(dims)
    for trial in range(3):
        n = rng.integers(0, 17, 4)
        p = 2 * np.pi * n / np.asarray(dims, float)
        if antiperiodic:
            p[0] += np.pi / dims[0]
        u = rng.standard_normal(12) + 1j * rng.standard_normal(12)
        psi = np.exp(1j * (c @ p))[:, None] * u[None, :]
        # c_sw = 1: plaquettes are trivial, so the clover term must vanish
        got = oracle.dirac_apply(dims, U, psi, m0, csw=1.0, antiperiodic_t=antiperiodic)
        want = plane_wave_expected(dims, u, p, theta, m0)
        assert rel(got, want) < 1e-14


def test_free_field_eigenvalues_closed_form():
    """Spectrum of the free operator on 4^4: m0 + sum(1 - cos p) +- i|sin p|, each 6-fold."""
    dims = (4, 4, 4, 4)
    V = synth.volume(dims)
    m0 = -0.2
    U = np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3)).copy()
    D = dense_from_oracle(dims, U, m0, 0.0)
    key = lambda z: z[np.lexsort((np.round(z.imag, 8), np.round(z.real, 8)))]
    ev = key(np.linalg.eigvals(D))
    want = []
    for n in np.ndindex(*dims):
        p = 2 * np.pi * np.asarray(n) / np.asarray(dims)
        re = m0 + np.sum(1 - np.cos(p))
        im = np.sqrt(np.sum(np.sin(p) ** 2))
        want += [re + 1j * im] * 6 + [re - 1j * im] * 6
    want = key(np.asarray(want))
    assert np.max(np.abs(ev - want)) < 1e-12


# --------------------------------------------------------------------------
def random_fields(dims, seed, smooth=False):
    V = synth.volume(dims)
    if smooth:
        U = synth.smooth_links(dims, seed).numpy()
    else:
        U = synth.haar_links(dims, seed)
    rng = np.random.default_rng(seed + 1)
    x = rng.standard_normal((V, 12)) + 1j * rng.standard_normal((V, 12))
    y = rng.standard_normal((V, 12)) + 1j * rng.standard_normal((V, 12))
    return U, x, y


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 8, 10), (2, 2, 2, 2)])
@pytest.mark.parametrize("antiperiodic", [False, True])
def test_adjoint_and_gamma5_hermiticity(dims, antiperiodic):
    U, x, y = random_fields(dims, 5)
    m0, csw = -0.4, 1.3
    Dx = oracle.dirac_apply(dims, U, x, m0, csw, antiperiodic_t=antiperiodic)
    DHy = oracle.dirac_apply(dims, U, y, m0, csw, antiperiodic_t=antiperiodic, dagger=True)
    lhs = np.vdot(y, Dx)
    assert abs(lhs - np.vdot(DHy, x)) / abs(lhs) < 1e-13
    g5 = np.kron(np.diag([1, 1, -1, -1]), np.eye(3))
    g5y = y @ g5.T
    g5Dg5y = oracle.dirac_apply(dims, U, g5y, m0, csw, antiperiodic_t=antiperiodic) @ g5.T
    assert rel(g5Dg5y, DHy) < 1e-13
    assert abs(lhs - np.vdot(g5Dg5y, x)) / abs(lhs) < 1e-13


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 4, 5, 2)])
def test_gauge_covariance(dims):
    """D[U'] (G psi) = G (D[U] psi) with U'_mu(x) = G(x) U_mu(x) G(x+mu)^H."""
    V = synth.volume(dims)
    U, x, _ = random_fields(dims, 21)
    Gx = synth.haar_su3(V, 99)
    c = coords(dims)
    Up = np.empty_like(U)
    for mu in range(4):
        e = np.zeros(4, int)
        e[mu] = 1
        nb = site_index(dims, c + e)
        Up[:, mu] = Gx @ U[:, mu] @ np.conj(np.swapaxes(Gx[nb], 1, 2))
    gpsi = np.einsum("vab,vsb->vsa", Gx, x.reshape(V, 4, 3)).reshape(V, 12)
    m0, csw = -0.3, 1.0
    lhs = oracle.dirac_apply(dims, Up, gpsi, m0, csw, antiperiodic_t=True)
    Dpsi = oracle.dirac_apply(dims, U, x, m0, csw, antiperiodic_t=True)
    rhs = np.einsum("vab,vsb->vsa", Gx, Dpsi.reshape(V, 4, 3)).reshape(V, 12)
    assert rel(lhs, rhs) < 1e-13
    # the clover term itself transforms as C' = (1 (x) G) C (1 (x) G)^H
    C = unpack_clover(oracle.clover_term(dims, U))
    Cp = unpack_clover(oracle.clover_term(dims, Up))
    GG = np.einsum("ab,vij->vaibj", np.eye(4), Gx).reshape(V, 12, 12)
    assert np.max(np.abs(Cp - GG @ C @ np.conj(np.swapaxes(GG, 1, 2)))) < 1e-13


# --------------------------------------------------------------------------
def unpack_clover(packed):
    """[V,42] packed -> [V,12,12] Hermitian block-diagonal (test's own unpacking)."""
    V = packed.shape[0]
    out = np.zeros((V, 12, 12), complex)
    upper = [(i, j) for i in range(6) for j in range(i + 1, 6)]
    for blk in range(2):
        o = 6 * blk
        for k in range(6):
            out[:, o + k, o + k] = packed[:, 21 * blk + k].real
        for k, (i, j) in enumerate(upper):
            out[:, o + i, o + j] = packed[:, 21 * blk + 6 + k]
            out[:, o + j, o + i] = np.conj(packed[:, 21 * blk + 6 + k])
    return out


def test_clover_invariants():
    dims = (4, 4, 4, 4)
    U, _, _ = random_fields(dims, 3, smooth=True)
    C = unpack_clover(oracle.clover_term(dims, U))
    assert np.max(np.abs(C - np.conj(np.swapaxes(C, 1, 2)))) == 0
    # gamma_mu gamma_nu is traceless for mu != nu
    assert np.max(np.abs(np.trace(C, axis1=1, axis2=2))) < 1e-14
    assert np.max(np.abs(C)) > 1e-2           # non-trivial for random links
    # pure-gauge configuration: all plaquettes are 1, so C = 0
    V = synth.volume(dims)
    Gx = synth.haar_su3(V, 7)
    c = coords(dims)
    Ug = np.empty((V, 4, 3, 3), complex)
    for mu in range(4):
        e = np.zeros(4, int)
        e[mu] = 1
        Ug[:, mu] = Gx @ np.conj(np.swapaxes(Gx[site_index(dims, c + e)], 1, 2))
    assert np.max(np.abs(oracle.clover_term(dims, Ug))) < 1e-13


def test_constant_field_strength_clover_closed_form():
    """Uniform abelian flux f in the T-Z plane and g in the Y-X plane.

    Every leaf of Eq. (1.12) is then diag(e^{if}, e^{-if}, 1) (or with g), so
    Q_TZ - Q_ZT = 8i S(f), S(f) = diag(sin f, -sin f, 0), and Eq. (1.11) gives
    C = -(i/2) [gamma_T gamma_Z (x) S(f) + gamma_Y gamma_X (x) S(g)].
    """
    dims = (4, 6, 4, 6)
    nT, nZ, nY, nX = dims
    V = synth.volume(dims)
    f = 2 * np.pi * 1 / (nT * nZ)
    g = 2 * np.pi * 2 / (nY * nX)
    c = coords(dims)
    t, z, y, x = c.T
    emb = lambda phi: np.stack([np.diag([np.exp(1j * a), np.exp(-1j * a), 1]) for a in phi])
    phT = np.where(t == nT - 1, -f * nT * z, 0.0)
    phZ = f * t
    phY = np.where(y == nY - 1, -g * nY * x, 0.0)
    phX = g * y
    U = np.stack([emb(phT), emb(phZ), emb(phY), emb(phX)], axis=1)
    # every leaf is the same plaquette
    for s in [0, 17, V - 1]:
        assert np.allclose(oracle.leaves(dims, U, s, 0, 1), 4 * np.diag([np.exp(1j * f), np.exp(-1j * f), 1]), atol=1e-13)
        assert np.allclose(oracle.leaves(dims, U, s, 2, 3), 4 * np.diag([np.exp(1j * g), np.exp(-1j * g), 1]), atol=1e-13)
        assert np.allclose(oracle.leaves(dims, U, s, 0, 2), 4 * np.eye(3), atol=1e-13)
    S = lambda a: np.diag([np.sin(a), -np.sin(a), 0])
    want = -0.5j * (np.kron(G[0] @ G[1], S(f)) + np.kron(G[2] @ G[3], S(g)))
    C = unpack_clover(oracle.clover_term(dims, U))
    assert np.max(np.abs(C - want[None])) < 1e-14
    # and the operator: A = (4 + m0) + csw C at every site
    m0, csw = 0.1, 1.7
    rng = np.random.default_rng(0)
    psi = rng.standard_normal((V, 12)) + 1j * rng.standard_normal((V, 12))
    hop_only = oracle.dirac_apply(dims, U, psi, m0, 0.0)
    full = oracle.dirac_apply(dims, U, psi, m0, csw)
    assert rel(full - hop_only, csw * psi @ want.T) < 1e-13


# --------------------------------------------------------------------------
def dense_from_oracle(dims, U, m0, csw, antiperiodic=False, dagger=False):
    V = synth.volume(dims)
    n = 12 * V
    E = np.eye(n, dtype=complex)
    cols = oracle.dirac_apply(dims, U, E.reshape(n, V, 12), m0, csw,
                              antiperiodic_t=antiperiodic, dagger=dagger)
    return cols.reshape(n, n).T


def dense_brute_force(dims, U, m0, csw, antiperiodic=False):
    """Eq. (1.10) from covariant differences plus Eq. (1.11), as dense matrices.

    Colour-site operators are (V*3)x(V*3) matrices; the full matrix has the
    row index 12*site + 3*sigma + c.
    """
    V = synth.volume(dims)
    c = coords(dims)
    I3V = np.eye(3 * V, dtype=complex)

    def fwd(mu):   # (Tf psi)(x) = s U_mu(x) psi(x+mu)
        T = np.zeros((3 * V, 3 * V), complex)
        e = np.zeros(4, int)
        e[mu] = 1
        for xs in range(V):
            ys = site_index(dims, c[xs] + e)
            s = -1.0 if (antiperiodic and mu == 0 and c[xs][0] == dims[0] - 1) else 1.0
            T[3 * xs:3 * xs + 3, 3 * ys:3 * ys + 3] += s * U[xs, mu]
        return T

    def bwd(mu):   # (Tb psi)(x) = s U_mu(x-mu)^H psi(x-mu)
        T = np.zeros((3 * V, 3 * V), complex)
        e = np.zeros(4, int)
        e[mu] = 1
        for xs in range(V):
            ys = site_index(dims, c[xs] - e)
            s = -1.0 if (antiperiodic and mu == 0 and c[xs][0] == 0) else 1.0
            T[3 * xs:3 * xs + 3, 3 * ys:3 * ys + 3] += s * U[ys, mu].conj().T
        return T

    def full(S, K):   # spin S (x) colour-site K -> index 12 x + 3 sigma + c
        M = np.einsum("ab,xiyj->xaiybj", S, K.reshape(V, 3, V, 3))
        return M.reshape(12 * V, 12 * V)

    I4 = np.eye(4)
    D = m0 * np.eye(12 * V, dtype=complex)
    for mu in range(4):
        d_up = fwd(mu) - I3V        # Delta^mu
        d_dn = I3V - bwd(mu)        # Delta_mu
        D += 0.5 * (full(G[mu], d_dn + d_up) - full(I4, d_dn @ d_up))
    if csw != 0.0:
        # Eq. (1.12) per site, all ordered pairs, then Eq. (1.11)
        Cfull = np.zeros((12 * V, 12 * V), complex)
        for xs in range(V):
            blk = np.zeros((12, 12), complex)
            for mu in range(4):
                for nu in range(4):
                    blk += -(1 / 32) * np.kron(G[mu] @ G[nu], leaf_sum(dims, U, c[xs], mu, nu)
                                               - leaf_sum(dims, U, c[xs], nu, mu))
            Cfull[12 * xs:12 * xs + 12, 12 * xs:12 * xs + 12] = blk
        D += csw * Cfull
    return D


def leaf_sum(dims, U, x, mu, nu):
    e = np.zeros((4, 4), int)
    np.fill_diagonal(e, 1)
    L = lambda pos, d: U[site_index(dims, pos), d]
    H = lambda M: M.conj().T
    m, n = e[mu], e[nu]
    return (L(x, mu) @ L(x + m, nu) @ H(L(x + n, mu)) @ H(L(x, nu))
            + L(x, nu) @ H(L(x - m + n, mu)) @ H(L(x - m, nu)) @ L(x - m, mu)
            + H(L(x - m, mu)) @ H(L(x - m - n, nu)) @ L(x - m - n, mu) @ L(x - n, nu)
            + H(L(x - n, nu)) @ L(x - n, mu) @ L(x - n + m, nu) @ H(L(x, mu)))


@pytest.mark.parametrize("dims,antiperiodic", [((2, 2, 2, 2), False), ((2, 2, 2, 2), True),
                                               ((3, 2, 4, 2), True)])
def test_dense_brute_force(dims, antiperiodic):
    U, _, _ = random_fields(dims, 31)
    m0, csw = -0.4, 1.0
    D_or = dense_from_oracle(dims, U, m0, csw, antiperiodic)
    D_bf = dense_brute_force(dims, U, m0, csw, antiperiodic)
    assert np.max(np.abs(D_or - D_bf)) / np.max(np.abs(D_bf)) < 1e-13
    D_h = dense_from_oracle(dims, U, m0, csw, antiperiodic, dagger=True)
    assert np.max(np.abs(D_h - D_bf.conj().T)) < 1e-13


def test_apply_sites_matches_full():
    dims = (4, 6, 4, 2)
    U, x, _ = random_fields(dims, 41, smooth=True)
    sites = synth.random_sites(dims, 25, 3)
    full = oracle.dirac_apply(dims, U, x, -0.35, 1.0, antiperiodic_t=True)
    part = oracle.dirac_apply_sites(dims, U, x, sites, -0.35, 1.0, antiperiodic_t=True)
    assert np.array_equal(part, full[sites])
    C = oracle.clover_term(dims, U)
    part2 = oracle.dirac_apply_sites(dims, U, x, sites, -0.35, 1.0, clover=C, antiperiodic_t=True)
    assert np.array_equal(part2, full[sites])
