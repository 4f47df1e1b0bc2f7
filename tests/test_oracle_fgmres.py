"""Pins of the oracle FGMRES (Algorithm 2) against a library routine and the
paper's exact-inverse argument (Sec. 1.3)."""
import numpy as np
import scipy.sparse.linalg as spla

import oracle
from paper_2407_00041_amd import synth


def _system(dims, seed, m0=-0.3, csw=1.0):
    V = synth.volume(dims)
    U = synth.smooth_links(dims, seed).numpy()
    C = oracle.clover_term(dims, U)
    A = lambda v: oracle.dirac_apply(dims, U, v.reshape(-1, V, 12), m0, csw, clover=C).reshape(v.shape)
    b = synth.gaussian_spinor(dims, seed + 1)
    return V, U, C, A, b


def test_residual_history_matches_scipy_gmres():
    """Without preconditioning FGMRES is GMRES; the minimal residual over each
    Krylov space is unique, so the per-step residual norms must agree with
    scipy's restarted GMRES."""
    dims = (4, 4, 4, 4)
    V, U, C, A, b = _system(dims, 1000)
    n = 12 * V
    hist = []
    x, info = oracle.fgmres(A, b, m=20, tol=1e-10, maxit=2000, history=hist)
    assert info["converged"]
    ref_hist = []
    op = spla.LinearOperator((n, n), matvec=lambda v: A(v.reshape(V, 12)).ravel(), dtype=complex)
    xs, code = spla.gmres(op, b.ravel(), rtol=1e-10, atol=0.0, restart=20, maxiter=200,
                          callback=ref_hist.append, callback_type="pr_norm")
    assert code == 0
    k = 0
    while k < min(len(hist), len(ref_hist)) and ref_hist[k] > 1e-9:
        assert abs(hist[k] - ref_hist[k]) <= 1e-8 * ref_hist[k], (k, hist[k], ref_hist[k])
        k += 1
    assert k > 40           # the comparison covered several restart cycles
    r = b - A(x)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-10
    assert np.linalg.norm(x.ravel() - xs) / np.linalg.norm(xs) < 1e-8


def test_exact_inverse_preconditioner_one_inner_iteration():
    """With M^{-1} = A^{-1}, FGMRES stops after one inner iteration with the
    exact solution (the breakdown h_21 = 0 ends the cycle)."""
    dims = (2, 2, 2, 2)
    V, U, C, A, b = _system(dims, 7, m0=-0.4)
    n = 12 * V
    cols = A(np.eye(n, dtype=complex).reshape(n, V, 12))
    Ad = cols.reshape(n, n).T
    Ainv = np.linalg.inv(Ad)
    inner = []
    pre = lambda v, j: (inner.append(j), (Ainv @ v.ravel()).reshape(v.shape))[1]
    x, info = oracle.fgmres(A, b, m=10, tol=1e-10, maxit=100, precond=pre)
    assert inner == [0]
    assert info["breakdown"] and info["converged"]
    assert info["applies"] == 3      # initial residual, one inner step, final residual
    assert np.linalg.norm(x.ravel() - Ainv @ b.ravel()) / np.linalg.norm(b) < 1e-12


def test_restart_and_maxit_accounting():
    dims = (2, 2, 2, 4)
    V, U, C, A, b = _system(dims, 3)
    x, info = oracle.fgmres(A, b, m=5, tol=1e-12, maxit=13)
    assert not info["converged"]
    assert info["applies"] == 13
    x2, info2 = oracle.fgmres(A, b, m=5, tol=1e-10, maxit=5000, x0=x)
    assert info2["converged"]
    assert np.linalg.norm(b - A(x2)) <= 1e-10 * np.linalg.norm(b - A(x)) * 1.01
    z, info0 = oracle.fgmres(A, np.zeros_like(b), m=5, tol=1e-10, maxit=50)
    assert info0["converged"] and info0["applies"] == 1 and not z.any()
