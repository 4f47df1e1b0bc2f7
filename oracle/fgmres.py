"""FGMRES, Algorithm 2 of Sec. 1.2, in plain NumPy (FP64).  Test infrastructure.

Steps in the paper's order and notation:

  x <- x0;  while not terminated:
      r <- b - A x;  beta <- ||r||;  v_1 <- r / beta                  (restart)
      for j = 1..m:
          z_j <- M_j^{-1} v_j;  w <- A z_j
          for i = 1..j:  h_ij <- <w, v_i>;  w <- w - h_ij v_i     (modified GS)
          h_{j+1,j} <- ||w||;  v_{j+1} <- w / h_{j+1,j}
      y <- argmin_y || beta e_1 - H_m y ||;  x <- x + Z_m y

Readings of what the paper leaves open (each also listed in the design notes):
  * <w, v_i> = v_i^H w (conjugate-linear in v_i): the only choice for which the
    update w - h_ij v_i removes the v_i component.
  * Termination (Sec. 1.2): ||b - A x|| < tol * ||b - A x0||, or the operator
    has been applied ``maxit`` times.  Inside a cycle the least-squares
    residual min_y ||beta e_1 - H_j y|| is evaluated after every step and the
    cycle ends as soon as it drops below the target; the true residual
    b - A x computed at the next restart is what decides convergence.
  * Early stop near breakdown: |h_{j+1,j}| < tol/10 ends the cycle (the
    paper's DDalphaAMG rule).
  * The least-squares problem is solved with numpy.linalg.lstsq (a library
    primitive) rather than Givens rotations.
  * "iterations" are counted as operator applications (restart residuals
    included), the quantity the paper's Count columns report.
"""
from __future__ import annotations

import numpy as np


def _dot(v, w):
    """<w, v> = v^H w."""
    return np.vdot(v.ravel(), w.ravel())


def _norm(v):
    return float(np.sqrt(np.vdot(v.ravel(), v.ravel()).real))


def fgmres(apply_A, b, m: int, tol: float, maxit: int, x0=None, precond=None,
           history: list | None = None):
    """Solve A x = b.

    apply_A(v) and precond(v, j) take and return arrays shaped like b.
    precond=None means M_j = I.  Returns (x, info) where info holds
    'applies', 'restarts', 'converged', 'true_residual' (relative to
    ||b - A x0||) and 'breakdown'.  If ``history`` is a list, the relative
    least-squares residual after every inner step is appended to it.
    """
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    applies = 0
    restarts = 0
    r0norm = None
    converged = False
    breakdown = False
    relres = np.inf
    while True:
        r = b - apply_A(x)                               # restart: residual
        applies += 1
        beta = _norm(r)                                  # its norm beta
        if r0norm is None:
            r0norm = beta
            if r0norm == 0.0:
                converged = True
                relres = 0.0
                break
        relres = beta / r0norm
        if relres < tol:
            converged = True
            break
        if applies >= maxit or breakdown:
            break
        restarts += 1
        V = [r / beta]                                   # first basis vector
        Z = []
        H = np.zeros((m + 1, m), np.complex128)          # Hessenberg matrix
        e1 = np.zeros(m + 1, np.complex128)
        e1[0] = beta
        ncols = 0
        for j in range(m):                               # Arnoldi steps
            z = V[j] if precond is None else precond(V[j], j)   # preconditioned direction z_j
            Z.append(z)
            w = apply_A(z)                               # w = A z_j
            applies += 1
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = _dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = _norm(w)                       # h_{j+1,j}
            ncols = j + 1
            y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], e1[:j + 2], rcond=None)
            est = float(np.linalg.norm(e1[:j + 2] - H[:j + 2, :j + 1] @ y)) / r0norm
            if history is not None:
                history.append(est)
            if abs(H[j + 1, j]) < tol / 10.0:
                breakdown = True
                break
            if est < tol or applies >= maxit:
                break
            V.append(w / H[j + 1, j])                    # next basis vector
        y, *_ = np.linalg.lstsq(H[:ncols + 1, :ncols], e1[:ncols + 1], rcond=None)  # least squares for y
        for k in range(ncols):                           # x += Z y
            x = x + y[k] * Z[k]
    return x, {"applies": applies, "restarts": restarts, "converged": converged,
               "true_residual": relres, "breakdown": breakdown}
