"""Seeded synthetic inputs: gauge links and Gaussian spinors.

This module draws random numbers and shapes them into SU(3) links and
spinor fields.  It holds none of the operator's arithmetic, so both the CPU
oracle side and the GPU side of a test consume the very same arrays.

Recipes (the paper's own gauge field is not available, so these stand in
for it):

* ``haar_links``: Haar-random SU(3): QR of a 3x3 matrix of i.i.d. complex
  Gaussians (N(0,1) + i N(0,1)), phases of R's diagonal moved into Q, then
  Q / det(Q)^{1/3} (principal cube root).  NumPy PCG64.
* ``smooth_links``: U = exp(i eps H) with H = sum_a w_a lambda_a, w_a ~ N(0,1)
  and lambda_a the eight Gell-Mann matrices (tr lambda_a lambda_b = 2 delta),
  eps = 0.3.  The exponential uses scaling and squaring of a degree-18
  Taylor polynomial (truncation error below 1e-20 after scaling the norm
  under 1/16).  torch, so it runs on the GPU for the large lattices; the
  random numbers come from a seeded torch.Generator on the chosen device.
* ``gaussian_spinor``: Re and Im of every component i.i.d. N(0,1).

Layouts match the canonical host layouts of the library and the oracle:
links [V, 4, 3, 3] complex128 (mu = T,Z,Y,X), spinors [V, 12] complex128.
"""
from __future__ import annotations

import numpy as np
import torch

GELL_MANN = np.zeros((8, 3, 3), np.complex128)
GELL_MANN[0][0, 1] = GELL_MANN[0][1, 0] = 1
GELL_MANN[1][0, 1] = -1j
GELL_MANN[1][1, 0] = 1j
GELL_MANN[2][0, 0] = 1
GELL_MANN[2][1, 1] = -1
GELL_MANN[3][0, 2] = GELL_MANN[3][2, 0] = 1
GELL_MANN[4][0, 2] = -1j
GELL_MANN[4][2, 0] = 1j
GELL_MANN[5][1, 2] = GELL_MANN[5][2, 1] = 1
GELL_MANN[6][1, 2] = -1j
GELL_MANN[6][2, 1] = 1j
GELL_MANN[7][0, 0] = GELL_MANN[7][1, 1] = 1 / np.sqrt(3)
GELL_MANN[7][2, 2] = -2 / np.sqrt(3)


def volume(dims) -> int:
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def haar_su3(n: int, seed: int) -> np.ndarray:
    """n Haar-random SU(3) matrices, [n, 3, 3] complex128."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=1, axis2=2)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    return Q / (det ** (1.0 / 3.0))[:, None, None]


def haar_links(dims, seed: int) -> np.ndarray:
    V = volume(dims)
    return haar_su3(4 * V, seed).reshape(V, 4, 3, 3)


def _expm_batched(X: torch.Tensor) -> torch.Tensor:
    """exp of a batch of 3x3 complex matrices: scaling and squaring."""
    nrm = torch.linalg.matrix_norm(X, ord=1).max().item() if X.numel() else 0.0
    s = max(0, int(np.ceil(np.log2(max(nrm, 1e-300) * 16.0)))) if nrm > 0 else 0
    Y = X / (2.0 ** s)
    eye = torch.eye(3, dtype=X.dtype, device=X.device).expand_as(Y)
    out = eye.clone()
    term = eye.clone()
    for k in range(1, 19):
        term = torch.matmul(term, Y) / k
        out = out + term
    for _ in range(s):
        out = torch.matmul(out, out)
    return out


def smooth_su3(n: int, seed: int, eps: float = 0.3, device="cpu",
               chunk: int = 1 << 22) -> torch.Tensor:
    """n matrices exp(i eps H), H random traceless Hermitian; [n,3,3] complex128."""
    device = torch.device(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    lam = torch.as_tensor(GELL_MANN, device=device)
    out = torch.empty((n, 3, 3), dtype=torch.complex128, device=device)
    for s0 in range(0, n, chunk):
        m = min(chunk, n - s0)
        w = torch.randn((m, 8), generator=gen, dtype=torch.float64, device=device)
        H = torch.einsum("na,aij->nij", w.to(torch.complex128), lam)
        out[s0:s0 + m] = _expm_batched(1j * eps * H)
    return out


def smooth_links(dims, seed: int, eps: float = 0.3, device="cpu") -> torch.Tensor:
    V = volume(dims)
    return smooth_su3(4 * V, seed, eps, device).reshape(V, 4, 3, 3)


def gaussian_spinor(dims, seed: int, nrhs: int | None = None, device=None):
    """Gaussian spinor field(s): numpy [V,12] (device None) or torch on device.

    With nrhs given the shape is [nrhs, V, 12].
    """
    V = volume(dims)
    shape = (V, 12) if nrhs is None else (nrhs, V, 12)
    if device is None:
        rng = np.random.default_rng(seed)
        return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    device = torch.device(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    re = torch.randn(shape, generator=gen, dtype=torch.float64, device=device)
    im = torch.randn(shape, generator=gen, dtype=torch.float64, device=device)
    return torch.complex(re, im)


def random_sites(dims, n: int, seed: int) -> np.ndarray:
    """n distinct site indices, always including the lattice corners 0 and V-1."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    n = min(n, V)
    s = rng.choice(V, size=n, replace=False)
    s[0] = 0
    if n > 1:
        s[1] = V - 1
    return np.unique(s)
