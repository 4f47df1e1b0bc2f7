"""Shared helpers of the test-suite (inputs, norms, GPU availability)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2407_00041_amd import synth

TOL = {"f64": 1e-13, "f32": 1e-6, "f16s": 5e-3}


def have_gpu() -> bool:
    return torch.cuda.is_available()


def need_gpu():
    if not have_gpu():
        pytest.skip("no GPU")


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def fields(dims, seed: int, kind: str = "smooth", nrhs: int = 1):
    """(links [V,4,3,3], psi [nrhs,V,12]) as host numpy complex128."""
    if kind == "haar":
        U = synth.haar_links(dims, seed)
    elif kind == "unit":
        V = synth.volume(dims)
        U = np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3)).copy()
    else:
        U = synth.smooth_links(dims, seed).numpy()
    psi = synth.gaussian_spinor(dims, seed + 1000, nrhs=nrhs)
    return U, psi


def to_dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()
