"""Regression fixtures in tests/golden (written by tests/golden/make_golden.py
from the FP64 oracle): the oracle must keep reproducing them, and the GPU
path must match them at each precision's tolerance."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2407_00041_amd import synth
from util import TOL, need_gpu, rel_l2

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def as_c128(pairs, shape):
    a = np.asarray(pairs, dtype=np.float64)
    return (a[:, 0] + 1j * a[:, 1]).reshape(shape)


def wc_inputs(g):
    dims = tuple(g["dims"])
    return dims, synth.haar_links(dims, 5), synth.gaussian_spinor(dims, 6)


def test_oracle_reproduces_wilson_clover_fixture():
    g = load("wilson_clover_3x2x4x2.json")
    dims, U, psi = wc_inputs(g)
    V = synth.volume(dims)
    got = oracle.dirac_apply(dims, U, psi, g["m0"], g["csw"], antiperiodic_t=g["antiperiodic_t"])
    assert rel_l2(got, as_c128(g["D_psi"], (V, 12))) < 1e-14
    sites = g["Ddag_psi_sites"]
    gotd = oracle.dirac_apply(dims, U, psi, g["m0"], g["csw"], antiperiodic_t=True, dagger=True)[sites]
    assert rel_l2(gotd, as_c128(g["Ddag_psi"], (len(sites), 12))) < 1e-14
    assert rel_l2(oracle.clover_term(dims, U)[0], as_c128(g["clover_site0"], (42,))) < 1e-14


def test_oracle_reproduces_fgmres_fixture():
    g = load("fgmres_2x2x2x2.json")
    dims = tuple(g["dims"])
    U = synth.smooth_links(dims, 7).numpy()
    b = synth.gaussian_spinor(dims, 8)
    hist = []
    x, info = oracle.fgmres(lambda v: oracle.dirac_apply(dims, U, v, g["m0"], g["csw"]), b, m=g["restart"],
                            tol=g["tol"], maxit=500, history=hist)
    assert info["applies"] == g["applies"]
    # the residual estimates come from LAPACK least squares, whose rounding
    # differs between CPUs: relative 1e-8, absolute 1e-13 (of ||r0|| = 1)
    assert np.allclose(hist, g["hist"], rtol=1e-8, atol=1e-13)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_gpu_matches_wilson_clover_fixture(prec):
    need_gpu()
    from paper_2407_00041_amd import DiracOp
    g = load("wilson_clover_3x2x4x2.json")
    dims, U, psi = wc_inputs(g)
    V = synth.volume(dims)
    op = DiracOp(dims, U, g["m0"], g["csw"], antiperiodic_t=True)
    x = torch.from_numpy(psi).to("cuda")
    got = op.apply(x, prec).cpu().numpy()
    assert rel_l2(got, as_c128(g["D_psi"], (V, 12))) < TOL[prec]
    gotd = op.apply(x, prec, dagger=True).cpu().numpy()[g["Ddag_psi_sites"]]
    assert rel_l2(gotd, as_c128(g["Ddag_psi"], (len(g["Ddag_psi_sites"]), 12))) < TOL[prec]


@pytest.mark.gpu
def test_gpu_fgmres_matches_fixture_count():
    need_gpu()
    from paper_2407_00041_amd import DiracOp
    g = load("fgmres_2x2x2x2.json")
    dims = tuple(g["dims"])
    U = synth.smooth_links(dims, 7).numpy()
    b = synth.gaussian_spinor(dims, 8)
    op = DiracOp(dims, U, g["m0"], g["csw"], precisions=("f64",))
    bn = op.pack(torch.from_numpy(b).to("cuda"), "f64")
    x, st, rc = op.solve(bn, restart=g["restart"], tol=g["tol"], maxit=500)
    assert rc == 0 and abs(st[0]["applies"] - g["applies"]) <= 2
