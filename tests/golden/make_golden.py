"""Writes the regression fixtures of this directory from the FP64 CPU oracle.

    python tests/golden/make_golden.py

Calls only ``oracle/`` (and the seeded input generators of synth.py, which
hold none of the operator's arithmetic).  The paper prints no worked
numerical example of the operator, so these fixtures are not the paper's
values: they freeze the oracle's results for small seeded inputs, so that a
later change of the oracle's arithmetic shows up in a test and has to be
justified; the oracle itself is pinned by the closed-form and brute-force
tests in tests/test_oracle_*.py.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2407_00041_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def cplx(a):
    a = np.asarray(a, dtype=np.complex128).ravel()
    return [[float(z.real), float(z.imag)] for z in a]


def wilson_clover():
    # a ragged, non-cubic lattice with one extent 2 (x + mu = x - mu there), anti-periodic T
    dims, m0, csw = (3, 2, 4, 2), -0.4, 1.25
    U = synth.haar_links(dims, 5)
    psi = synth.gaussian_spinor(dims, 6)
    sites = [0, 17, 47]
    return {
        "about": "Wilson-clover operator of Eq. (1.13) with the clover term of Eqs. (1.11)-(1.12), FP64 oracle",
        "dims": list(dims), "m0": m0, "csw": csw, "antiperiodic_t": True,
        "links": "synth.haar_links(dims, 5)", "psi": "synth.gaussian_spinor(dims, 6)",
        "D_psi": cplx(oracle.dirac_apply(dims, U, psi, m0, csw, antiperiodic_t=True)),
        "Ddag_psi_sites": sites,
        "Ddag_psi": cplx(oracle.dirac_apply(dims, U, psi, m0, csw, antiperiodic_t=True, dagger=True)[sites]),
        "clover_site0": cplx(oracle.clover_term(dims, U)[0]),
    }


def fgmres():
    # Algorithm 2 with M = I on a 2^4 lattice, restart 10, to 1e-10
    dims, m0, csw = (2, 2, 2, 2), -0.3, 1.0
    U = synth.smooth_links(dims, 7).numpy()
    b = synth.gaussian_spinor(dims, 8)
    hist = []
    x, info = oracle.fgmres(lambda v: oracle.dirac_apply(dims, U, v, m0, csw), b, m=10, tol=1e-10, maxit=500,
                            history=hist)
    r = b - oracle.dirac_apply(dims, U, x, m0, csw)
    return {
        "about": "FGMRES (Algorithm 2, modified Gram-Schmidt, M = I), FP64 oracle",
        "dims": list(dims), "m0": m0, "csw": csw, "restart": 10, "tol": 1e-10,
        "links": "synth.smooth_links(dims, 7)", "b": "synth.gaussian_spinor(dims, 8)",
        "applies": int(info["applies"]),
        "true_relres": float(np.linalg.norm(r) / np.linalg.norm(b)),
        "hist": [float(h) for h in hist],
    }


if __name__ == "__main__":
    oracle.build(force=False)
    for name, fn in (("wilson_clover_3x2x4x2.json", wilson_clover), ("fgmres_2x2x2x2.json", fgmres)):
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(fn(), f, indent=1)
            f.write("\n")
        print("wrote", name)
