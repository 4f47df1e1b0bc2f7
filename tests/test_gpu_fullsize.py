"""Oracle checks of the benchmark's full-size configurations that the other
files do not cover: plain FP64 FGMRES(30) on D and on the even-odd reduced
system S at 48^3 x 96 (Algorithm 2 at the benchmarked size), the 41-RHS FP32
launch over batches {1, 4, 12, 24}, FP32 S at sampled even sites, and the
32^4 operator with two-row links and compact clover in its autotuned launch."""
import numpy as np
import pytest
import torch

import oracle
from oracle import evenodd
from paper_2407_00041_amd import DiracOp, _lib, synth, tune_get, tune_set
from util import TOL, need_gpu, rel_l2

pytestmark = pytest.mark.gpu

DIMS48 = (96, 48, 48, 48)


def _links(dims, seed):
    Ud = synth.smooth_links(dims, seed, device="cuda")
    U = Ud.cpu().numpy()
    del Ud
    return U


def _true_relres(dims, U, m0, csw, x, b):
    r = b - oracle.dirac_apply(dims, U, x, m0, csw)
    return np.linalg.norm(r) / np.linalg.norm(b)


@pytest.fixture
def restore_tuning():
    need_gpu()
    keys = ("order", "block", "tchunk", "nr_f32")
    saved = {k: tune_get(k) for k in keys}
    explicit = tune_get("explicit")
    yield
    _lib.load().dirac_tune_clear()
    for k, v in saved.items():
        tune_set(k, v)
    tune_set("explicit", explicit)    # setting a knob marks the launch explicit: restore the flag last


@pytest.mark.parametrize("schur", [False, True])
def test_full_size_fp64_fgmres30(schur):
    """48^3 x 96, c_sw = 1, m0 = -0.35, two-row links and compact clover: the
    plain FP64 FGMRES(30) solve the benchmark compares the mixed solver with, on
    D and on S, to 1e-10; the full system's true residual of the returned
    solution is recomputed by the oracle operator over the whole lattice."""
    need_gpu()
    m0, csw = -0.35, 1.0
    U = _links(DIMS48, 1004)
    bd = synth.gaussian_spinor(DIMS48, 2401, nrhs=1, device="cuda")
    op = DiracOp(DIMS48, U, m0, csw, precisions=("f64",), compress_links=True, compress_clover=True,
                 even_odd=schur)
    bn = op.pack(bd, "f64")
    x, st, rc = op.solve(bn, restart=30, tol=1e-10, maxit=2000, schur=schur)
    assert rc == 0 and st[0]["converged"], st[0]
    assert st[0]["true_residual"] < 1e-10
    xg = op.unpack(x, "f64").cpu().numpy()[0]
    del op, x, bn
    torch.cuda.empty_cache()
    assert _true_relres(DIMS48, U, m0, csw, xg, bd.cpu().numpy()[0]) <= 1e-10 * 1.01


def test_full_size_41_rhs_batched_launch(restore_tuning):
    """48^3 x 96, FP32, two-row links, compact clover: the benchmark's one call
    over uneven batches {1, 4, 12, 24} (41 right-hand sides), in the
    configuration its autotuner selects and in the link-stationary kernel with
    launches of 6 right-hand sides over plane tiles and both z-pair walks;
    300 sampled sites of every right-hand side against the oracle."""
    m0, csw = -0.35, 1.0
    U = _links(DIMS48, 1003)
    op = DiracOp(DIMS48, U, m0, csw, precisions=("f64", "f32"), compress_links=True, compress_clover=True)
    V = op.V
    sizes = [1, 4, 12, 24]
    n = sum(sizes)
    psid = synth.gaussian_spinor(DIMS48, 2100, nrhs=n, device="cuda")
    nat = op.pack(psid, "f32")
    sites = synth.random_sites(DIMS48, 300, 17)
    st = torch.from_numpy(sites).cuda()
    want = []
    for r in range(n):
        want.append(oracle.dirac_apply_sites(DIMS48, U, psid[r].cpu().numpy(), sites, m0, csw))
    del psid
    torch.cuda.empty_cache()
    rb = op.field_bytes("f32", 1)
    tune_set("explicit", 0)
    cfg = op.autotune("f32", n)
    for explicit in (None, 1, 2, 4):
        if explicit:
            for k, v in (("order", 5), ("block", 128), ("tchunk", 6), ("nr_f32", explicit)):
                tune_set(k, v)
        outs, batches, r0 = [], [], 0
        for s in sizes:
            o = op.empty("f32", s)
            outs.append(o)
            batches.append((o, nat[r0 * rb:(r0 + s) * rb], s))
            r0 += s
        op.apply_batched(batches, "f32")
        r0 = 0
        for o, s in zip(outs, sizes):
            got = op.unpack(o, "f32", s).reshape(s, V, 12)[:, st].cpu().numpy()
            for k in range(s):
                assert rel_l2(got[k], want[r0 + k]) < TOL["f32"], (explicit, cfg, s, k)
            r0 += s
        del outs, batches
    del nat, op
    torch.cuda.empty_cache()


def test_full_size_reduced_operator_f32_sampled():
    """48^3 x 96 (benchmark operator, even-odd): FP32 S on a pair of
    right-hand sides at 192 sampled even sites against the oracle's
    neighbourhood evaluation of S."""
    need_gpu()
    m0, csw = -0.35, 1.0
    U = _links(DIMS48, 1006)
    op = DiracOp(DIMS48, U, m0, csw, precisions=("f64", "f32"), compress_links=True, compress_clover=True,
                 even_odd=True)
    psi = synth.gaussian_spinor(DIMS48, 2601, nrhs=2, device="cuda")
    even_sites = evenodd.sites_of(DIMS48, 0)
    rng = np.random.default_rng(14)
    pick = np.sort(rng.choice(len(even_sites), 192, replace=False))
    e, o = op.split(op.pack(psi, "f32"), "f32", 2)
    out, tmp = op.empty_parity("f32", 2), op.empty_parity("f32", 2)
    op.apply_schur_native(out, e, tmp, 2, "f32")
    o.zero_()
    got = op.unpack(op.merge(out, o, "f32", 2), "f32", 2)[:, torch.from_numpy(even_sites[pick]).cuda()]
    got = got.cpu().numpy()
    del e, o, out, tmp, op
    for r in range(2):
        xe = psi[r].cpu().numpy()[even_sites]
        want = evenodd.schur_sites(DIMS48, U, xe, even_sites[pick], m0, csw)
        assert rel_l2(got[r], want) < TOL["f32"], r
    torch.cuda.empty_cache()


def test_full_size_32_compressed_autotuned():
    """32^4, c_sw = 1, m0 = -0.3, two-row links and compact clover, the
    autotuned FP64 launch the 32^4 workload times (and FP32/FP16S): 1500
    sampled sites against the oracle."""
    need_gpu()
    dims = (32, 32, 32, 32)
    m0, csw = -0.3, 1.0
    U = _links(dims, 1002)
    psid = synth.gaussian_spinor(dims, 2000, nrhs=1, device="cuda")
    op = DiracOp(dims, U, m0, csw, precisions=("f64", "f32", "f16s"), compress_links=True, compress_clover=True)
    explicit = tune_get("explicit")
    tune_set("explicit", 0)
    try:
        sites = synth.random_sites(dims, 1500, 19)
        want = oracle.dirac_apply_sites(dims, U, psid.cpu().numpy()[0], sites, m0, csw)
        st = torch.from_numpy(sites).cuda()
        for prec in ("f64", "f32", "f16s"):
            op.autotune(prec, 1)
            got = op.apply(psid, prec).reshape(op.V, 12)[st].cpu().numpy()
            assert rel_l2(got, want) < TOL[prec], prec
    finally:
        _lib.load().dirac_tune_clear()
        tune_set("explicit", explicit)
    del op
    torch.cuda.empty_cache()
