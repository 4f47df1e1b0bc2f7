"""GPU FGMRES (Algorithm 2) through the C ABI against the oracle FGMRES:
same operator-application count (the paper's regression criterion), same
residual history, and a true residual verified with the oracle operator."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2407_00041_amd import DiracOp, WdiracError, synth
from util import fields, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def setup(dims, seed, m0, csw=1.0, nrhs=1, precisions=("f64", "f32", "f16s")):
    U = synth.smooth_links(dims, seed).numpy()
    b = synth.gaussian_spinor(dims, seed + 1, nrhs=nrhs)
    op = DiracOp(dims, U, m0, csw, precisions=precisions)
    bn = op.pack(to_dev(b), "f64")
    return U, b, op, bn


def true_relres(dims, U, m0, csw, x, b):
    r = b - oracle.dirac_apply(dims, U, x, m0, csw)
    return np.linalg.norm(r) / np.linalg.norm(b)


@pytest.mark.parametrize("dims,m", [((4, 4, 4, 4), 20), ((8, 4, 6, 4), 10), ((8, 8, 8, 8), 20)])
def test_fp64_matches_oracle_fgmres(dims, m):
    need_gpu()
    m0, csw = -0.3, 1.0
    U, b, op, bn = setup(dims, 1000, m0, csw)
    x, st, rc = op.solve(bn, restart=m, tol=1e-10, maxit=3000)
    assert rc == 0 and st[0]["converged"]
    xg = op.unpack(x, "f64").cpu().numpy()[0]
    hist = []
    A = lambda v: oracle.dirac_apply(dims, U, v, m0, csw)
    xo, info = oracle.fgmres(A, b, m=m, tol=1e-10, maxit=3000, history=hist)
    assert abs(st[0]["applies"] - info["applies"]) <= 2, (st[0]["applies"], info["applies"])
    k = 0
    while k < min(len(hist), len(st[0]["hist"])) and hist[k] > 1e-9:
        assert abs(st[0]["hist"][k] - hist[k]) <= 1e-8 * hist[k], (k, st[0]["hist"][k], hist[k])
        k += 1
    assert true_relres(dims, U, m0, csw, xg, b) <= 1e-10 * 1.01
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) < 1e-8


@pytest.mark.parametrize("mode", ["mixed_f32", "mixed_f16s"])
def test_mixed_precision_reaches_fp64_tolerance(mode):
    need_gpu()
    dims = (8, 8, 8, 8)
    m0, csw = -0.35, 1.0
    U, b, op, bn = setup(dims, 3, m0, csw)
    x, st, rc = op.solve(bn, restart=10, tol=1e-10, maxit=200, mode=mode, inner_restart=30, inner_tol=1e-2,
                         inner_maxit=30)
    assert rc == 0 and st[0]["converged"], st[0]
    assert st[0]["inner_applies"] > 0
    phases = st[0]["seconds_apply"] + st[0]["seconds_precond"] + st[0]["seconds_ortho"]
    assert st[0]["seconds_apply"] > 0 and st[0]["seconds_precond"] > 0 and st[0]["seconds_ortho"] > 0
    assert phases <= st[0]["seconds"] * 1.05
    xg = op.unpack(x, "f64").cpu().numpy()[0]
    assert true_relres(dims, U, m0, csw, xg, b) <= 1e-10 * 1.01
    x64, st64, _ = op.solve(bn, restart=20, tol=1e-10, maxit=3000)
    x64 = op.unpack(x64, "f64").cpu().numpy()[0]
    # both solutions satisfy the same residual bound, so they agree to about cond * 1e-10
    assert np.linalg.norm(xg - x64) / np.linalg.norm(x64) < 1e-8


@pytest.mark.parametrize("mode", ["f64", "mixed_f32", "mixed_f16s"])
def test_multi_rhs_equals_single_solves(mode):
    need_gpu()
    dims = (4, 4, 6, 4)
    U, b, op, bn = setup(dims, 5, -0.3, 1.0, nrhs=3)
    x, st, rc = op.solve(bn, nrhs=3, restart=8, tol=1e-10, maxit=2000, mode=mode)
    assert rc == 0
    rb = op.field_bytes("f64", 1)
    for r in range(3):
        xr, sr, _ = op.solve(bn[r * rb:(r + 1) * rb], nrhs=1, restart=8, tol=1e-10, maxit=2000, mode=mode)
        assert torch.equal(x[r * rb:(r + 1) * rb], xr)
        assert sr[0]["applies"] == st[r]["applies"]


@pytest.mark.parametrize("mode", ["mixed_f32", "mixed_f16s"])
def test_graph_inner_cycles_equal_stepwise(mode):
    """Inner cycles replayed as captured graphs give bit-identical iterates to
    the step-by-step issue, on every replay (graphs are replayed across outer
    steps and restarts; eager solves run between the graph solves)."""
    need_gpu()
    dims = (4, 4, 6, 4)
    U, b, op, bn = setup(dims, 7, -0.3, 1.0, nrhs=3)
    kw = dict(nrhs=3, restart=6, tol=1e-10, maxit=500, mode=mode, inner_restart=12, inner_tol=0.05, inner_maxit=12)
    xe, se, rc = op.solve(bn, **kw)
    assert rc == 0
    for rep in range(3):
        xg, sg, rcg = op.solve(bn, graph=True, **kw)
        assert rcg == 0
        assert torch.equal(xg, xe), rep
        for r in range(3):
            assert sg[r]["applies"] == se[r]["applies"]
            assert sg[r]["inner_applies"] == se[r]["inner_applies"]
            assert sg[r]["hist"] == se[r]["hist"]
        xe2, _, _ = op.solve(bn, **kw)  # eager work between graph solves
        assert torch.equal(xe2, xe)


@pytest.mark.parametrize("graph", [False, True])
def test_inner_gmres_near_exact_on_2x4(graph):
    """On a 2^4 lattice (dimension 192) an inner GMRES(192) to 1e-5 is nearly
    the exact inverse, so the outer FGMRES needs only a few FP64 applications
    (the exact-preconditioner limit of Algorithm 2); this exercises the
    device-side Givens rotations and triangular solve over long cycles."""
    need_gpu()
    dims = (2, 2, 2, 2)
    m0, csw = -0.3, 1.0
    U, b, op, bn = setup(dims, 11, m0, csw)
    x, st, rc = op.solve(bn, restart=10, tol=1e-10, maxit=50, mode="mixed_f32", inner_restart=192, inner_tol=1e-5,
                         inner_maxit=192, graph=graph)
    assert rc == 0 and st[0]["converged"], st[0]
    assert st[0]["applies"] <= 5, st[0]
    xg = op.unpack(x, "f64").cpu().numpy()[0]
    assert true_relres(dims, U, m0, csw, xg, b) <= 1e-10 * 1.01


@pytest.mark.parametrize("mode", ["f64", "mixed_f16s"])
def test_waves_equal_one_lockstep_solve(mode):
    """Five right-hand sides in waves of 2 (one workspace sized for a wave) give
    the same solutions, bit for bit, as all five in one lockstep solve."""
    need_gpu()
    dims = (4, 4, 6, 4)
    U, b, op, bn = setup(dims, 9, -0.3, 1.0, nrhs=5)
    kw = dict(nrhs=5, restart=8, tol=1e-10, maxit=2000, mode=mode, inner_restart=10, inner_tol=0.1, inner_maxit=10)
    x_all, s_all, rc = op.solve(bn, **kw)
    assert rc == 0
    wb = op.workspace_bytes(5, 8, mode, 10, wave=2)
    assert wb < op.workspace_bytes(5, 8, mode, 10)
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    x_w, s_w, rc = op.solve(bn, wave=2, work=work, **kw)
    assert rc == 0
    assert torch.equal(x_w, x_all)
    assert [s["applies"] for s in s_w] == [s["applies"] for s in s_all]


def test_maxit_zero_rhs_and_warm_start():
    need_gpu()
    dims = (4, 4, 4, 4)
    m0, csw = -0.3, 1.0
    U, b, op, bn = setup(dims, 7, m0, csw)
    x, st, rc = op.solve(bn, restart=5, tol=1e-12, maxit=13)
    assert rc == 1 and not st[0]["converged"] and st[0]["applies"] == 13
    A = lambda v: oracle.dirac_apply(dims, U, v, m0, csw)
    xo, info = oracle.fgmres(A, b, m=5, tol=1e-12, maxit=13)
    assert info["applies"] == 13
    assert np.linalg.norm(op.unpack(x, "f64").cpu().numpy()[0] - xo) / np.linalg.norm(xo) < 1e-10
    # resume from the returned iterate
    x2, st2, rc2 = op.solve(bn, x0=x, restart=20, tol=1e-10, maxit=3000)
    assert rc2 == 0 and st2[0]["converged"]
    # b = 0: converged immediately with one application
    z = torch.zeros_like(bn)
    x3, st3, rc3 = op.solve(z, restart=5, tol=1e-10, maxit=50)
    assert rc3 == 0 and st3[0]["applies"] == 1 and not x3.any()


def test_solver_argument_errors():
    need_gpu()
    dims = (2, 2, 2, 4)
    U, b, op, bn = setup(dims, 1, -0.3, 1.0, precisions=("f64",))
    with pytest.raises(WdiracError) as e:
        op.solve(bn, mode="mixed_f16s")
    assert e.value.code == -1 or e.value.code == -4
    with pytest.raises(WdiracError):
        op.solve(bn, restart=0)


def test_full_size_fp64_fgmres_32():
    """32^4, c_sw = 1, m0 = -0.3, FGMRES(20) to 1e-10 (the FP64 solver workload):
    the true residual of the GPU solution, checked by the oracle operator."""
    need_gpu()
    dims = (32, 32, 32, 32)
    m0, csw = -0.3, 1.0
    Ud = synth.smooth_links(dims, 1002, device="cuda")
    bd = synth.gaussian_spinor(dims, 2000, nrhs=1, device="cuda")
    U = Ud.cpu().numpy()
    op = DiracOp(dims, U, m0, csw, precisions=("f64",))
    bn = op.pack(bd, "f64")
    x, st, rc = op.solve(bn, restart=20, tol=1e-10, maxit=3000)
    assert rc == 0 and st[0]["converged"]
    xg = op.unpack(x, "f64").cpu().numpy()[0]
    assert true_relres(dims, U, m0, csw, xg, bd.cpu().numpy()[0]) <= 1e-10 * 1.01


def test_full_size_mixed_fgmres_bench_configuration():
    """48^3 x 96, c_sw = 1, m0 = -0.35, two-row links and compact clover, the
    benchmark's mixed solver (FP64 FGMRES(8), inner GMRES(10) on the FP16S
    operator to 0.1) to 1e-10: the true residual of the GPU solution, computed
    by the oracle operator over the whole lattice."""
    need_gpu()
    dims = (96, 48, 48, 48)
    m0, csw = -0.35, 1.0
    Ud = synth.smooth_links(dims, 1004, device="cuda")
    bd = synth.gaussian_spinor(dims, 2400, nrhs=1, device="cuda")
    U = Ud.cpu().numpy()
    del Ud
    op = DiracOp(dims, U, m0, csw, precisions=("f64", "f16s"), compress_links=True, compress_clover=True)
    bn = op.pack(bd, "f64")
    x, st, rc = op.solve(bn, restart=8, tol=1e-10, maxit=500, mode="mixed_f16s", inner_restart=10, inner_tol=0.1,
                         inner_maxit=10)
    assert rc == 0 and st[0]["converged"], st[0]
    assert st[0]["true_residual"] < 1e-10
    xg = op.unpack(x, "f64").cpu().numpy()[0]
    del op, x, bn
    torch.cuda.empty_cache()
    assert true_relres(dims, U, m0, csw, xg, bd.cpu().numpy()[0]) <= 1e-10 * 1.01


@pytest.mark.parametrize("schur", [False, True])
@pytest.mark.parametrize("where", ["b", "x0"])
def test_nonfinite_input_is_reported_not_converged(schur, where):
    """A NaN in one right-hand side's b (or x0) of a 3-RHS lockstep solve is
    reported as its own outcome (nonfinite, not converged, true residual NaN,
    status ENONFINITE, x left at x0), and the other two right-hand sides are
    solved exactly as their single solves, bit for bit."""
    need_gpu()
    from paper_2407_00041_amd import ENONFINITE
    dims = (4, 4, 6, 4)
    U = synth.smooth_links(dims, 21).numpy()
    b = synth.gaussian_spinor(dims, 22, nrhs=3)
    op = DiracOp(dims, U, -0.3, 1.0, precisions=("f64",), even_odd=True)
    bn = op.pack(to_dev(b), "f64")
    rb = op.field_bytes("f64", 1)
    x0 = torch.zeros_like(bn)
    bad = bn.clone() if where == "b" else bn
    tgt = bad if where == "b" else x0
    v = tgt[rb:2 * rb].view(torch.float64)
    v[17] = float("nan")
    kw = dict(nrhs=3, restart=8, tol=1e-10, maxit=2000, schur=schur)
    x0_before = x0.clone()
    x, st, rc = op.solve(bad, x0=x0, **kw)
    assert rc == ENONFINITE
    assert st[1]["nonfinite"] and not st[1]["converged"]
    assert np.isnan(st[1]["true_residual"])
    assert torch.equal(x[rb:2 * rb].view(torch.float64).nan_to_num(123.0),
                       x0_before[rb:2 * rb].view(torch.float64).nan_to_num(123.0))
    for r in (0, 2):
        assert not st[r]["nonfinite"] and st[r]["converged"]
        xr, sr, rcr = op.solve(bn[r * rb:(r + 1) * rb], nrhs=1, restart=8, tol=1e-10, maxit=2000, schur=schur)
        assert rcr == 0
        assert torch.equal(x[r * rb:(r + 1) * rb], xr), r
        assert sr[0]["applies"] == st[r]["applies"]
        assert sr[0]["hist"] == st[r]["hist"]


def test_library_chosen_wave():
    """wave = 0: fgmres_workspace_bytes sizes a wave from the free device
    memory (a whole number of right-hand sides), and fgmres_solve runs as many
    right-hand sides per wave as the workspace it is given holds, reporting
    the wave in the stats; the solutions equal one lockstep solve."""
    need_gpu()
    dims = (4, 4, 6, 4)
    U, b, op, bn = setup(dims, 9, -0.3, 1.0, nrhs=5, precisions=("f64",))
    per = op.workspace_bytes(1, 8, "f64", wave=1)
    auto = op.workspace_bytes(5, 8, "f64", wave=0)
    assert auto == 5 * per  # a tiny lattice: all five fit
    kw = dict(nrhs=5, restart=8, tol=1e-10, maxit=2000)
    x_all, s_all, rc = op.solve(bn, **kw)
    assert rc == 0 and all(s["wave"] == 5 for s in s_all)
    work = torch.empty(2 * per + 100, dtype=torch.uint8, device="cuda")
    x_w, s_w, rc = op.solve(bn, wave=0, work=work, **kw)
    assert rc == 0 and all(s["wave"] == 2 for s in s_w)
    assert torch.equal(x_w, x_all)
    # a workspace smaller than one right-hand side's is rejected
    from paper_2407_00041_amd import _lib
    small = torch.empty(per, dtype=torch.uint8, device="cuda")
    x = torch.zeros_like(bn)
    stats = (_lib.FgmresStats * 5)()
    p = op._params(8, 1e-10, 2000, "f64", 30, 1e-2, 30)
    rc = op.lib.fgmres_solve(op.handle, x.data_ptr(), bn.data_ptr(), 5, ctypes.byref(p), stats, small.data_ptr(),
                             per - 256, torch.cuda.current_stream().cuda_stream)
    assert rc == _lib.EINVAL and b"workspace too small" in op.lib.dirac_last_error()


def test_create_rejects_nonfinite_links_and_clover():
    need_gpu()
    dims = (2, 2, 2, 4)
    U = synth.smooth_links(dims, 3).numpy()
    bad = U.copy()
    bad[5, 2, 1, 1] = complex(np.inf, 0.0)
    with pytest.raises(WdiracError) as e:
        DiracOp(dims, bad, -0.3, 1.0, precisions=("f64",))
    assert e.value.code == -1 and "NaN or Inf" in str(e.value)
    C = oracle.clover_term(dims, U)
    C[3, 7] = complex(0.0, np.nan)
    with pytest.raises(WdiracError) as e:
        DiracOp(dims, U, -0.3, 1.0, clover=C, precisions=("f64",))
    assert e.value.code == -1 and "NaN or Inf" in str(e.value)
