"""Differentiation: the link-derivative kernel against the oracle's exact
derivative, central finite differences through the GPU apply, and
torch.autograd.gradcheck of the autograd Function (dL/dx = D^H g, dL/dU)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2407_00041_amd import DiracOp, synth
from paper_2407_00041_amd.autograd import dirac_apply
from util import need_gpu, rel_l2, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,csw,ap,kind", [((4, 4, 4, 4), 1.0, False, "smooth"),
                                              ((2, 2, 2, 2), 1.0, True, "haar"),
                                              ((3, 4, 2, 4), 0.0, True, "haar"),
                                              ((4, 2, 6, 2), 1.3, False, "haar"),
                                              # 720 sites per T-slice: six 128-site eighths, the last one ragged
                                              # (80 sites), two XCDs without a tile in each slice
                                              ((3, 6, 10, 12), 1.0, True, "haar")])
def test_force_matches_oracle_every_link(dims, csw, ap, kind):
    need_gpu()
    V = synth.volume(dims)
    U = synth.smooth_links(dims, 4).numpy() if kind == "smooth" else synth.haar_links(dims, 4)
    x = synth.gaussian_spinor(dims, 5, nrhs=2)
    eta = synth.gaussian_spinor(dims, 6, nrhs=2)
    op = DiracOp(dims, U, -0.3, csw, antiperiodic_t=ap, precisions=("f64",))
    xn, en = op.pack(to_dev(x), "f64"), op.pack(to_dev(eta), "f64")
    G = op.force(en, xn, 2, raw=True).cpu().numpy()
    F = op.force(en, xn, 2).cpu().numpy()
    sites = np.repeat(np.arange(V), 4)
    dirs = np.tile(np.arange(4), V)
    Go, Fo = oracle.force_links(dims, U, eta, x, sites, dirs, csw=csw, antiperiodic_t=ap)
    assert rel_l2(G.reshape(-1, 3, 3), Go) < 1e-12
    assert rel_l2(F.reshape(-1, 3, 3), Fo) < 1e-12


def test_force_full_size_24_48_sampled_and_fd():
    """24^3 x 48, c_sw = 1: 64 random links against the oracle and against
    central differences (h = 1e-6) of L = Re<eta, D(U) x> through the GPU
    apply (the link moved along a random su(3) generator each time)."""
    need_gpu()
    dims = (48, 24, 24, 24)
    V = synth.volume(dims)
    m0, csw = -0.3, 1.0
    U = synth.smooth_links(dims, 77, device="cuda").cpu().numpy()
    x = synth.gaussian_spinor(dims, 78, nrhs=1, device="cuda")
    eta = synth.gaussian_spinor(dims, 79, nrhs=1, device="cuda")
    op = DiracOp(dims, U, m0, csw, precisions=("f64",))
    xn, en = op.pack(x, "f64"), op.pack(eta, "f64")
    G = op.force(en, xn, 1, raw=True).reshape(V, 4, 3, 3)
    F = op.force(en, xn, 1).reshape(V, 4, 3, 3)
    rng = np.random.default_rng(3)
    sites = rng.integers(0, V, 64)
    dirs = rng.integers(0, 4, 64)
    Go, Fo = oracle.force_links(dims, U, eta.cpu().numpy(), x.cpu().numpy(), sites, dirs, csw=csw)
    s_t, d_t = torch.from_numpy(sites).cuda(), torch.from_numpy(dirs).cuda()
    assert rel_l2(G[s_t, d_t].cpu().numpy(), Go) < 1e-12
    assert rel_l2(F[s_t, d_t].cpu().numpy(), Fo) < 1e-12
    h = 1e-6
    for k in range(64):
        a = int(rng.integers(0, 8))
        T = 0.5j * synth.GELL_MANN[a]
        ev, W = np.linalg.eigh(-1j * T)                   # T = i W diag(ev) W^H
        dL = 0.0
        outs = []
        for sgn in (+1, -1):
            Up = U.copy()
            E = W @ np.diag(np.exp(1j * sgn * h * ev)) @ W.conj().T   # exp(+-h T)
            Up[sites[k], dirs[k]] = E @ U[sites[k], dirs[k]]
            opp = DiracOp(dims, Up, m0, csw, precisions=("f64",))
            outs.append(opp.apply(x, "f64"))
            del opp
        dL = torch.sum((torch.conj(eta) * (outs[0] - outs[1])).real).item() / (2 * h)
        want = np.trace(np.conj(Fo[k]).T @ T).real
        assert abs(dL - want) <= 1e-6 * max(1.0, abs(want)), (k, dL, want)


def test_autograd_dx_is_adjoint_apply():
    need_gpu()
    dims = (4, 4, 4, 4)
    U = synth.smooth_links(dims, 9).numpy()
    op = DiracOp(dims, U, -0.3, 1.0, precisions=("f64",))
    x = to_dev(synth.gaussian_spinor(dims, 10, nrhs=2)).requires_grad_(True)
    g = to_dev(synth.gaussian_spinor(dims, 11, nrhs=2))
    y = dirac_apply(x, None, dims, op=op)
    y.backward(g)
    want = op.apply(g, "f64", dagger=True)
    assert torch.allclose(x.grad, want, rtol=0, atol=0)


def test_gradcheck_x_and_links():
    need_gpu()
    dims = (2, 2, 2, 2)
    U = torch.from_numpy(synth.haar_links(dims, 12)).cuda()
    x = to_dev(synth.gaussian_spinor(dims, 13, nrhs=1))
    Ur = U.clone().requires_grad_(True)
    xr = x.clone().requires_grad_(True)
    f = lambda xx, uu: dirac_apply(xx, uu, dims, op=None, m0=-0.2, csw=1.0, antiperiodic_t=True)
    assert torch.autograd.gradcheck(f, (xr, Ur), eps=1e-6, atol=1e-7, rtol=1e-6, fast_mode=True)


def test_force_workspace_size_and_rejection():
    """The clover pass needs 6 planes x 80 B per site of workspace; without
    clover none; a short workspace is rejected before any launch."""
    need_gpu()
    import ctypes
    from paper_2407_00041_amd import _lib
    dims = (2, 2, 4, 2)
    V = synth.volume(dims)
    U = synth.haar_links(dims, 21)
    x = to_dev(synth.gaussian_spinor(dims, 22, nrhs=1))
    op = DiracOp(dims, U, -0.3, 1.0, precisions=("f64",))
    op0 = DiracOp(dims, U, -0.3, 0.0, precisions=("f64",))
    assert op.lib.dirac_force_workspace_bytes(op.handle) == 6 * 80 * V
    assert op0.lib.dirac_force_workspace_bytes(op0.handle) == 0
    xn = op.pack(x, "f64")
    out = torch.empty((V, 4, 3, 3), dtype=torch.complex128, device="cuda")
    work = torch.empty(6 * 80 * V - 16, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    rc = op.lib.dirac_force(op.handle, out.data_ptr(), xn.data_ptr(), xn.data_ptr(), 1, 0, work.data_ptr(),
                            work.numel(), s)
    assert rc == _lib.EINVAL
    rc = op.lib.dirac_force(op.handle, out.data_ptr(), xn.data_ptr(), xn.data_ptr(), 1, 0, None, 0, s)
    assert rc == _lib.EINVAL
    G0 = op0.force(xn, xn, 1, raw=True)
    rc = op0.lib.dirac_force(op0.handle, out.data_ptr(), xn.data_ptr(), xn.data_ptr(), 1, 1, None, 0, s)
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(out, G0)
