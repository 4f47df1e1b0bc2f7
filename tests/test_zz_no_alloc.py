"""The allocation-free even-odd operator (dirac_apply_schur_noalloc) through
the C ABI: bit-identical to dirac_apply_schur with a caller's scratch, on two
calls in a row (the second on a smaller input), at every precision and for S
and S^H; a request beyond its static scratch is rejected."""
import ctypes

import pytest
import torch

from paper_2407_00041_amd import DiracOp, _lib, synth
from util import need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _op(dims, seed):
    U = synth.smooth_links(dims, seed).numpy()
    return DiracOp(dims, U, -0.3, 1.0, precisions=("f64", "f32", "f16s"), compress_links=True,
                   compress_clover=True, even_odd=True)


def test_noalloc_schur_equals_schur_with_workspace():
    need_gpu()
    lib = _lib.load()
    st = torch.cuda.current_stream().cuda_stream
    for dims, nrhs, seed in (((8, 8, 8, 8), 3, 90), ((4, 4, 4, 6), 1, 91)):
        op = _op(dims, seed)
        psi = to_dev(synth.gaussian_spinor(dims, seed + 10, nrhs=nrhs))
        for prec in ("f64", "f32", "f16s"):
            e, _ = op.split(op.pack(psi, prec), prec, nrhs)
            for dag in (False, True):
                ref, tmp = op.empty_parity(prec, nrhs), op.empty_parity(prec, nrhs)
                op.apply_schur_native(ref, e, tmp, nrhs, prec, dagger=dag)
                got = op.empty_parity(prec, nrhs)
                got.fill_(7)
                rc = lib.dirac_apply_schur_noalloc(op.handle, got.data_ptr(), e.data_ptr(), nrhs,
                                                   {"f64": 0, "f32": 1, "f16s": 2}[prec], int(dag), st)
                assert rc == 0, lib.dirac_last_error()
                torch.cuda.synchronize()
                assert torch.equal(got, ref), (dims, prec, dag)
        op.close()


def test_noalloc_schur_rejects_more_than_its_scratch():
    need_gpu()
    lib = _lib.load()
    dims = (16, 16, 16, 16)
    op = _op(dims, 92)
    nrhs = 22                          # 22 FP64 odd fields of 6.3 MB: above 128 MiB
    assert op.parity_field_bytes("f64", nrhs) > (128 << 20)
    e = op.empty_parity("f64", nrhs)
    e.zero_()
    out = op.empty_parity("f64", nrhs)
    rc = lib.dirac_apply_schur_noalloc(op.handle, out.data_ptr(), e.data_ptr(), nrhs, 0, 0,
                                       torch.cuda.current_stream().cuda_stream)
    assert rc == _lib.EINVAL and b"static scratch" in lib.dirac_last_error()
    op.close()
