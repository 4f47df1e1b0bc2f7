"""Register-blocked multi-RHS applies, the persistent batched launch and the
launch-parameter knobs: every right-hand side must equal its own single
apply bit for bit (the arithmetic per right-hand side does not depend on the
blocking or the tile order) and the oracle within tolerance."""
import numpy as np
import pytest
import torch

import oracle
from paper_2407_00041_amd import DiracOp, TUNE_KEYS, WdiracError, tune_get, tune_set
from util import TOL, fields, need_gpu, rel_l2, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture
def restore_tuning():
    need_gpu()
    saved = {k: tune_get(k) for k in TUNE_KEYS}
    yield
    for k, v in saved.items():
        tune_set(k, v)


def singles(op, nat, prec, nrhs, dagger=False):
    rb = op.field_bytes(prec, 1)
    out = []
    for r in range(nrhs):
        o = op.empty(prec, 1)
        op.apply_native(o, nat[r * rb:(r + 1) * rb], 1, prec, dagger)
        out.append(o)
    return torch.cat(out)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("nr", [1, 2, 4])
def test_register_blocks_match_single_applies(prec, nr, restore_tuning):
    dims = (4, 6, 4, 10)
    U, psi = fields(dims, 21, nrhs=7)
    op = DiracOp(dims, U, -0.3, 1.0, antiperiodic_t=True)
    nat = op.pack(to_dev(psi), prec)
    tune_set("nr_" + prec, nr)
    for dag in (False, True):
        out = op.empty(prec, 7)
        op.apply_native(out, nat, 7, prec, dag)
        ref = singles(op, nat, prec, 7, dag)
        assert torch.equal(out, ref)
    got = op.unpack(out, prec, 7).cpu().numpy()
    want = oracle.dirac_apply(dims, U, psi, -0.3, 1.0, antiperiodic_t=True, dagger=True)
    for r in range(7):
        assert rel_l2(got[r], want[r]) < TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f16s", "f64"])
def test_persistent_batched_launch(prec, restore_tuning):
    dims = (6, 4, 4, 6)
    sizes = [1, 4, 3, 2]
    U, psi = fields(dims, 5, nrhs=sum(sizes))
    op = DiracOp(dims, U, -0.35, 1.0)
    nat = op.pack(to_dev(psi), prec)
    rb = op.field_bytes(prec, 1)
    for pb in (0, 8, 64, 4096):
        tune_set("persistent_blocks", pb)
        outs, batches, r0 = [], [], 0
        for n in sizes:
            o = op.empty(prec, n)
            outs.append(o)
            batches.append((o, nat[r0 * rb:(r0 + n) * rb], n))
            r0 += n
        op.apply_batched(batches, prec)
        got = torch.cat(outs)
        assert torch.equal(got, singles(op, nat, prec, sum(sizes)))
    g = op.unpack(got, prec, sum(sizes)).cpu().numpy()
    want = oracle.dirac_apply(dims, U, psi, -0.35, 1.0)
    for r in range(sum(sizes)):
        assert rel_l2(g[r], want[r]) < TOL[prec]


def test_many_register_blocks_split_launches(restore_tuning):
    """More register blocks than one launch holds (> 24) still give every RHS."""
    dims = (2, 2, 4, 4)
    U, psi = fields(dims, 8, nrhs=30)
    op = DiracOp(dims, U, 0.1, 1.0)
    tune_set("nr_f32", 1)
    nat = op.pack(to_dev(psi), "f32")
    out = op.empty("f32", 30)
    op.apply_native(out, nat, 30, "f32")
    assert torch.equal(out, singles(op, nat, "f32", 30))


@pytest.mark.parametrize("order", [0, 1, 2, 6])
@pytest.mark.parametrize("block", [64, 128, 192, 256])
@pytest.mark.parametrize("dims", [(5, 3, 7, 4), (3, 11, 4, 6)])
def test_tile_orders_and_blocks(order, block, dims, restore_tuning):
    # slices not divisible by 8 or by the block; Z extents below 8 and a ragged
    # second z-block of eight planes (order 6)
    U, psi = fields(dims, 2)
    op = DiracOp(dims, U, -0.3, 1.0)
    nat = op.pack(to_dev(psi), "f64")
    tune_set("order", 2)
    tune_set("block", 256)
    ref = op.empty("f64")
    op.apply_native(ref, nat)
    tune_set("order", order)
    tune_set("block", block)
    out = op.empty("f64")
    op.apply_native(out, nat)
    assert torch.equal(out, ref)
    want = oracle.dirac_apply(dims, U, psi, -0.3, 1.0)
    assert rel_l2(op.unpack(out, "f64").cpu().numpy(), want) < 1e-13


@pytest.mark.parametrize("tchunk", [1, 3, 8])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("compact", [False, True])
def test_column_sweep_order(tchunk, prec, dagger, compact, restore_tuning):
    """Tile order 3 (lanes walk columns along T with register-carried T
    neighbours): ragged T-chunks, anti-periodic T, several right-hand sides,
    packed and compact clover storage."""
    dims = (5, 3, 7, 4)
    U, psi = fields(dims, 31, nrhs=3)
    op = DiracOp(dims, U, -0.3, 1.0, antiperiodic_t=True, compress_clover=compact)
    tune_set("order", 3)
    tune_set("tchunk", tchunk)
    got = op.apply(to_dev(psi), prec, dagger=dagger).cpu().numpy()
    want = oracle.dirac_apply(dims, U, psi, -0.3, 1.0, antiperiodic_t=True, dagger=dagger)
    for r in range(3):
        assert rel_l2(got[r], want[r]) < TOL[prec], (r, rel_l2(got[r], want[r]))


@pytest.mark.parametrize("block", [64, 128, 192, 256])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_patch_order_equals_column_order(block, prec, restore_tuning):
    """Tile order 4 (column sweep over z-y-x patches of a work-group) runs the
    same per-site arithmetic as order 3, so the results agree bit for bit;
    extents ragged against the 16 x 4 x block/64 patch in every direction."""
    dims = (5, 5, 7, 18)
    U, psi = fields(dims, 43, nrhs=3)
    op = DiracOp(dims, U, -0.3, 1.0, antiperiodic_t=True)
    nat = op.pack(to_dev(psi), prec)
    tune_set("block", block)
    for tchunk in (1, 3):
        tune_set("tchunk", tchunk)
        for dag in (False, True):
            # zeroed: FP16S fields end in alignment padding the kernels never write
            tune_set("order", 3)
            ref = op.empty(prec, 3).zero_()
            op.apply_native(ref, nat, 3, prec, dag)
            tune_set("order", 4)
            out = op.empty(prec, 3).zero_()
            op.apply_native(out, nat, 3, prec, dag)
            assert torch.equal(out, ref), (tchunk, dag)
    got = op.unpack(out, prec, 3).cpu().numpy()
    want = oracle.dirac_apply(dims, U, psi, -0.3, 1.0, antiperiodic_t=True, dagger=True)
    for r in range(3):
        assert rel_l2(got[r], want[r]) < TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f16s", "f64"])
@pytest.mark.parametrize("compress", [True, False])
@pytest.mark.parametrize("compact", [False, True])
@pytest.mark.parametrize("dims", [(5, 3, 7, 4), (2, 10, 5, 6), (2, 5, 12, 16)])
@pytest.mark.parametrize("group", [1, 7])
@pytest.mark.parametrize("zw", [1, 2, 4])
def test_stationary_order_equals_site_kernel(prec, compress, compact, dims, group, zw, restore_tuning):
    """Tile order 5 (links and clover kept on chip for every right-hand side
    of the launch) runs the site kernel's arithmetic, so results agree bit for
    bit; 70 right-hand sides in uneven batches need two launches (ten in
    groups of 7, the tchunk knob), over plane tiles, z-pair tiles and z-pair
    tiles walked in (y, x) blocks (the nr knob); the planes leave a ragged
    last tile, the lattices ragged z-blocks and z-pairs (Z extents 3, 10 and
    5), and the third lattice three 64-site tiles per plane in (y, x) blocks
    of two.  FP64 and full links fall back to order 2."""
    sizes = [1, 24, 45]
    n = sum(sizes)
    U, psi = fields(dims, 47, nrhs=n)
    op = DiracOp(dims, U, -0.3, 1.0, antiperiodic_t=True, compress_links=compress, compress_clover=compact)
    nat = op.pack(to_dev(psi), prec)
    rb = op.field_bytes(prec, 1)
    tune_set("nr_" + prec, 1)
    tune_set("block", 128)
    for dag in (False, True):
        tune_set("order", 2)
        tune_set("nr_" + prec, 1)
        ref = op.empty(prec, n).zero_()
        op.apply_native(ref, nat, n, prec, dag)
        tune_set("order", 5)
        tune_set("tchunk", group)
        tune_set("nr_" + prec, zw)
        out = op.empty(prec, n).zero_()
        batches, r0 = [], 0
        for k in sizes:
            batches.append((out[r0 * rb:(r0 + k) * rb], nat[r0 * rb:(r0 + k) * rb], k))
            r0 += k
        op.apply_batched(batches, prec, dagger=dag)
        assert torch.equal(out, ref), dag
    got = op.unpack(out, prec, n).cpu().numpy()
    for r in (0, 1, 37, n - 1):
        want = oracle.dirac_apply(dims, U, psi[r], -0.3, 1.0, antiperiodic_t=True, dagger=True)
        assert rel_l2(got[r], want) < TOL[prec]


def test_batched_argument_errors(restore_tuning):
    dims = (2, 2, 2, 4)
    U, psi = fields(dims, 1, nrhs=2)
    op = DiracOp(dims, U, -0.3, 1.0)
    nat = op.pack(to_dev(psi), "f32")
    o = op.empty("f32", 2)
    rb = op.field_bytes("f32", 1)
    with pytest.raises(WdiracError):      # two outputs overlap
        op.apply_batched([(o, nat[:rb], 1), (o, nat[rb:], 1)], "f32")
    with pytest.raises(WdiracError):
        tune_set("block", 100)
    with pytest.raises(WdiracError):
        tune_set("nosuchkey", 1)
    with pytest.raises(WdiracError):
        tune_set("order", 7)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_column_sweep_two_row_links(prec, restore_tuning):
    dims = (6, 4, 3, 4)
    U, psi = fields(dims, 41, nrhs=3)
    op = DiracOp(dims, U, -0.25, 1.0, antiperiodic_t=True, compress_links=True)
    tune_set("order", 3)
    tune_set("tchunk", 4)
    got = op.apply(to_dev(psi), prec).cpu().numpy()
    want = oracle.dirac_apply(dims, U, psi, -0.25, 1.0, antiperiodic_t=True)
    for r in range(3):
        assert rel_l2(got[r], want[r]) < TOL[prec]
