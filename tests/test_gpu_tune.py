"""The autotuner: its choices are valid configurations, launches that use them
still match the oracle, the cache file records them, and the full-size
lattice in the benchmark's configuration (two-row links, autotuned launch)
agrees with the oracle at sampled sites."""
import json

import numpy as np
import pytest
import torch

import oracle
from paper_2407_00041_amd import DiracOp, _lib, synth, tune_get, tune_set
from util import TOL, fields, need_gpu, rel_l2, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture
def clean_table():
    need_gpu()
    explicit = tune_get("explicit")
    tune_set("explicit", 0)
    yield
    _lib.load().dirac_tune_clear()
    tune_set("explicit", explicit)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_autotuned_launch_matches_oracle(prec, nrhs, clean_table, tmp_path, monkeypatch):
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("WDIRAC_TUNE_CACHE", str(cache))
    dims = (6, 4, 6, 4)
    U, psi = fields(dims, 12, nrhs=nrhs)
    op = DiracOp(dims, U, -0.3, 1.0, antiperiodic_t=True, compress_links=True)
    cfg = op.autotune(prec, nrhs)
    assert cfg["order"] in (0, 2, 3, 4, 5, 6) and cfg["block"] in (128, 256) and cfg["nr"] in (1, 2, 4)
    assert cfg["persistent"] in (0, 1) and (nrhs > 1 or cfg["persistent"] == 0)
    assert cfg["us"] > 0
    got = op.apply(to_dev(psi), prec).cpu().numpy()
    want = oracle.dirac_apply(dims, U, psi, -0.3, 1.0, antiperiodic_t=True)
    for r in range(nrhs):
        assert rel_l2(got[r], want[r]) < TOL[prec]
    lines = [json.loads(x) for x in cache.read_text().splitlines()]
    assert lines[-1]["order"] == cfg["order"] and lines[-1]["nr"] == cfg["nr"]
    assert lines[-1]["persistent"] == cfg["persistent"]
    assert lines[-1]["key"].startswith("gfx950|6x4x6x4|")


def test_full_size_bench_configuration(clean_table):
    """48^3 x 96, c_sw = 1, m0 = -0.35, two-row links, compact clover, autotuned
    FP64/FP32/FP16S launches (as bench.py times them): 1500 sampled sites vs the oracle."""
    dims = (96, 48, 48, 48)
    V = synth.volume(dims)
    m0, csw = -0.35, 1.0
    Ud = synth.smooth_links(dims, 1003, device="cuda")
    psid = synth.gaussian_spinor(dims, 2000, nrhs=1, device="cuda")
    U = Ud.cpu().numpy()
    del Ud
    psi = psid.cpu().numpy()[0]
    op = DiracOp(dims, U, m0, csw, precisions=("f64", "f32", "f16s"), compress_links=True, compress_clover=True)
    sites = synth.random_sites(dims, 1500, 9)
    want = oracle.dirac_apply_sites(dims, U, psi, sites, m0, csw)
    st = torch.from_numpy(sites).cuda()
    for prec in ("f64", "f32", "f16s"):
        op.autotune(prec, 1)
        got = op.apply(psid, prec).reshape(V, 12)[st].cpu().numpy()
        assert rel_l2(got, want) < TOL[prec], prec
    del op
    torch.cuda.empty_cache()


def test_full_size_batched_launch(clean_table):
    """48^3 x 96, FP32, two-row links, compact clover, uneven batches {1, 4} in one launch, with
    the autotuned configuration and with the link-stationary kernel (the one
    the benchmark's 41-RHS batch selects): 1000 sampled sites of every
    right-hand side vs the oracle."""
    dims = (96, 48, 48, 48)
    V = synth.volume(dims)
    m0, csw = -0.35, 1.0
    Ud = synth.smooth_links(dims, 1005, device="cuda")
    U = Ud.cpu().numpy()
    del Ud
    op = DiracOp(dims, U, m0, csw, precisions=("f64", "f32"), compress_links=True, compress_clover=True)
    psid = synth.gaussian_spinor(dims, 2300, nrhs=5, device="cuda")
    nat = op.pack(psid, "f32")
    rb = op.field_bytes("f32", 1)
    sites = synth.random_sites(dims, 1000, 13)
    st = torch.from_numpy(sites).cuda()
    want = [oracle.dirac_apply_sites(dims, U, psid[r].cpu().numpy(), sites, m0, csw) for r in range(5)]
    del psid
    op.autotune("f32", 5)
    saved_order = tune_get("order")
    for explicit_order in (None, 5):
        if explicit_order is not None:
            tune_set("order", explicit_order)
        out = op.empty("f32", 5)
        op.apply_batched([(out[:rb], nat[:rb], 1), (out[rb:], nat[rb:], 4)], "f32")
        got = op.unpack(out, "f32", 5)
        for r in range(5):
            assert rel_l2(got[r][st].cpu().numpy(), want[r]) < TOL["f32"], (explicit_order, r)
        del out, got
    tune_set("order", saved_order)
    del op, nat
    torch.cuda.empty_cache()
