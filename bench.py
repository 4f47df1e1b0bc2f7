#!/usr/bin/env python3
"""Benchmark of the Wilson-clover Dirac operator on one MI355X.

    python bench.py [--steps K] [--warmup W] [--dims T Z Y X] [--no-cpu-baseline]

A step is one FP64 application of D (Eq. (1.13) with the clover term) to one
Gaussian right-hand side on the 48^3 x 96 lattice (T = 96) with smoothed
random SU(3) links exp(0.3 i H), c_sw = 1, m0 = -0.35; inputs are resident in
HBM before the timed region.  Prints ONE JSON line.  The FP32 and FP16S
applies on the same lattice are timed after the main measurement and reported
in "extra".  The CPU oracle is timed on a bounded contiguous slab of sites
("cpu_baseline").
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FLOP_HOP = 1320                # flop/site, hopping term (the paper's convention)
FLOP_FULL = 1872               # flop/site, with clover (504) and combine (48)
# algorithmic bytes per site and right-hand side: in + out spinor + links + clover
BYTES_SITE = {"f64": 192 + 192 + 576 + 576, "f32": 96 + 96 + 288 + 288, "f16s": 52 + 52 + 144 + 144}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dims", type=int, nargs=4, default=[96, 48, 48, 48])
    ap.add_argument("--m0", type=float, default=-0.35)
    ap.add_argument("--csw", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_applies(torch, op, out, inp, prec, steps, warmup, stream):
    for _ in range(warmup):
        op.apply_native(out, inp, 1, prec, stream=stream)
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        op.apply_native(out, inp, 1, prec, stream=stream)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps        # ms per apply


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   "multi-GPU halo exchange is not part of this build"}))
        sys.exit(2)
    import torch

    import paper_2407_00041_amd as wd
    from paper_2407_00041_amd import synth

    dims = tuple(a.dims)
    V = int(np.prod(dims))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"[bench] generating inputs {dims} V={V}")
    t0 = time.time()
    Ud = synth.smooth_links(dims, 1003, device=dev)
    psid = synth.gaussian_spinor(dims, 2000, nrhs=1, device=dev)
    U = Ud.cpu().numpy()
    del Ud
    log(f"[bench] inputs ready in {time.time() - t0:.1f}s; creating operator")
    op = wd.DiracOp(dims, U, a.m0, a.csw, precisions=("f64", "f32", "f16s"))
    stream = torch.cuda.current_stream()
    inp = {p: op.pack(psid, p) for p in ("f64", "f32", "f16s")}
    out = {p: op.empty(p, 1) for p in ("f64", "f32", "f16s")}
    torch.cuda.synchronize()

    log(f"[bench] timing FP64 apply: {a.warmup} warmup + {a.steps} steps")
    ms = time_applies(torch, op, out["f64"], inp["f64"], "f64", a.steps, a.warmup, stream)
    apps = 1000.0 / ms
    gbs = BYTES_SITE["f64"] * V / (ms * 1e-3) / 1e9
    log(f"[bench] FP64: {ms:.4f} ms/apply, {apps:.1f} apps/s, {gbs:.0f} GB/s")

    extra = {"f64": {"ms": ms, "apps_per_s": apps, "alg_GBps": gbs,
                     "GFLOPs_1320": FLOP_HOP * V / (ms * 1e-3) / 1e9,
                     "GFLOPs_1872": FLOP_FULL * V / (ms * 1e-3) / 1e9}}
    if not a.no_extra:
        for p in ("f32", "f16s"):
            m = time_applies(torch, op, out[p], inp[p], p, max(10, a.steps // 2), a.warmup, stream)
            extra[p] = {"ms": m, "apps_per_s": 1000.0 / m,
                        "alg_GBps": BYTES_SITE[p] * V / (m * 1e-3) / 1e9,
                        "GFLOPs_1320": FLOP_HOP * V / (m * 1e-3) / 1e9}
            log(f"[bench] {p}: {m:.4f} ms/apply")
    if a.copy_probe:
        n = 1 << 30
        src = torch.empty(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy probe done (1 GiB x 5)")

    res = {
        "metric": "Dirac apps/s & HBM GB/s; mixed vs FP64 FGMRES time to 1e-10 at 48^3x96",
        "value": apps,
        "unit": "Dirac apps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded exp(0.3iH) SU(3) links, Gaussian spinor)",
        "config": {"workload": f"Wilson-clover D apply, {dims[1]}^3x{dims[0]} (T,Z,Y,X = {dims}), "
                               f"FP64, 1 RHS, csw={a.csw}, m0={a.m0}, periodic",
                   "lattice": list(dims), "sites": V, "nrhs": 1, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "wd::dslash_kernel<0,false>",
                     "alg_bytes_per_site": BYTES_SITE["f64"]},
        "extra": extra,
    }
    if not a.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        psi = psid.reshape(V, 12).cpu().numpy()
        res["cpu_baseline"] = cpu_baseline_run(dims, U, psi, a.m0, a.csw)
        log(f"[bench] cpu baseline {res['cpu_baseline']['value']:.4f} apps/s")
    print(json.dumps(res), flush=True)


def cpu_baseline_run(dims, U, psi, m0, csw, target_s=3.0):
    """Oracle apply on a contiguous slab of T-slices (clover rows built first,
    outside the timed call); the slab is sized from a one-slice calibration so
    the timed apply takes about target_s seconds."""
    import oracle
    V = int(np.prod(dims))
    slab = int(np.prod(dims[1:]))
    s1 = np.arange(slab, dtype=np.int64)
    C1 = oracle.clover_term_sites(dims, U, s1)
    t = time.perf_counter()
    oracle.dirac_apply_sites(dims, U, psi, s1, m0, csw, clover_rows=C1)
    dt1 = time.perf_counter() - t
    nsl = int(max(1, min(dims[0], round(target_s / max(dt1, 1e-6)))))
    sites = np.arange(nsl * slab, dtype=np.int64)
    Cs = oracle.clover_term_sites(dims, U, sites)
    t = time.perf_counter()
    oracle.dirac_apply_sites(dims, U, psi, sites, m0, csw, clover_rows=Cs)
    dt = time.perf_counter() - t
    apps = len(sites) / (dt * V)
    return {"value": apps, "unit": "Dirac apps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"FP64 oracle apply on {nsl} of {dims[0]} T-slices ({len(sites)} of {V} sites, "
                      f"clover rows precomputed), {dt:.2f} s, scaled to the whole lattice",
            "cpu": _cpu_model()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
