#!/usr/bin/env python3
"""Benchmark of the Wilson-clover Dirac operator and FGMRES on one MI355X.

    python bench.py [--steps K] [--warmup W] [--dims T Z Y X] [--fgmres-rhs N]
                    [--no-fgmres] [--no-batched] [--no-cpu-baseline]

Workload: the 48^3 x 96 lattice (T = 96) with smoothed random SU(3) links
exp(0.3 i H), c_sw = 1, m0 = -0.35, Gaussian right-hand sides; every input is
seeded and synthetic and resident in HBM before any timed region.

A step is one FP64 application of D (Eq. (1.13) with the clover term) to one
right-hand side: `value` is applications per second, `roofline` relates the
stencil kernel's algorithmic bytes per launch to the HBM peak.  After the
timed steps (reported under "extra"):
  * single FP32 and FP16S applies;
  * one FP32 launch over uneven batches {1, 4, 12, 24} (autotuned: tile order,
    register blocks or the link-stationary kernel);
  * the even-odd reduced operator S alone (one right-hand side, and pairs);
  * 12 right-hand sides solved to 1e-10 by plain FP64 FGMRES(30) and by the
    mixed solver (FP64 outer FGMRES(8) whose preconditioner is an inner
    GMRES(10) on the FP16S operator, relative tolerance 0.1), in memory-sized
    waves: wall time, applications and the difference between the two
    solutions; then both again on the even-odd reduced system (half-lattice
    vectors, odd sites reconstructed; the same tolerance relative to the full
    system's |b|);
  * 32^4: FP64 apply rate and plain FP64 FGMRES(20) to 1e-10;
  * 24^3 x 48: forward + backward through the autograd Function and the force
    kernel alone.
The CPU oracle's apply is timed on a bounded slab of sites ("cpu_baseline").
Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FLOP_HOP = 1320                # flop/site, hopping term (the paper's convention)
FLOP_FULL = 1872               # flop/site, with clover (504) and combine (48)
# algorithmic bytes per site and right-hand side: in + out spinor + links + clover;
# the links are stored as two rows (4 directions x 6 complex per site; the
# third row is rebuilt in the kernel) and each clover chirality block as its
# spin-diagonal difference and off-diagonal 3x3 blocks (27 reals + 1 pad)
LINK_BYTES = {"f64": 384, "f32": 192, "f16s": 96}
CLOVER_BYTES = {"f64": 448, "f32": 224, "f16s": 112}
SPINOR_BYTES = {"f64": 192, "f32": 96, "f16s": 52}
BYTES_SITE = {p: 2 * SPINOR_BYTES[p] + LINK_BYTES[p] + CLOVER_BYTES[p] for p in LINK_BYTES}
KERNEL_SOURCES = ["paper_2407_00041_amd/csrc/dslash.hip", "paper_2407_00041_amd/csrc/dslash.h",
                  "paper_2407_00041_amd/csrc/stencil.h",
                  "paper_2407_00041_amd/csrc/tune.hip",
                  "paper_2407_00041_amd/csrc/spinor_io.h", "paper_2407_00041_amd/csrc/common.h"]
TRAFFIC_PROFILE = "profiles/dslash_f64_48x96_hbm_traffic.md"
# mixed solver: FP64 outer FGMRES, inner GMRES on the reduced-precision operator
MIXED = {"mode": "mixed_f16s", "restart": 8, "inner_restart": 10, "inner_tol": 0.1}
TUNE_FIXED = False


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dims", type=int, nargs=4, default=[96, 48, 48, 48])
    ap.add_argument("--m0", type=float, default=-0.35)
    ap.add_argument("--csw", type=float, default=1.0)
    ap.add_argument("--fgmres-rhs", type=int, default=12)
    ap.add_argument("--no-fgmres", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip every measurement after the main one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fixed-launch", type=int, nargs=4, metavar=("ORDER", "BLOCK", "TCHUNK", "NR"),
                    help="use this launch configuration for every stencil launch instead of autotuning "
                         "(reproducible profiling runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB elementwise copy (counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile():
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not b or m.group(1) != kernel_hash():
        return None
    return float(b.group(1))


def time_launches(torch, fn, steps, warmup, stream):
    for _ in range(warmup):
        fn()
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps        # ms per launch


# Algorithmic bytes per full-lattice site of one application of the even-odd
# reduced operator S (two launches over V/2 sites: A_oo^-1 H_oe, then
# A_ee - H_eo), with two-row links, compact A on the even sites and packed
# A^-1 on the odd ones; per half-site: FP64 192 in + 8 x 96 links + 576 A^-1 +
# 192 out, then 192 self + 192 in + 768 links + 448 A + 192 out (3520, i.e.
# 1760 per site); in pairs the links and A / A^-1 are shared by two right-hand
# sides (1120 per site per RHS).  FP32 / FP16S likewise with 96 / 52 B spinors,
# 48 / 24 B links, 288 / 144 B A^-1 and 224 / 112 B compact A.
SCHUR_BYTES_SITE = {"f64": (1760, 1120), "f32": (880, 560), "f16s": (450, 290)}


def schur_apply_run(torch, op, psid, stream, steps=20):
    """The reduced operator S: ms per application for one right-hand side and
    per right-hand side of a pair, at every precision."""
    res = {}
    V = op.V
    for p in ("f64", "f32", "f16s"):
        nat = op.pack(torch.cat([psid, psid]), p)
        e, o = op.split(nat, p, 2)
        del nat, o
        out, tmp = op.empty_parity(p, 2), op.empty_parity(p, 2)
        rb = op.parity_field_bytes(p, 1)
        one = time_launches(torch, lambda: op.apply_schur_native(out[:rb], e[:rb], tmp[:rb], 1, p), steps, 3,
                            stream)
        two = time_launches(torch, lambda: op.apply_schur_native(out, e, tmp, 2, p), steps, 3, stream) / 2
        b1, b2 = SCHUR_BYTES_SITE[p]
        res[p] = {"ms_single": one, "ms_per_rhs_pair": two, "alg_bytes_per_site": [b1, b2],
                  "alg_GBps_single": b1 * V / (one * 1e-3) / 1e9, "alg_GBps_pair": b2 * V / (two * 1e-3) / 1e9}
        del e, out, tmp
    torch.cuda.empty_cache()
    return res


def batched_run(torch, op, dims, stream, steps):
    from paper_2407_00041_amd import synth
    sizes = [1, 4, 12, 24]
    n = sum(sizes)
    psi = synth.gaussian_spinor(dims, 2100, nrhs=n, device="cuda")
    nat = op.pack(psi, "f32")
    del psi
    rb = op.field_bytes("f32", 1)
    outs, batches, r0 = [], [], 0
    for s in sizes:
        o = op.empty("f32", s)
        outs.append(o)
        batches.append((o, nat[r0 * rb:(r0 + s) * rb], s))
        r0 += s
    tuned = {"fixed": True} if TUNE_FIXED else op.autotune("f32", n)
    ms = time_launches(torch, lambda: op.apply_batched(batches, "f32", stream=stream), steps, 3, stream)
    res = {"batches": sizes, "prec": "f32", "ms_per_launch": ms, "rhs_applies_per_s": n * 1000.0 / ms,
           "alg_GBps": (LINK_BYTES["f32"] + CLOVER_BYTES["f32"] + 192 * n) * op.V / (ms * 1e-3) / 1e9,
           "launch": tuned}
    del outs, batches, nat
    torch.cuda.empty_cache()
    return res


def fgmres_run(torch, op, dims, nrhs_total):
    """Plain FP64 FGMRES(30) vs the mixed FP16S-preconditioned FGMRES on the
    same right-hand sides, in waves sized to the free HBM, on D x = b and on
    the even-odd reduced system."""
    from paper_2407_00041_amd import synth
    p64 = dict(restart=30, tol=1e-10, maxit=5000, mode="f64")
    pmx = dict(restart=MIXED["restart"], tol=1e-10, maxit=500, mode=MIXED["mode"],
               inner_restart=MIXED["inner_restart"], inner_tol=MIXED["inner_tol"], inner_maxit=MIXED["inner_restart"])
    fb = op.field_bytes("f64", 1)
    free, _ = torch.cuda.mem_get_info()
    per = max(op.workspace_bytes(1, 30, "f64"),
              op.workspace_bytes(1, pmx["restart"], pmx["mode"], pmx["inner_restart"])) + 5 * fb
    wave = int(max(1, min(nrhs_total, (free - (8 << 30)) // per)))
    log(f"[bench] fgmres: {nrhs_total} RHS in waves of {wave} "
        f"(free {free / 2**30:.0f} GiB, {per / 2**30:.1f} GiB per RHS)")
    # one workspace for every wave and both solvers (allocation is not timed)
    wbytes = max(op.workspace_bytes(wave, 30, "f64"),
                 op.workspace_bytes(wave, pmx["restart"], pmx["mode"], pmx["inner_restart"]))
    work = torch.empty(wbytes, dtype=torch.uint8, device="cuda")
    inner = "f16s" if pmx["mode"].endswith("f16s") else "f32"
    for n in sorted({1, wave, nrhs_total % wave or wave}):     # the solvers' batched applies
        if not TUNE_FIXED:
            op.autotune("f64", n)
            op.autotune(inner, n)
    t64 = tmx = t64r = tmxr = 0.0
    ph64 = {"apply": 0.0, "precond": 0.0, "ortho": 0.0}
    phmx = {"apply": 0.0, "precond": 0.0, "ortho": 0.0}
    a64, amx, ainner, errs, res64, resmx = [], [], [], [], [], []
    a64r, amxr, ainr, errsr, res64r, resmxr = [], [], [], [], [], []
    for w0 in range(0, nrhs_total, wave):
        nw = min(wave, nrhs_total - w0)
        b = op.pack(synth.gaussian_spinor(dims, 3000 + w0, nrhs=nw, device="cuda"), "f64")
        torch.cuda.synchronize()
        t = time.perf_counter()
        x64, st64, _ = op.solve(b, nrhs=nw, work=work, **p64)
        torch.cuda.synchronize()
        t64 += time.perf_counter() - t
        t = time.perf_counter()
        xmx, stmx, _ = op.solve(b, nrhs=nw, work=work, **pmx)
        torch.cuda.synchronize()
        tmx += time.perf_counter() - t
        xmx_keep = xmx
        for k in ph64:  # GPU time per phase of this wave (shared by its right-hand sides)
            ph64[k] += st64[0]["seconds_" + k]
            phmx[k] += stmx[0]["seconds_" + k]
        del xmx
        t = time.perf_counter()
        x64r, st64r, _ = op.solve(b, nrhs=nw, work=work, schur=True, **p64)
        torch.cuda.synchronize()
        t64r += time.perf_counter() - t
        t = time.perf_counter()
        xmxr, stmxr, _ = op.solve(b, nrhs=nw, work=work, schur=True, **pmx)
        torch.cuda.synchronize()
        tmxr += time.perf_counter() - t
        for r in range(nw):
            u = x64[r * fb:(r + 1) * fb].view(torch.float64)
            nu = torch.linalg.vector_norm(u)
            for xs, e in ((xmx_keep, errs), (x64r, errsr), (xmxr, errsr)):
                v = xs[r * fb:(r + 1) * fb].view(torch.float64)
                e.append(float(torch.linalg.vector_norm(u - v) / nu))
            a64.append(st64[r]["applies"])
            amx.append(stmx[r]["applies"])
            ainner.append(stmx[r]["inner_applies"])
            res64.append(st64[r]["true_residual"])
            resmx.append(stmx[r]["true_residual"])
            a64r.append(st64r[r]["applies"])
            amxr.append(stmxr[r]["applies"])
            ainr.append(stmxr[r]["inner_applies"])
            res64r.append(st64r[r]["true_residual"])
            resmxr.append(stmxr[r]["true_residual"])
        log(f"[bench] fgmres after RHS {w0 + nw}: fp64 {t64:.2f}s mixed {tmx:.2f}s; even-odd reduced: "
            f"fp64 {t64r:.2f}s mixed {tmxr:.2f}s")
        del b, x64, xmx_keep, x64r, xmxr
        torch.cuda.empty_cache()
    return {"nrhs": nrhs_total, "wave": wave, "tol": 1e-10,
            "fp64": {"solver": "FGMRES(30), FP64", "seconds": t64, "phase_seconds": ph64, "applies": a64,
                     "true_residual_max": max(res64), "converged": all(r < 1e-10 for r in res64)},
            "mixed": {"solver": f"FP64 FGMRES({pmx['restart']}), preconditioner inner GMRES({pmx['inner_restart']}) "
                                f"on the {pmx['mode'][6:].upper()} operator (relative tol {pmx['inner_tol']})",
                      "seconds": tmx, "phase_seconds": phmx, "fp64_applies": amx, "fp16s_applies": ainner,
                      "true_residual_max": max(resmx), "converged": all(r < 1e-10 for r in resmx)},
            "speedup_mixed_vs_fp64": t64 / tmx if tmx > 0 else None,
            "error_vs_fp64_max": max(errs),
            "even_odd": {
                "fp64": {"solver": "FGMRES(30), FP64, on S = A_ee - H_eo A_oo^-1 H_oe", "seconds": t64r,
                         "applies_of_S": a64r, "true_residual_max": max(res64r),
                         "converged": all(r < 1e-10 for r in res64r)},
                "mixed": {"solver": "the mixed solver above on S (FP16S S in the inner GMRES)", "seconds": tmxr,
                          "fp64_applies_of_S": amxr, "fp16s_applies_of_S": ainr,
                          "true_residual_max": max(resmxr), "converged": all(r < 1e-10 for r in resmxr)},
                "speedup_mixed_vs_fp64": t64r / tmxr if tmxr > 0 else None,
                "speedup_vs_full_system": {"fp64": t64 / t64r if t64r > 0 else None,
                                           "mixed": tmx / tmxr if tmxr > 0 else None},
                "speedup_mixed_even_odd_vs_plain_fp64": t64 / tmxr if tmxr > 0 else None,
                "error_vs_plain_fp64_max": max(errsr)}}


def config32_run(torch, stream):
    """32^4, c_sw = 1, m0 = -0.3, one right-hand side: the FP64 apply rate and
    plain FP64 FGMRES(20) to 1e-10 (the 32^4 solver workload)."""
    import paper_2407_00041_amd as wd
    from paper_2407_00041_amd import synth
    dims = (32, 32, 32, 32)
    V = 32 ** 4
    U = synth.smooth_links(dims, 1002, device="cuda").cpu().numpy()
    op = wd.DiracOp(dims, U, -0.3, 1.0, precisions=("f64",), compress_links=True, compress_clover=True)
    tuned = {"fixed": True} if TUNE_FIXED else op.autotune("f64", 1)
    x = op.pack(synth.gaussian_spinor(dims, 2000, nrhs=1, device="cuda"), "f64")
    y = op.empty("f64", 1)
    ms = time_launches(torch, lambda: op.apply_native(y, x, 1, "f64", stream=stream), 100, 10, stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, st, rc = op.solve(x, restart=20, tol=1e-10, maxit=3000)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t
    res = {"dims": list(dims), "apply_ms": ms, "apps_per_s": 1000.0 / ms,
           "alg_GBps": BYTES_SITE["f64"] * V / (ms * 1e-3) / 1e9, "launch": tuned,
           "fgmres20_fp64": {"seconds": ts, "applies": st[0]["applies"], "true_residual": st[0]["true_residual"],
                             "converged": st[0]["converged"], "phase_seconds": {
                                 k: st[0]["seconds_" + k] for k in ("apply", "precond", "ortho")}}}
    del op, x, y
    torch.cuda.empty_cache()
    return res


def differentiation_run(torch):
    """24^3 x 48, c_sw = 1, FP64: L = Re<eta, D(U) x>; forward plus backward
    through the autograd Function (dL/dx by the adjoint apply, dL/dU by the
    force kernel), and the force kernel alone."""
    import paper_2407_00041_amd as wd
    from paper_2407_00041_amd import synth
    from paper_2407_00041_amd.autograd import dirac_apply
    dims = (48, 24, 24, 24)
    m0, csw = -0.3, 1.0
    Ut = synth.smooth_links(dims, 1005, device="cuda")
    op = wd.DiracOp(dims, Ut.cpu().numpy(), m0, csw, precisions=("f64",))
    x = synth.gaussian_spinor(dims, 3001, nrhs=1, device="cuda").requires_grad_(True)
    eta = synth.gaussian_spinor(dims, 3002, nrhs=1, device="cuda")
    links = Ut.clone().requires_grad_(True)

    def step():
        y = dirac_apply(x, links, dims, op=op, m0=m0, csw=csw)
        loss = (eta.conj() * y).sum().real
        return torch.autograd.grad(loss, (x, links))

    cur = torch.cuda.current_stream()
    ms_fb = time_launches(torch, step, 10, 2, cur)
    en = op.pack(eta.detach(), "f64")
    xn = op.pack(x.detach(), "f64")
    ms_force = time_launches(torch, lambda: op.force(en, xn, 1), 20, 3, cur)
    res = {"dims": list(dims), "forward_backward_ms": ms_fb, "force_kernel_ms": ms_force,
           "note": "forward + backward include the canonical <-> native conversions of the autograd binding"}
    del op, x, eta, links, en, xn
    torch.cuda.empty_cache()
    return res


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


def main():
    global TUNE_FIXED
    a = parse()
    TUNE_FIXED = bool(a.fixed_launch)
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the library has no multi-GPU "
                                   "halo exchange"}))
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
    op = wd.DiracOp(dims, U, a.m0, a.csw, precisions=("f64", "f32", "f16s"), compress_links=True,
                    compress_clover=True, even_odd=True)
    stream = torch.cuda.current_stream()
    inp = {p: op.pack(psid, p) for p in ("f64", "f32", "f16s")}
    out = {p: op.empty(p, 1) for p in ("f64", "f32", "f16s")}
    torch.cuda.synchronize()

    if a.fixed_launch:
        o, blk, tch, nr = a.fixed_launch
        for k, v in (("order", o), ("block", blk), ("tchunk", tch), ("nr_f64", nr), ("nr_f32", nr), ("nr_f16s", nr)):
            wd.tune_set(k, v)
        tuned = {p: {"order": o, "block": blk, "tchunk": tch, "nr": nr, "fixed": True} for p in ("f64", "f32", "f16s")}
    else:
        tuned = {p: op.autotune(p, 1) for p in ("f64", "f32", "f16s")}
    log(f"[bench] launches: {tuned}")
    log(f"[bench] timing FP64 apply: {a.warmup} warmup + {a.steps} steps")
    ms = time_launches(torch, lambda: op.apply_native(out["f64"], inp["f64"], 1, "f64", stream=stream),
                       a.steps, a.warmup, stream)
    apps = 1000.0 / ms
    gbs = BYTES_SITE["f64"] * V / (ms * 1e-3) / 1e9
    log(f"[bench] FP64: {ms:.4f} ms/apply, {apps:.1f} apps/s, {gbs:.0f} GB/s")

    extra = {"f64": {"ms": ms, "apps_per_s": apps, "alg_GBps": gbs, "launch": tuned["f64"],
                     "GFLOPs_1320": FLOP_HOP * V / (ms * 1e-3) / 1e9,
                     "GFLOPs_1872": FLOP_FULL * V / (ms * 1e-3) / 1e9}}
    if not a.no_extra:
        # achievable streaming rate on this device: an elementwise kernel reading
        # 4 GiB and writing 4 GiB (a same-dtype copy_ would take the slower blit path)
        n = 1 << 30
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        cms = time_launches(torch, lambda: torch.mul(src, 2.0, out=dst), 10, 3, torch.cuda.current_stream())
        copy_gbs = 2 * n * 4 / (cms * 1e-3) / 1e9
        del src, dst
        torch.cuda.empty_cache()
        extra["f64"]["copy_GBps"] = copy_gbs
        extra["f64"]["alg_frac_of_copy"] = gbs / copy_gbs
        log(f"[bench] device copy {copy_gbs:.0f} GB/s; FP64 apply at {gbs / copy_gbs:.3f} of it")
        for p in ("f32", "f16s"):
            m = time_launches(torch, lambda: op.apply_native(out[p], inp[p], 1, p, stream=stream),
                              max(10, a.steps // 2), a.warmup, stream)
            extra[p] = {"ms": m, "apps_per_s": 1000.0 / m, "alg_GBps": BYTES_SITE[p] * V / (m * 1e-3) / 1e9,
                        "launch": tuned[p],
                        "GFLOPs_1320": FLOP_HOP * V / (m * 1e-3) / 1e9}
            log(f"[bench] {p}: {m:.4f} ms/apply")
    if a.copy_probe:
        n = 1 << 28
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] copy probe done (1 GiB read + 1 GiB write, x5)")
    del inp, out
    torch.cuda.empty_cache()
    if not a.no_extra and not a.no_batched:
        log("[bench] batched FP32 launch {1,4,12,24}")
        extra["batched"] = batched_run(torch, op, dims, stream, 10)
        extra["batched"]["per_rhs_rate_vs_fp64_single"] = extra["batched"]["rhs_applies_per_s"] / apps
        log(f"[bench] batched: {extra['batched']['rhs_applies_per_s']:.0f} RHS-applies/s")
    if not a.no_extra:
        extra["even_odd_apply"] = schur_apply_run(torch, op, psid, stream)
        log("[bench] even-odd S: " + ", ".join(f"{p} {v['ms_single']:.3f} ms ({v['ms_per_rhs_pair']:.3f} per RHS of a "
                                                f"pair)" for p, v in extra["even_odd_apply"].items()))
    if not a.no_extra and not a.no_fgmres and a.fgmres_rhs > 0:
        extra["fgmres"] = fgmres_run(torch, op, dims, a.fgmres_rhs)
    if not a.no_extra:
        log("[bench] 32^4: FP64 apply and FGMRES(20)")
        extra["config_32"] = config32_run(torch, stream)
        log(f"[bench] 32^4: {extra['config_32']['apply_ms']:.4f} ms/apply, FGMRES(20) "
            f"{extra['config_32']['fgmres20_fp64']['seconds']:.2f} s")
        log("[bench] 24^3x48: differentiation")
        extra["differentiation"] = differentiation_run(torch)
        log(f"[bench] 24^3x48: forward+backward {extra['differentiation']['forward_backward_ms']:.2f} ms")

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
        "data": "synthetic (seeded exp(0.3iH) SU(3) links, Gaussian spinors)",
        "config": {"workload": f"Wilson-clover D apply, {dims[1]}^3x{dims[0]} (T,Z,Y,X = {list(dims)}), "
                               f"FP64, 1 RHS, csw={a.csw}, m0={a.m0}, periodic",
                   "lattice": list(dims), "sites": V, "nrhs": 1, "parallelism": "single GPU",
                   "link_storage": "two rows per SU(3) link (third rebuilt in the kernel)",
                   "clover_storage": "per chirality block (A_00 - A_11)/2 and A_01 (27 of 36 reals)"},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": traffic_from_profile(),
                     "kernel": ("wd::dslash_column_kernel<0, false, 1>" if tuned["f64"]["order"] == 3
                                else "wd::dslash_kernel<0, false, 1>"),
                     "alg_bytes_per_site": BYTES_SITE["f64"], "alg_bytes_per_launch": BYTES_SITE["f64"] * V,
                     "kernel_source_sha256_16": kernel_hash()},
        "extra": extra,
    }
    if not a.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        psi = psid.reshape(V, 12).cpu().numpy()
        res["cpu_baseline"] = cpu_baseline_run(dims, U, psi, a.m0, a.csw)
        log(f"[bench] cpu baseline {res['cpu_baseline']['value']:.4f} apps/s")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
