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
    system's |b|); FGMRES with the SAP preconditioner and with the two-level
    multigrid (its setup timed on its own);
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
# (outer restart, inner restart, inner tolerance) of the mixed solver tried on one right-hand side, on D and on S
MIXED_SWEEP = [(8, 10, 0.1), (8, 10, 0.05), (8, 16, 0.05), (16, 10, 0.05), (8, 6, 0.2)]
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
    ap.add_argument("--solve-profile", action="store_true",
                    help="only the mixed even-odd solve of --fgmres-rhs right-hand sides, bracketed by one FP32 "
                         "apply on each side (markers for a kernel trace)")
    ap.add_argument("--solve-wave", type=int, default=0,
                    help="right-hand sides per wave of --solve-profile (0: as many as the free HBM allows)")
    ap.add_argument("--summarize-solve", nargs=3, metavar=("TRACE_DIR", "SOLVE_LOG", "OUT_MD"),
                    help="kernel-time breakdown of a --solve-profile run under rocprofv3 --kernel-trace")
    ap.add_argument("--fixed-launch", type=int, nargs=4, metavar=("ORDER", "BLOCK", "TCHUNK", "NR"),
                    help="use this launch configuration for every stencil launch instead of autotuning "
                         "(reproducible profiling runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB elementwise copy (counter calibration)")
    ap.add_argument("--kernel-suite", metavar="MANIFEST",
                    help="run every product kernel at the benchmark sizes (for rocprofv3), write the manifest of "
                         "their algorithmic bytes and exit")
    ap.add_argument("--summarize", nargs=5, metavar=("MANIFEST", "TRACE_DIR", "FETCH_DIR", "WRITE_DIR", "OUT_MD"),
                    help="join a kernel-suite manifest with rocprofv3 output into a summary and exit (no GPU)")
    ap.add_argument("--summary-command", default="", help="command text recorded in the summary")
    ap.add_argument("--summarize-headline", nargs=3, metavar=("TRACE_DIR", "BENCH_LOG", "OUT_MD"),
                    help="summarize a rocprofv3 kernel trace of the default FP64 bench run (the last steps + warmup "
                         "dispatches of its stencil kernel) against the bench's own timing, and exit (no GPU)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the oracle FGMRES solves to convergence instead of a bounded sample")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def all_sources_hash() -> str:
    """Hash of every library source (kernels and host code), recorded in the kernel-suite summary."""
    import glob
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2407_00041_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNELS_PROFILE = "profiles/kernels_48x96_traffic.md"


def kernel_profile_rows():
    """{pattern: counted bytes per launch} from the committed kernel-suite summary, when it was taken on the
    current sources (else {})."""
    path = os.path.join(ROOT, KERNELS_PROFILE)
    if not os.path.exists(path):
        return {}
    text = open(path).read()
    m = re.search(r"sources_sha256_16:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != all_sources_hash():
        return {}
    rows = {}
    for line in text.splitlines():
        c = [x.strip() for x in line.split("|")]
        if len(c) > 11 and c[1].startswith("`"):
            try:
                rows[c[1].strip("`")] = {"counted_GB_per_launch": float(c[8]) + float(c[9]),
                                         "counted_GBps": float(c[10]), "avg_us": float(c[4])}
            except ValueError:
                pass
    return rows


def traffic_from_profile(pattern="dslash_column_kernel<0, false, 1>"):
    """HBM bytes per launch of the FP64 stencil from the committed counter summaries (the kernel-suite summary,
    else the stencil's own), if they were taken on the current stencil sources (else None)."""
    suite = os.path.join(ROOT, KERNELS_PROFILE)
    if os.path.exists(suite):
        text = open(suite).read()
        m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
        if m and m.group(1) == kernel_hash():
            for line in text.splitlines():
                c = [x.strip() for x in line.split("|")]
                if len(c) > 11 and c[1].strip("`") == pattern:
                    try:
                        return (float(c[8]) + float(c[9])) * 1e9
                    except ValueError:
                        pass
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
           "note": "ms_per_launch is one dirac_apply_batched call (the link-stationary kernel may split it into "
                   "launches of launch.tchunk right-hand sides)",
           "alg_GBps": (LINK_BYTES["f32"] + CLOVER_BYTES["f32"] + 192 * n) * op.V / (ms * 1e-3) / 1e9,
           "launch": tuned}
    del outs, batches, nat
    torch.cuda.empty_cache()
    return res


SAP_DEFAULT = {"block": (4, 4, 4, 4), "cycles": 1, "mr_iters": 4, "prec": "f32"}
# two-level multigrid preconditioner: aggregates of 4^4 sites (a 24 x 12^3 coarse lattice at 48^3 x 96), 8 test
# vectors, SAP smoother as above, coarse GMRES(30) to 5e-2, the interpolation stored in FP32 (FP64 accumulation)
AMG_DEFAULT = {"agg": (4, 4, 4, 4), "ntv": 8, "init_iters": 3, "setup_iters": 1, "smoother": SAP_DEFAULT,
               "coarse_restart": 30, "coarse_maxit": 300, "coarse_tol": 0.05, "prec": "f32"}
# alternatives tried on one right-hand side in the solver comparison: P in FP64, two smoother cycles, and more
# test vectors with a second setup pass
AMG_SWEEP = [("p64", dict(AMG_DEFAULT, prec="f64")),
             ("c2", dict(AMG_DEFAULT, smoother=dict(SAP_DEFAULT, cycles=2))),
             ("n12_s2_c2", dict(AMG_DEFAULT, ntv=12, setup_iters=2, smoother=dict(SAP_DEFAULT, cycles=2)))]


def solver_sweep(op, bn, configs):
    """Wall time to 1e-10 of one right-hand side for each candidate configuration (best of the list is used for
    the 12-RHS run; the sweep itself is not part of any reported time)."""
    import torch
    out = []
    for name, kw in configs:
        # the workspace is allocated outside the timed region
        work = torch.empty(op.workspace_bytes(1, kw["restart"], kw["mode"], kw.get("inner_restart", 30), wave=1,
                                              schur=kw.get("schur", False), sap=kw.get("sap"), amg=kw.get("amg")),
                           dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st, rc = op.solve(bn, work=work, wave=1, **kw)
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t, name, kw, st[0]["applies"], rc))
        del work
    return out


def amg_pass_bytes(ntv, prec):
    """Algorithmic bytes per fine site of one restriction or prolongation: the ntv interpolation columns (12
    complex entries per site, FP64 or FP32) and the FP64 fine field."""
    return ntv * (192 if prec == "f64" else 96) + 192


def amg_run(torch, op, dims, stream, steps=10):
    """The two-level multigrid of the benchmark: setup time (from seeded Gaussian test vectors), then its kernels
    (restriction, prolongation, coarse operator) and one application of M timed on one right-hand side.  Returns
    the results and the handle (reused by the solver comparison)."""
    from paper_2407_00041_amd import TwoLevel, synth
    N = AMG_DEFAULT["ntv"]
    V = op.V
    torch.cuda.synchronize()
    t = time.perf_counter()
    tv = op.pack(synth.gaussian_spinor(dims, 4000, nrhs=N, device="cuda"), "f64")
    mg = TwoLevel(op, tv, **AMG_DEFAULT)
    del tv
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    b = op.pack(synth.gaussian_spinor(dims, 4001, nrhs=1, device="cuda"), "f64")
    c = mg.restrict(b)
    ms_r = time_launches(torch, lambda: mg.restrict(b, stream=stream), steps, 2, stream)
    ms_p = time_launches(torch, lambda: mg.prolong(c, stream=stream), steps, 2, stream)
    ms_c = time_launches(torch, lambda: mg.coarse_apply(c, stream=stream), steps, 2, stream)
    s0 = mg.stats()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        mg.precond(b, stream=stream)
    torch.cuda.synchronize()
    ms_m = (time.perf_counter() - t) / 3 * 1e3
    s1 = mg.stats()
    rp = amg_pass_bytes(N, AMG_DEFAULT.get("prec", "f64")) * V
    rc = mg.Vc * (5 * 4 * N * N + 4 * N) * 16
    res = {"params": {k: (list(v) if isinstance(v, tuple) else v) for k, v in AMG_DEFAULT.items() if k != "smoother"},
           "smoother": {k: (list(v) if isinstance(v, tuple) else v) for k, v in AMG_DEFAULT["smoother"].items()},
           "coarse_dims": list(mg.coarse_dims), "unknowns_per_coarse_site": mg.unknowns, "setup_seconds": setup_s,
           "restrict_ms": ms_r, "prolong_ms": ms_p, "coarse_apply_ms": ms_c,
           "restrict_alg_bytes": rp, "coarse_apply_alg_bytes": rc,
           "precond_ms": ms_m, "coarse_applies_per_precond": (s1["coarse_applies"] - s0["coarse_applies"]) / 3}
    del b, c
    return res, mg


# the mixed solver on S as the bench's one-RHS sweep picks it at 48^3 x 96 (outer FGMRES(16), inner GMRES(10) on the
# FP16S S to 0.05): the configuration --solve-profile runs without sweeping
EO_MIXED_PROFILE = dict(tol=1e-10, restart=16, maxit=500, mode="mixed_f16s", schur=True, inner_restart=10,
                        inner_tol=0.05, inner_maxit=10)
MARKER = r"dslash_\w*kernel<1, "   # the FP32 full-lattice stencil, which the even-odd mixed solve never launches


def solve_profile_run(torch, op, dims, nrhs_total, wave_max=0):
    """The mixed even-odd solve alone, in waves sized to the free HBM as in fgmres_run, between two FP32 applies
    whose dispatches mark the solve's window in a kernel trace."""
    from paper_2407_00041_amd import synth
    for n in (1, 2, 3, 6):
        op.autotune("f64", n)
        op.autotune("f16s", n)
    kw = EO_MIXED_PROFILE
    fb = op.field_bytes("f64", 1)
    b_all = op.pack(torch.cat([synth.gaussian_spinor(dims, 3000 + q, nrhs=1, device="cuda")
                               for q in range(nrhs_total)]), "f64")
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    per = op.workspace_bytes(1, kw["restart"], kw["mode"], kw["inner_restart"], wave=1, schur=True) + 3 * fb
    wave = int(max(1, min(nrhs_total, (free - (8 << 30)) // per)))
    if wave_max > 0:
        wave = min(wave, wave_max)
    work = torch.empty(op.workspace_bytes(wave, kw["restart"], kw["mode"], kw["inner_restart"], wave=wave,
                                          schur=True), dtype=torch.uint8, device="cuda")
    bs = [b_all[w0 * fb:min(w0 + wave, nrhs_total) * fb] for w0 in range(0, nrhs_total, wave)]
    m_in, m_out = op.empty("f32", 1), op.empty("f32", 1)
    m_in.zero_()
    torch.cuda.synchronize()
    op.apply_native(m_out, m_in, 1, "f32")
    t, applies, inner = time.perf_counter(), 0, 0
    for w0, b in zip(range(0, nrhs_total, wave), bs):
        nw = min(wave, nrhs_total - w0)
        x, st, _ = op.solve(b, nrhs=nw, work=work, wave=wave, **kw)
        applies += sum(st[k]["applies"] for k in range(nw))
        inner += sum(st[k]["inner_applies"] for k in range(nw))
        del x
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    op.apply_native(m_out, m_in, 1, "f32")
    torch.cuda.synchronize()
    log(f"[bench] solve-profile: mixed on S, {nrhs_total} RHS in waves of {wave}: {el:.3f} s, {applies} outer "
        f"applications of S, {inner} FP16S ones")


def summarize_solve(trace_dir, solve_log, out_md, command):
    """Kernel time of the --solve-profile window (between the last two FP32 stencil dispatches), per kernel and
    per role."""
    import re
    kt = sorted(_read_csv(_find(trace_dir, "kernel_trace.csv")), key=lambda r: int(r["Start_Timestamp"]))
    marks = [i for i, r in enumerate(kt) if re.search(MARKER, r["Kernel_Name"])]
    if len(marks) < 2:
        raise ValueError("fewer than two FP32 stencil dispatches in the trace")
    win = kt[marks[-2] + 1:marks[-1]]
    wall = (int(win[-1]["End_Timestamp"]) - int(win[0]["Start_Timestamp"])) * 1e-9
    roles = [("FP16S S, inner GMRES (parity kernels)", r"parity_\w*kernel<2, "),
             ("FP64 parity kernels: outer S, prepare, reconstruct, true residual", r"parity_\w*kernel<0, "),
             ("inner vector kernels (FP16S basis)", r"k_site_"),
             ("outer vector kernels (FP64 basis)", r"k_mdot_all|k_axpy_multi|k_update|k_residual|k_scale"),
             ("reductions and small solver kernels", r"k_colsum|k_inner_"),
             ("copies (runtime blits, parity split and merge)", r"copyBuffer|parity_copy_kernel")]
    per, role_t = {}, {name: 0.0 for name, _ in roles}
    role_t["other"] = 0.0
    total = 0.0
    for r in win:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
        total += d
        name = re.sub(r"^void |\(anonymous namespace\)::", "", r["Kernel_Name"]).split("(")[0]
        c, t = per.get(name, (0, 0.0))
        per[name] = (c + 1, t + d)
        role = next((n for n, pat in roles if re.search(pat, r["Kernel_Name"])), "other")
        role_t[role] += d
    line = next((ln for ln in open(solve_log).read().splitlines() if ln.startswith("[bench] solve-profile")), "")
    lines = ["# Mixed even-odd FGMRES, 48^3 x 96, 12 right-hand sides to 1e-10: kernel time by role", "",
             "Command (repo root, MI355X):", "", "```", command, "```", "",
             f"Solve log: `{line.strip()}`.", "",
             f"Window: {len(win)} dispatches between the two FP32 marker applies; {wall:.3f} s from the first "
             f"dispatch's start to the last one's end, {total:.3f} s of kernel time ({total / wall:.1%} busy).", "",
             "| role | kernel s | share of kernel time |", "|---|---|---|"]
    for name, t in sorted(role_t.items(), key=lambda kv: -kv[1]):
        lines.append(f"| {name} | {t:.3f} | {t / total:.1%} |")
    lines += ["", "| kernel | calls | total s | avg us |", "|---|---|---|---|"]
    for name, (c, t) in sorted(per.items(), key=lambda kv: -kv[1][1])[:12]:
        lines.append(f"| `{name[:100]}` | {c} | {t:.3f} | {t / c * 1e6:.1f} |")
    lines += ["", f"sources_sha256_16: {all_sources_hash()}", ""]
    with open(out_md, "w") as f:
        f.write("\n".join(lines))
    log(f"[bench] wrote {out_md}")


def fgmres_run(torch, op, dims, nrhs_total, mg=None, amg_setup_s=None):
    """12 right-hand sides to 1e-10, in waves sized to the free HBM, by every
    solver: plain FP64 FGMRES(30) (the reference), plain FP64 at the restart a
    one-RHS sweep picks, the mixed FP64/FP16S solver at the (outer restart,
    inner restart, inner tolerance) a one-RHS sweep picks and at outer restart
    30, FGMRES with the SAP preconditioner, FP64 and mixed on the even-odd
    reduced system (the mixed one swept on S), and FGMRES with the two-level
    multigrid (one setup for all right-hand sides).  Times are summed over the waves; errors
    are against the FP64 FGMRES(30) solution."""
    from paper_2407_00041_amd import synth
    base = dict(tol=1e-10)
    b1 = op.pack(synth.gaussian_spinor(dims, 3000, nrhs=1, device="cuda"), "f64")
    for n in (1, 2, 3, 6):    # batched applies of the solvers' waves (tuning buckets 1, 2, 3-4, 5-8)
        if not TUNE_FIXED:
            op.autotune("f64", n)
            op.autotune("f16s", n)
    sweep64 = solver_sweep(op, b1, [(f"r{m}", dict(base, restart=m, maxit=5000, mode="f64"))
                                    for m in (10, 16, 20, 30, 50)])
    best64 = min(sweep64)
    sweep_sap = solver_sweep(op, b1, [(f"r{m} c{c} mr{k}", dict(base, restart=m, maxit=500, mode="sap",
                                                                sap=dict(SAP_DEFAULT, cycles=c, mr_iters=k)))
                                      for m in (10, 16) for c, k in ((1, 4), (2, 4), (1, 6))])
    best_sap = min(sweep_sap)
    sweep_mixed = {}
    for schur in (False, True):
        sweep_mixed[schur] = solver_sweep(
            op, b1, [(f"r{o} i{ir} t{t}", dict(base, restart=o, maxit=500, mode=MIXED["mode"], schur=schur,
                                               inner_restart=ir, inner_tol=t, inner_maxit=ir))
                     for o, ir, t in MIXED_SWEEP])
    best_mixed = {k: min(v) for k, v in sweep_mixed.items()}
    log("[bench] fp64 restart sweep " + ", ".join(f"{n} {t:.2f}s/{a}" for t, n, _, a, _ in sweep64))
    log("[bench] sap sweep " + ", ".join(f"{n} {t:.3f}s/{a}" for t, n, _, a, _ in sweep_sap))
    for schur in (False, True):
        log(f"[bench] mixed sweep{' on S' if schur else ''} " +
            ", ".join(f"{n} {t:.3f}s/{a}" for t, n, _, a, _ in sweep_mixed[schur]))
    del b1

    def mixed_desc(kw, what):
        return (f"FP64 FGMRES({kw['restart']}){what}, preconditioner inner GMRES({kw['inner_restart']}) on the FP16S "
                f"operator (relative tol {kw['inner_tol']}), the fastest of a one-RHS sweep")
    solvers = [
        ("fp64", "FGMRES(30), FP64", dict(base, restart=30, maxit=5000, mode="f64")),
        ("fp64_best_restart", f"FGMRES({best64[2]['restart']}), FP64 (fastest restart of 10/16/20/30/50 on one RHS)",
         best64[2]),
        ("mixed", mixed_desc(best_mixed[False][2], ""), best_mixed[False][2]),
        ("mixed_restart30", "the mixed solver with outer FGMRES(30)", dict(best_mixed[False][2], restart=30)),
        ("sap", f"FP64 FGMRES({best_sap[2]['restart']}), preconditioner SAP (FP32, 4^4 blocks, red-black, "
                f"{best_sap[2]['sap']['cycles']} cycle(s), {best_sap[2]['sap']['mr_iters']} MR steps)", best_sap[2]),
        ("even_odd_fp64", "FGMRES(30), FP64, on S = A_ee - H_eo A_oo^-1 H_oe",
         dict(base, restart=30, maxit=5000, mode="f64", schur=True)),
        ("even_odd_mixed", mixed_desc(best_mixed[True][2], " on S (FP16S S in the inner GMRES)"),
         best_mixed[True][2]),
    ]
    # two-level multigrid: one setup serves every right-hand side (its time is reported on its own); a few
    # multigrid configurations are tried on one right-hand side and the fastest solves all twelve
    from paper_2407_00041_amd import TwoLevel

    def make_mg(cfg):
        torch.cuda.synchronize()
        t = time.perf_counter()
        tv = op.pack(synth.gaussian_spinor(dims, 4000, nrhs=cfg["ntv"], device="cuda"), "f64")
        m = TwoLevel(op, tv, **cfg)
        del tv
        torch.cuda.synchronize()
        return m, time.perf_counter() - t

    if mg is None:
        mg, amg_setup_s = make_mg(AMG_DEFAULT)
    b1 = op.pack(synth.gaussian_spinor(dims, 3000, nrhs=1, device="cuda"), "f64")
    sweep_amg = []
    best_amg = None
    for k, (name, cfg) in enumerate([("default", AMG_DEFAULT)] + AMG_SWEEP):
        m, ts = (mg, amg_setup_s) if k == 0 else make_mg(cfg)
        (t1, _, _, ap, _), = solver_sweep(op, b1, [(name, dict(base, restart=16, maxit=500, mode="amg", amg=m))])
        sweep_amg.append((t1, name, cfg, ap, ts, None))
        torch.cuda.empty_cache()
        if best_amg is None or t1 < best_amg[0]:
            if best_amg is not None:
                best_amg[5].close()
            best_amg = (t1, name, cfg, ap, ts, m)
        else:
            m.close()
    del b1
    _, amg_name, amg_cfg, _, amg_setup_s, mg = best_amg
    log("[bench] amg sweep " + ", ".join(f"{n} {t:.3f}s/{a} (setup {ts:.2f}s)" for t, n, _, a, ts, _ in sweep_amg))
    log(f"[bench] AMG setup {amg_setup_s:.2f} s (coarse lattice {mg.coarse_dims}, {mg.unknowns} unknowns per site)")
    sm = amg_cfg["smoother"]
    solvers.append(("amg", f"FP64 FGMRES(16), preconditioner two-level multigrid ({amg_cfg['agg']} aggregates, "
                           f"{amg_cfg['ntv']} test vectors, {amg_cfg['init_iters']} + {amg_cfg['setup_iters']} setup "
                           f"passes, SAP post-smoothing with {sm['cycles']} cycle(s) of {sm['mr_iters']} MR steps, "
                           f"coarse GMRES to {amg_cfg['coarse_tol']}, P stored in {amg_cfg.get('prec', 'f64')}); "
                           f"setup time excluded, reported separately",
                    dict(base, restart=16, maxit=500, mode="amg", amg=mg)))
    fb = op.field_bytes("f64", 1)
    torch.cuda.empty_cache()
    # every solver in waves as large as its own workspace allows in the free HBM (lockstep right-hand sides share
    # batched applications); the FP64 FGMRES(30) solutions (kept on the host) are the reference of the errors
    rec = {k: {"solver": d, "seconds": 0.0, "applies": [], "inner_applies": [], "true_residual": [], "err": [],
               "wave": 0, "phase_seconds": {"apply": 0.0, "precond": 0.0, "ortho": 0.0}} for k, d, _ in solvers}
    ref = {}
    for key, _, kw in solvers:
        free, _ = torch.cuda.mem_get_info()
        per = op.workspace_bytes(1, kw["restart"], kw["mode"], kw.get("inner_restart", 30), wave=1,
                                 schur=kw.get("schur", False), sap=kw.get("sap"), amg=kw.get("amg")) + 3 * fb
        wave = int(max(1, min(nrhs_total, (free - (8 << 30)) // per)))
        work = torch.empty(op.workspace_bytes(wave, kw["restart"], kw["mode"], kw.get("inner_restart", 30),
                                              wave=wave, schur=kw.get("schur", False), sap=kw.get("sap"),
                                              amg=kw.get("amg")), dtype=torch.uint8, device="cuda")
        r = rec[key]
        r["wave"] = wave
        for w0 in range(0, nrhs_total, wave):
            nw = min(wave, nrhs_total - w0)
            b = op.pack(torch.cat([synth.gaussian_spinor(dims, 3000 + q, nrhs=1, device="cuda")
                                   for q in range(w0, w0 + nw)]), "f64")
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, st, _ = op.solve(b, nrhs=nw, work=work, wave=wave, **kw)
            torch.cuda.synchronize()
            r["seconds"] += time.perf_counter() - t
            for ph in r["phase_seconds"]:
                r["phase_seconds"][ph] += sum(st[k]["seconds_" + ph] for k in range(0, nw, wave))
            for k in range(nw):
                v = x[k * fb:(k + 1) * fb].view(torch.float64).cpu()
                if key == "fp64":
                    ref[w0 + k] = v
                u = ref[w0 + k]
                r["err"].append(float(torch.linalg.vector_norm(u - v) / torch.linalg.vector_norm(u)))
                r["applies"].append(st[k]["applies"])
                r["inner_applies"].append(st[k]["inner_applies"])
                r["true_residual"].append(st[k]["true_residual"])
            del x, b
        del work
        torch.cuda.empty_cache()
        log(f"[bench] fgmres {key}: {nrhs_total} RHS in waves of {wave}, {r['seconds']:.2f} s, "
            f"applies {sum(r['applies'])}")
    amg_stats = mg.stats()
    mg.close()
    torch.cuda.empty_cache()
    out = {"nrhs": nrhs_total, "tol": 1e-10,
           "amg_setup_seconds": amg_setup_s, "amg_coarse": {"dims": list(mg.coarse_dims), "unknowns_per_site":
                                                             mg.unknowns, **amg_stats},
           "sweeps_one_rhs_seconds": {"fp64": {n: t for t, n, *_ in sweep64},
                                      "sap": {n: t for t, n, *_ in sweep_sap},
                                      "mixed": {n: t for t, n, *_ in sweep_mixed[False]},
                                      "mixed_on_S": {n: t for t, n, *_ in sweep_mixed[True]},
                                      "amg": {n: {"solve": t, "applies": a, "setup": ts}
                                              for t, n, _, a, ts, _ in sweep_amg}},
           "amg_config": amg_name}
    for k, r in rec.items():
        out[k] = {"solver": r["solver"], "seconds": r["seconds"], "wave": r["wave"],
                  "phase_seconds": r["phase_seconds"], "applies": r["applies"], "true_residual_max": max(r["true_residual"]),
                  "converged": all(x < 1e-10 for x in r["true_residual"]),
                  "error_vs_fp64_max": max(r["err"])}
        if any(r["inner_applies"]):
            out[k]["inner_applies"] = r["inner_applies"]
    t64 = rec["fp64"]["seconds"]
    out["speedup_vs_fp64"] = {k: t64 / r["seconds"] for k, r in rec.items() if r["seconds"] > 0}
    out["speedup_vs_fp64_best_restart"] = {k: rec["fp64_best_restart"]["seconds"] / r["seconds"]
                                           for k, r in rec.items() if r["seconds"] > 0}
    return out


def sap_run(torch, op, psid, stream, steps=10):
    """One SAP application (FP32 4^4 blocks, one red-black cycle, 4 MR steps) on one right-hand side: time,
    algorithmic bytes and flops per cycle (model in the design notes)."""
    bn = op.pack(psid, "f64")
    x = torch.empty_like(bn)
    ms = time_launches(torch, lambda: op.sap(bn, x=x, **SAP_DEFAULT), steps, 2, stream)
    V = op.V
    ab = SAP_BYTES_SITE_CYCLE * V
    fl = SAP_FLOP_SITE_CYCLE * V
    del bn, x
    return {"ms_per_cycle": ms, "params": {k: list(v) if isinstance(v, tuple) else v for k, v in SAP_DEFAULT.items()},
            "alg_bytes_per_cycle": ab, "alg_GBps": ab / (ms * 1e-3) / 1e9, "frac_hbm": ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "flop_per_cycle": fl, "TFLOPs": fl / (ms * 1e-3) / 1e12, "frac_fp32_vector": fl / (ms * 1e-3) / 157.3e12}


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


# ---------------------------------------------------------------------------
# Per-kernel measurement.  Every product kernel runs at the benchmark sizes in
# `kernel_suite` (for rocprofv3 kernel traces and FETCH_SIZE / WRITE_SIZE
# counter runs); the suite writes a manifest of the algorithmic bytes of its
# dispatches, kernel by kernel, which `summarize_profile` joins with the
# profiler's CSV output into the committed summaries.

FIELD = {"f64": 192, "f32": 96, "f16s": 52}           # bytes per site of one native field
SAP_BYTES_SITE_CYCLE = 992   # FP32 SAP (two-row links, compact clover), first cycle from x = 0, per site
SAP_FLOP_SITE_CYCLE = 9000   # with 4 MR steps per block solve (model in the design notes)
FORCE_BYTES_SITE = {"insert": 384 + 480, "link": 576 + 384 + 480 + 576}
# even-odd reduced operator, two right-hand sides per launch: bytes per half-lattice site of each launch
SCHUR_PAIR_BYTES_HALF = {"f64": (2112, 2368), "f32": (1056, 1184), "f16s": (544, 616)}
PREC_ID = {"f64": 0, "f32": 1, "f16s": 2}


def _fixed(wd, order, block, tchunk, nr):
    for k, v in (("order", order), ("block", block), ("tchunk", tchunk), ("nr_f64", nr), ("nr_f32", nr),
                 ("nr_f16s", nr)):
        wd.tune_set(k, v)


def site_pass_bytes(nv, field, extra_w):
    """Bytes of the per-site Gram-Schmidt launches for nv basis vectors (passes of 8): every pass reads its
    vectors and w; extra_w adds w's write per pass."""
    passes = max(1, -(-nv // 8))
    return [(min(8, nv - 8 * k) + 1 + extra_w) * field for k in range(passes)]


def kernel_suite(torch, manifest_path, dims=(96, 48, 48, 48)):
    """Every product kernel at the benchmark sizes, with fixed launch
    configurations (no autotuning inside the profiled region); writes the
    manifest {pattern: {"dispatches": n, "alg_bytes": total, "note": ...}}."""
    import paper_2407_00041_amd as wd
    from paper_2407_00041_amd import synth
    V = int(np.prod(dims))
    Ud = synth.smooth_links(dims, 1003, device="cuda")
    psid = synth.gaussian_spinor(dims, 2000, nrhs=2, device="cuda")
    U = Ud.cpu().numpy()
    del Ud
    op = wd.DiracOp(dims, U, -0.35, 1.0, precisions=("f64", "f32", "f16s"), compress_links=True,
                    compress_clover=True, even_odd=True)
    man = {}

    # a pattern's dispatches are its first `dispatches` matches in launch order (its last ones with
    # select = "last"): later solver sections launch the same kernels with other sizes
    def add(pattern, n, nbytes, note):
        e = man.setdefault(pattern, {"dispatches": 0, "alg_bytes": 0.0, "note": note})
        e["dispatches"] += n
        e["alg_bytes"] += float(nbytes)

    st = torch.cuda.current_stream()
    reps = 5
    # single applies (the benchmark's launches: column sweep FP64/FP32, T-sweep site kernel FP16S)
    for p, cfg, pat in (("f64", (3, 256, 2, 1), r"dslash_column_kernel<0, false, 1>"),
                        ("f32", (3, 256, 2, 1), r"dslash_column_kernel<1, false, 1>"),
                        ("f16s", (2, 256, 4, 1), r"dslash_kernel<2, false, 1>")):
        _fixed(wd, *cfg)
        x = op.pack(psid[:1], p)
        y = op.empty(p, 1)
        for _ in range(reps):
            op.apply_native(y, x, 1, p, stream=st)
        add(pat, reps, reps * BYTES_SITE[p] * V, f"D apply {p}, 1 RHS")
        del x, y
    torch.cuda.synchronize()
    log("[suite] single applies done")
    # one FP32 apply over batches {1, 4, 12, 24}: the link-stationary kernel over z-pair tiles walked in (y, x)
    # blocks, in launches of 16 right-hand sides
    group = 16
    _fixed(wd, 5, 128, group, 4)
    sizes = [1, 4, 12, 24]
    n = sum(sizes)
    nat = op.pack(synth.gaussian_spinor(dims, 2100, nrhs=n, device="cuda"), "f32")
    rb = op.field_bytes("f32", 1)
    outs, batches, r0 = [], [], 0
    for k in sizes:
        o = op.empty("f32", k)
        outs.append(o)
        batches.append((o, nat[r0 * rb:(r0 + k) * rb], k))
        r0 += k
    for _ in range(2):
        op.apply_batched(batches, "f32", stream=st)
    nl = -(-n // group)
    add(r"dslash_stationary_kernel<1, false>", 2 * nl,
        2 * (nl * (LINK_BYTES["f32"] + CLOVER_BYTES["f32"]) + 192 * n) * V,
        f"batched FP32 apply, 41 RHS in batches {{1,4,12,24}}, z-pair tiles in (y, x) blocks, launches of {group} RHS")
    _fixed(wd, 5, 128, 1, 1)     # the later sections' launches as before
    del outs, batches, nat
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log("[suite] batched launch done")
    # even-odd reduced operator S on pairs of right-hand sides
    for p in ("f64", "f32", "f16s"):
        e, o = op.split(op.pack(psid, p), p, 2)
        out, tmp = op.empty_parity(p, 2), op.empty_parity(p, 2)
        for _ in range(3):
            op.apply_schur_native(out, e, tmp, 2, p, stream=st)
        bo, be = SCHUR_PAIR_BYTES_HALF[p]
        kern = "parity_column_kernel" if p != "f16s" else "parity_kernel"
        i = PREC_ID[p]
        add(kern + rf"<(P,DAG,SELF,HOP,INV,ROWS = )?{i}, false, 0, true, true", 3, 3 * bo * V / 2,
            f"S (pair), odd launch A_oo^-1 H_oe, {p}")
        add(kern + rf"<(P,DAG,SELF,HOP,INV,ROWS = )?{i}, false, 2, true, false", 3, 3 * be * V / 2,
            f"S (pair), even launch A_ee - H_eo, {p}")
        del e, o, out, tmp
    torch.cuda.synchronize()
    log("[suite] even-odd done")
    # SAP, FP32 blocks of 4^4, one red-black cycle, 4 MR steps (two launches per cycle)
    bn = op.pack(psid[:1], "f64")
    for _ in range(3):
        op.sap(bn, block=(4, 4, 4, 4), cycles=1, mr_iters=4, prec="f32")
    add(r"sap_pass_kernel<1, true, true>", 6, 3 * SAP_BYTES_SITE_CYCLE * V, "SAP cycle FP32 4^4 blocks (2 passes)")
    torch.cuda.synchronize()
    log("[suite] SAP done")
    # two-level multigrid: restriction, prolongation (8 test vectors on 4^4 aggregates) and the coarse operator
    from paper_2407_00041_amd import TwoLevel
    N = AMG_DEFAULT["ntv"]
    tv = op.pack(synth.gaussian_spinor(dims, 4000, nrhs=N, device="cuda"), "f64")
    mg = TwoLevel(op, tv, **dict(AMG_DEFAULT, init_iters=0, setup_iters=0))
    del tv
    c = mg.restrict(bn)
    for _ in range(3):
        mg.restrict(bn)
        mg.prolong(c)
        mg.coarse_apply(c)
    torch.cuda.synchronize()
    pp = AMG_DEFAULT.get("prec", "f64")
    add(r"k_restrict", 4, 4 * amg_pass_bytes(N, pp) * V, f"AMG restriction P^H f ({N} test vectors, P in {pp})")
    add(r"k_prolong", 3, 3 * amg_pass_bytes(N, pp) * V, f"AMG prolongation P c ({N} test vectors, P in {pp})")
    add(r"k_coarse_apply", 3, 3 * mg.Vc * (5 * 4 * N * N + 4 * N) * 16,
        "AMG coarse operator D_c (self + 4 forward blocks once, vectors in and out)")
    mg.close()
    del c
    log("[suite] multigrid done")
    # one cycle of plain FP64 FGMRES(30) (the outer Gram-Schmidt kernels), and the mixed solver's inner cycles
    _fixed(wd, 3, 256, 2, 1)
    x, stt, _ = op.solve(bn, restart=30, tol=1e-14, maxit=31)
    assert stt[0]["applies"] == 32, stt[0]["applies"]
    vec = 192.0 * V
    add(r"dslash_column_kernel<0, false, 1>", 32, 32 * BYTES_SITE["f64"] * V, "D apply inside FGMRES")
    add(r"k_mdot_all", 30, sum(j + 2 for j in range(30)) * vec, "outer inner products, nv = 1..30 (w once)")
    add(r"k_axpy_multi", 30, sum(j + 3 for j in range(30)) * vec, "outer CGS update, nv = 1..30")
    add(r"k_residual", 2, 2 * 3 * vec, "restart residual b - D x")
    add(r"k_update", 1, 32 * vec, "x += Z y, 30 vectors")
    del x
    torch.cuda.synchronize()
    _fixed(wd, 2, 256, 4, 1)   # inner FP16S applies: the T-sweep site kernel
    x, stm, _ = op.solve(bn, restart=8, tol=1e-14, maxit=9, mode="mixed_f16s", inner_restart=10, inner_tol=1e-14,
                         inner_maxit=10)
    steps = stm[0]["applies"] - 2
    assert stm[0]["inner_applies"] == 10 * steps, stm[0]
    f16 = 52.0 * V
    mdot = sum(sum(site_pass_bytes(k + 1, f16, 0)) for k in range(10)) * steps
    axpy = sum(sum(site_pass_bytes(k + 1, f16, 1)) for k in range(10)) * steps
    nmd = sum(len(site_pass_bytes(k + 1, f16, 0)) for k in range(10)) * steps
    add(r"dslash_kernel<2, false, 1>", 10 * steps, 10 * steps * BYTES_SITE["f16s"] * V, "inner FP16S applies")
    add(r"k_site_mdot<2>", nmd, mdot, "inner inner products (FP16S fields)")
    add(r"k_site_axpy<2>", nmd, axpy, "inner orthogonalisation (FP16S fields)")
    add(r"k_site_combine<2>", 2 * steps, steps * (10 * 52 + 192 + 2 * 192) * V, "inner solution into Z (FP64)")
    add(r"k_site_scale<0, 2>", steps, steps * (192 + 52) * V, "outer v_j to the inner FP16S start vector")
    del x, bn
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    del op
    log("[suite] solver cycles done")
    # the link derivative at 24^3 x 48
    fd = (48, 24, 24, 24)
    Vf = int(np.prod(fd))
    Uf = synth.smooth_links(fd, 1005, device="cuda").cpu().numpy()
    opf = wd.DiracOp(fd, Uf, -0.3, 1.0, precisions=("f64",))
    en = opf.pack(synth.gaussian_spinor(fd, 3002, nrhs=1, device="cuda"), "f64")
    xn = opf.pack(synth.gaussian_spinor(fd, 3001, nrhs=1, device="cuda"), "f64")
    for _ in range(3):
        opf.force(en, xn, 1)
    add(r"force_insert_kernel", 3, 3 * FORCE_BYTES_SITE["insert"] * Vf, "force pass 1 at 24^3x48")
    add(r"force_link_kernel", 3, 3 * FORCE_BYTES_SITE["link"] * Vf, "force pass 2 at 24^3x48")
    torch.cuda.synchronize()
    del opf, en, xn
    # copy probe of known size (counter calibration): 1 GiB read, 1 GiB written, 5 times
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    add(r"vectorized_elementwise_kernel<4, at::native::[AB]UnaryFunctor<float, float, float, "
        r"at::native::binary_internal::MulFunctor<float", 5, 5 * 2 * (1 << 30),
        "copy probe (torch.mul), 1 GiB in + 1 GiB out")
    man[list(man)[-1]]["select"] = "last"
    wd.tune_set("explicit", 0)
    # the sources this run was built from (the summary records these, not the sources present when it is written)
    man["_sources"] = {"all": all_sources_hash(), "kernel": kernel_hash()}
    with open(manifest_path, "w") as f:
        json.dump(man, f, indent=1)
    log(f"[bench] kernel suite done; manifest {manifest_path}")


def _read_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _find(d, suffix):
    import glob
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def summarize_headline(trace_dir, bench_log, out_md, command):
    """The timed FP64 stencil launches of one bench run under rocprofv3 --kernel-trace: the bench times
    `warmup + steps` launches of its autotuned kernel last (autotuning launches of the same kernel come
    earlier), so the last that many dispatches of that kernel are the timed ones."""
    text = open(bench_log).read()
    j = json.loads(next(ln for ln in reversed(text.splitlines()) if ln.startswith("{")))
    kern, n = j["roofline"]["kernel"], j["steps"] + j["warmup"]
    ev = next(ln for ln in text.splitlines() if ln.startswith("[bench] FP64:"))
    kt = sorted(_read_csv(_find(trace_dir, "kernel_trace.csv")), key=lambda r: int(r["Dispatch_Id"]))
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3 for r in kt
            if r["Kernel_Name"].startswith("void " + kern + "(") or r["Kernel_Name"].startswith(kern + "(")]
    seen, durs = len(durs), durs[-n:]
    avg = sum(durs) / len(durs)
    alg = j["roofline"]["alg_bytes_per_launch"]
    stats = _read_csv(_find(trace_dir, "kernel_stats.csv"))
    lines = [f"# FP64 Wilson-clover stencil, 48^3 x 96, one RHS: kernel trace of the bench command", "",
             "Command (repo root, MI355X):", "", "```", command, "```", "",
             f"Kernel `{kern}` (launch {json.dumps(j['extra']['f64']['launch'])}).",
             f"Bench's own HIP-event timing in the same run: `{ev.strip()}`.", "",
             f"Timed dispatches (the last {n} of {seen}; earlier ones are the autotuner's candidates): average "
             f"{avg:.1f} us (min {min(durs):.1f}, max {max(durs):.1f}). Algorithmic bytes per launch "
             f"{j['roofline']['alg_bytes_per_site']} B/site x {j['config']['sites']} sites = {alg / 1e9:.2f} GB -> "
             f"{alg / (avg * 1e-6) / 1e9:.0f} GB/s = {alg / (avg * 1e-6) / 1e9 / HBM_PEAK_GBS:.3f} of 8 TB/s.", "",
             "Top kernels of the whole run (input generation, operator setup and autotuning included):", "",
             "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:8]:
        name = r["Name"] if len(r["Name"]) < 110 else r["Name"][:60] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    lines += ["", f"kernel_source_sha256_16: {kernel_hash()}", ""]
    with open(out_md, "w") as f:
        f.write("\n".join(lines))
    log(f"[bench] wrote {out_md}")


def summarize_profile(manifest_path, trace_dir, fetch_dir, write_dir, out_md, command):
    """Join the suite's manifest with rocprofv3 output: per kernel pattern the
    dispatch count, average duration, algorithmic GB/s, and the counter bytes
    (FETCH_SIZE scaled by the copy probe's calibration, WRITE_SIZE likewise)."""
    man = json.load(open(manifest_path))
    src = man.pop("_sources", {"all": all_sources_hash(), "kernel": kernel_hash()})
    kt = sorted(_read_csv(_find(trace_dir, "kernel_trace.csv")), key=lambda r: int(r["Dispatch_Id"]))

    def counters(d, name):
        rows = sorted(_read_csv(_find(d, "counter_collection.csv")), key=lambda r: int(r["Dispatch_Id"]))
        out = []
        for r in rows:
            if r.get("Counter_Name", "") == name:
                out.append((r["Kernel_Name"], float(r["Counter_Value"])))
        return out

    fetch = counters(fetch_dir, "FETCH_SIZE")
    write = counters(write_dir, "WRITE_SIZE")
    res = {}

    def pick(items, e):
        n = e["dispatches"]
        return items[-n:] if e.get("select") == "last" else items[:n]

    for pat, e in man.items():
        rx = re.compile(pat)
        durs = pick([(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9 for r in kt
                     if rx.search(r["Kernel_Name"])], e)
        fk = pick([v for k, v in fetch if rx.search(k)], e)
        wk = pick([v for k, v in write if rx.search(k)], e)
        res[pat] = {"note": e["note"], "dispatches": e["dispatches"], "seen": len(durs),
                    "seconds": sum(durs), "alg_bytes": e["alg_bytes"],
                    "fetch_kib": sum(fk), "write_kib": sum(wk), "counted": (len(fk), len(wk))}
    probe = next(p for p in res if "MulFunctor<float" in p)
    cal_f = res[probe]["alg_bytes"] / 2 / max(res[probe]["fetch_kib"] * 1024, 1)
    cal_w = res[probe]["alg_bytes"] / 2 / max(res[probe]["write_kib"] * 1024, 1)
    lines = ["# Product kernels at the benchmark sizes: time, algorithmic and counted HBM traffic", "",
             "Commands (repo root, MI355X; three separate runs of the same kernel suite, then the join):", "",
             "```", command, "```", "",
             f"Calibration: the suite's copy probe (1 GiB read + 1 GiB written per dispatch) reads as FETCH_SIZE x "
             f"{cal_f:.3f} and WRITE_SIZE x {cal_w:.3f}; both factors are applied below.  Counter bytes are measured "
             f"at the L2's memory side (Infinity Cache hits included), an upper bound on HBM bytes.", "",
             "| kernel (pattern) | what | dispatches | avg us | alg GB/launch | alg GB/s | frac of 8 TB/s | "
             "counted read GB/launch | counted write GB/launch | counted GB/s | counted / alg |",
             "|---|---|---|---|---|---|---|---|---|---|---|"]
    for pat, r in res.items():
        n = max(r["seen"], 1)
        avg = r["seconds"] / n
        ab = r["alg_bytes"] / max(r["dispatches"], 1)
        rd = r["fetch_kib"] * 1024 * cal_f / max(r["counted"][0], 1)
        wr = r["write_kib"] * 1024 * cal_w / max(r["counted"][1], 1)
        ag = ab / avg / 1e9 if avg > 0 else 0.0
        cg = (rd + wr) / avg / 1e9 if avg > 0 else 0.0
        lines.append(f"| `{pat}` | {r['note']} | {r['seen']} (expected {r['dispatches']}) | {avg * 1e6:.1f} | "
                     f"{ab / 1e9:.4f} | {ag:.0f} | {ag / HBM_PEAK_GBS:.3f} | {rd / 1e9:.4f} | {wr / 1e9:.4f} | "
                     f"{cg:.0f} | {(rd + wr) / ab if ab else 0:.2f} |")
    lines += ["", f"sources_sha256_16: {src['all']}", f"kernel_source_sha256_16: {src['kernel']}", ""]
    with open(out_md, "w") as f:
        f.write("\n".join(lines))
    log(f"[bench] wrote {out_md}")


def kernel_table(extra, V):
    """One roofline entry per product kernel measured in this run (HIP events on the launch stream), with the
    counted traffic of the committed kernel-suite summary when it matches the sources."""
    prof = kernel_profile_rows()
    rows = []

    def row(kernel, what, ms, alg_bytes, pattern, flops=None):
        r = {"kernel": kernel, "what": what, "ms": ms, "alg_bytes": alg_bytes,
             "alg_GBps": alg_bytes / (ms * 1e-3) / 1e9, "frac_of_8TBps": alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
             "counted": prof.get(pattern)}
        if flops:
            r["TFLOPs"] = flops / (ms * 1e-3) / 1e12
        rows.append(r)

    for p, pat in (("f64", "dslash_column_kernel<0, false, 1>"), ("f32", "dslash_column_kernel<1, false, 1>"),
                   ("f16s", "dslash_kernel<2, false, 1>")):
        if p in extra:
            row(pat, f"D apply {p}, 1 RHS", extra[p]["ms"], BYTES_SITE[p] * V, pat)
    if "batched" in extra:
        b = extra["batched"]
        n = sum(b["batches"])
        row("dslash_stationary_kernel<1, false>", f"FP32 apply, {n} RHS in batches {b['batches']}",
            b["ms_per_launch"], (LINK_BYTES["f32"] + CLOVER_BYTES["f32"] + 192 * n) * V,
            "dslash_stationary_kernel<1, false>")
    for p, e in extra.get("even_odd_apply", {}).items():
        row(f"parity kernels {p}", f"S = A_ee - H_eo A_oo^-1 H_oe, {p}, per RHS of a pair (two launches)",
            e["ms_per_rhs_pair"], e["alg_bytes_per_site"][1] * V, None)
    if "sap" in extra:
        row("sap_pass_kernel<1, true, true>", "SAP cycle, FP32 4^4 blocks, 4 MR steps (two launches)",
            extra["sap"]["ms_per_cycle"], extra["sap"]["alg_bytes_per_cycle"], "sap_pass_kernel<1, true, true>",
            extra["sap"]["flop_per_cycle"])
    if "amg" in extra:
        m = extra["amg"]
        pp = m["params"].get("prec", "f64")
        row("k_restrict", f"AMG restriction P^H f, P in {pp}, 8 test vectors", m["restrict_ms"],
            m["restrict_alg_bytes"], "k_restrict")
        row("k_prolong", f"AMG prolongation P c, P in {pp}, 8 test vectors", m["prolong_ms"], m["restrict_alg_bytes"],
            "k_prolong")
        row("k_coarse_apply", "AMG coarse operator D_c, FP64", m["coarse_apply_ms"], m["coarse_apply_alg_bytes"],
            "k_coarse_apply")
    if "differentiation" in extra:
        d = extra["differentiation"]
        Vf = int(np.prod(d["dims"]))
        row("force_insert_kernel + force_link_kernel", "link derivative at 24^3x48 (two passes)",
            d["force_kernel_ms"], (FORCE_BYTES_SITE["insert"] + FORCE_BYTES_SITE["link"]) * Vf, None)
    return rows


def cpu_info():
    """CPU model and identification numbers from /proc/cpuinfo, and the CPU set this process may use."""
    info = {"logical_cpus_in_affinity": len(os.sched_getaffinity(0)), "logical_cpus_at_start": len(START_CPUS),
            "os_cpu_count": os.cpu_count()}
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k = k.strip()
            if k in ("model name", "vendor_id", "cpu family", "model", "stepping", "cpu MHz") and k not in info:
                info[k] = v.strip()
    except OSError:
        pass
    return info


# the CPU set the process started with (the GPU runtime may narrow the main thread's mask once it initialises)
START_CPUS = os.sched_getaffinity(0)


def _oracle_threads():
    """Restore the process's starting CPU set on this thread (OpenMP threads inherit it) and use one oracle thread
    per CPU in it."""
    import oracle
    try:
        os.sched_setaffinity(0, START_CPUS)
    except OSError:
        pass
    n = len(os.sched_getaffinity(0))
    oracle.set_threads(n)
    return oracle.num_threads()


def cpu_baseline_run(dims, U, psi, m0, csw, target_s=3.0):
    """Oracle apply on a contiguous slab of T-slices (clover rows built first,
    outside the timed call); the slab is sized from a one-slice calibration so
    the timed apply takes about target_s seconds."""
    import oracle
    threads = _oracle_threads()
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
    return {"value": apps, "unit": "Dirac apps/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle apply on {nsl} of {dims[0]} T-slices ({len(sites)} of {V} sites, "
                      f"clover rows precomputed), {dt:.2f} s, scaled to the whole lattice; threads = the "
                      f"process's CPU affinity set, OMP_PROC_BIND=close",
            "cpu": cpu_info()}


def oracle_fgmres_model(dims, site_rate, steps, restart=20, full_args=None, sample_sites=1 << 18):
    """The oracle FGMRES (Algorithm 2, modified Gram-Schmidt) on the host, as a bounded sample.

    The oracle's operator application is timed by cpu_baseline_run (sites per second, ``site_rate``); one
    modified Gram-Schmidt inner iteration (an inner product and a vector update in NumPy) is timed on a vector of
    ``sample_sites`` sites and scaled to the lattice; the solve is extrapolated from the iteration structure the
    GPU solve of the same system reported (applications; step j of a restart cycle costs j + 1 inner iterations).
    With full_args = (U, m0, csw, seed) the oracle FGMRES runs to 1e-10 and is timed whole instead."""
    import oracle
    V = int(np.prod(dims))
    if full_args is not None:
        from paper_2407_00041_amd import synth
        U, m0, csw, seed = full_args
        b = synth.gaussian_spinor(dims, seed)
        C = oracle.clover_term(dims, U)
        t = time.perf_counter()
        _, info = oracle.fgmres(lambda v: oracle.dirac_apply(dims, U, v, m0, csw, clover=C), b, m=restart,
                                tol=1e-10, maxit=10 * steps)
        return {"seconds": time.perf_counter() - t, "applies": info["applies"], "extrapolated": False}
    t_apply = V / site_rate
    n = min(V, sample_sites)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(12 * n) + 1j * rng.standard_normal(12 * n)
    w = rng.standard_normal(12 * n) + 1j * rng.standard_normal(12 * n)
    t = time.perf_counter()
    for _ in range(5):
        h = np.vdot(v, w)
        w = w - h * v
    t_gs = (time.perf_counter() - t) / 5 * (V / n)
    cycles = -(-(steps - 1) // (restart + 1))   # each ends with the next cycle's (or the final) residual
    arnoldi = steps - cycles - 1
    gs = 0
    left = arnoldi
    while left > 0:
        k = min(restart, left)
        gs += k * (k + 1) // 2
        left -= k
    est = steps * t_apply + gs * t_gs
    return {"seconds": est, "applies": steps, "extrapolated": True, "t_apply_s": t_apply, "t_gs_inner_s": t_gs,
            "model": f"{steps} applications x {t_apply:.2f} s (the timed oracle apply rate) + {gs} Gram-Schmidt "
                     f"inner iterations x {t_gs:.3f} s (NumPy, timed on {n} sites and scaled), restart {restart}, "
                     f"iteration counts of the GPU solve"}


def main():
    global TUNE_FIXED
    # the oracle's OpenMP threads stay on the CPUs of this process's affinity set, packed
    os.environ.setdefault("OMP_PROC_BIND", "close")
    a = parse()
    TUNE_FIXED = bool(a.fixed_launch)
    if a.summarize_headline:
        summarize_headline(*a.summarize_headline, command=a.summary_command)
        return
    if a.summarize:
        summarize_profile(*a.summarize, command=a.summary_command)
        return
    if a.summarize_solve:
        summarize_solve(*a.summarize_solve, command=a.summary_command)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the library has no multi-GPU "
                                   "halo exchange"}))
        sys.exit(2)
    import torch

    import paper_2407_00041_amd as wd
    from paper_2407_00041_amd import synth

    if a.kernel_suite:
        torch.cuda.set_device(0)
        kernel_suite(torch, a.kernel_suite)
        return

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
    if a.solve_profile:
        del psid
        solve_profile_run(torch, op, dims, a.fgmres_rhs, a.solve_wave)
        return
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
        y64 = op.unpack(out["f64"], "f64")
        n64 = torch.linalg.vector_norm(y64)
        for p in ("f32", "f16s"):
            m = time_launches(torch, lambda: op.apply_native(out[p], inp[p], 1, p, stream=stream),
                              max(10, a.steps // 2), a.warmup, stream)
            err = float(torch.linalg.vector_norm(op.unpack(out[p], p) - y64) / n64)
            extra[p] = {"ms": m, "apps_per_s": 1000.0 / m, "alg_GBps": BYTES_SITE[p] * V / (m * 1e-3) / 1e9,
                        "launch": tuned[p], "GFLOPs_1320": FLOP_HOP * V / (m * 1e-3) / 1e9,
                        "rel_error_vs_fp64_apply": err}
            log(f"[bench] {p}: {m:.4f} ms/apply, error vs FP64 {err:.2e}")
        del y64
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
    if not a.no_extra:
        extra["sap"] = sap_run(torch, op, psid, stream)
        log(f"[bench] SAP cycle (FP32, 4^4 blocks, 4 MR): {extra['sap']['ms_per_cycle']:.3f} ms, "
            f"{extra['sap']['alg_GBps']:.0f} GB/s, {extra['sap']['TFLOPs']:.1f} TFLOP/s")
    mg = None
    if not a.no_extra:
        extra["amg"], mg = amg_run(torch, op, dims, stream)
        log(f"[bench] AMG: setup {extra['amg']['setup_seconds']:.2f} s, restrict {extra['amg']['restrict_ms']:.3f} ms, "
            f"prolong {extra['amg']['prolong_ms']:.3f} ms, coarse apply {extra['amg']['coarse_apply_ms']:.3f} ms, "
            f"M {extra['amg']['precond_ms']:.1f} ms")
    if not a.no_extra and not a.no_fgmres and a.fgmres_rhs > 0:
        extra["fgmres"] = fgmres_run(torch, op, dims, a.fgmres_rhs, mg, extra["amg"]["setup_seconds"])
    elif mg is not None:
        mg.close()
    mg = None
    if not a.no_extra:
        log("[bench] 32^4: FP64 apply and FGMRES(20)")
        extra["config_32"] = config32_run(torch, stream)
        log(f"[bench] 32^4: {extra['config_32']['apply_ms']:.4f} ms/apply, FGMRES(20) "
            f"{extra['config_32']['fgmres20_fp64']['seconds']:.2f} s")
        log("[bench] 24^3x48: differentiation")
        extra["differentiation"] = differentiation_run(torch)
        log(f"[bench] 24^3x48: forward+backward {extra['differentiation']['forward_backward_ms']:.2f} ms")

    if not a.no_extra:
        extra["kernels"] = kernel_table(extra, V)
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
        if not a.no_extra:
            # the oracle FGMRES beside the GPU solves: FGMRES(20) at 32^4, and one right-hand side of the
            # 48^3 x 96 FP64 FGMRES(30) run extrapolated to the 12 right-hand sides
            site_rate = res["cpu_baseline"]["value"] * V
            c32 = extra.get("config_32", {}).get("fgmres20_fp64", {})
            if c32:
                full = None
                if a.cpu_full:
                    U32 = synth.smooth_links((32, 32, 32, 32), 1002, device="cuda").cpu().numpy()
                    full = (U32, -0.3, 1.0, 2000)
                o32 = oracle_fgmres_model((32, 32, 32, 32), site_rate, c32["applies"], 20, full)
                o32["gpu_seconds"] = c32["seconds"]
                res["cpu_baseline"]["fgmres20_32^4"] = o32
                log(f"[bench] oracle FGMRES(20) 32^4: {o32['seconds']:.1f} s (GPU {c32['seconds']:.2f} s)")
            f64 = extra.get("fgmres", {}).get("fp64")
            if f64:
                o48 = oracle_fgmres_model(dims, site_rate, int(f64["applies"][0]), 30)
                o48["rhs"] = 12
                o48["seconds_12_rhs_extrapolated"] = 12 * o48["seconds"]
                o48["gpu_seconds_12_rhs"] = f64["seconds"]
                res["cpu_baseline"]["fgmres30_48^3x96"] = o48
                log(f"[bench] oracle FGMRES(30) 48^3x96, 12 RHS (extrapolated): "
                    f"{o48['seconds_12_rhs_extrapolated']:.0f} s (GPU {f64['seconds']:.1f} s)")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
