"""Host logic of the measurement tooling (CPU only): the kernel-suite join of
bench.py (manifest + kernel trace + FETCH_SIZE/WRITE_SIZE counters ->
per-kernel table) and the headline kernel-trace summary, on synthetic
rocprofv3-style CSV files with known values; and the lookup of the
committed summaries by the bench."""
import csv
import json
import os

import pytest

import bench


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)


PROBE = "vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<float, float, float, at::native::binary_internal::MulFunctor<float"


def _suite(tmp_path):
    """Two kernels and the copy probe: kernel A (3 dispatches of 2 ms, 4 GB algorithmic each, FETCH 1.5 GiB and
    WRITE 1 GiB raw per dispatch), kernel B (1 dispatch), probe 2 dispatches reading as FETCH_SIZE = half its
    bytes (factor 2) and WRITE_SIZE = its bytes (factor 1)."""
    gib = 1 << 30
    man = {
        "kernelA<0>": {"dispatches": 3, "alg_bytes": 3 * 4e9, "note": "kernel A"},
        "kernelB": {"dispatches": 1, "alg_bytes": 1e9, "note": "kernel B", "select": "last"},
        PROBE.replace("AUnaryFunctor", "[AB]UnaryFunctor"): {"dispatches": 2, "alg_bytes": 2 * 2 * gib,
                                                               "note": "copy probe"},
        "_sources": {"all": "a" * 16, "kernel": "b" * 16},
    }
    mp = tmp_path / "manifest.json"
    mp.write_text(json.dumps(man))
    seq = ([("void kernelA<0>(int)", 2_000_000)] * 3 + [("void kernelB(float)", 500_000)] * 2 +
           [("void " + PROBE + ">(int)", 400_000)] * 2)
    t0 = 1_000_000
    trace = []
    for i, (name, dur) in enumerate(seq):
        trace.append({"Dispatch_Id": i + 1, "Kernel_Name": name, "Start_Timestamp": t0, "End_Timestamp": t0 + dur})
        t0 += dur + 1000
    for d in ("trace", "fetch", "write"):
        _write_csv(str(tmp_path / d / "x_kernel_trace.csv"), trace)
    # counters (KiB per dispatch): kernel B's second dispatch differs from its first, so "last" is visible
    fetch = {"void kernelA<0>(int)": 1.5 * gib / 1024, "void kernelB(float)": 0.25 * gib / 1024,
             "void " + PROBE + ">(int)": gib / 2 / 1024}
    write = {"void kernelA<0>(int)": gib / 1024, "void kernelB(float)": 0.125 * gib / 1024,
             "void " + PROBE + ">(int)": gib / 1024}
    for d, vals, cname in (("fetch", fetch, "FETCH_SIZE"), ("write", write, "WRITE_SIZE")):
        rows = []
        seen_b = 0
        for i, (name, _) in enumerate(seq):
            v = vals[name]
            if "kernelB" in name:
                seen_b += 1
                v = v * seen_b       # the last dispatch of B counts twice its first
            rows.append({"Dispatch_Id": i + 1, "Kernel_Name": name, "Counter_Name": cname, "Counter_Value": v})
        _write_csv(str(tmp_path / d / "x_counter_collection.csv"), rows)
    return mp


def _table(md):
    rows = {}
    for line in md.splitlines():
        c = [x.strip() for x in line.split("|")]
        if len(c) > 11 and c[1].startswith("`"):
            rows[c[1].strip("`")] = c
    return rows


def test_suite_join_calibration_and_rows(tmp_path):
    mp = _suite(tmp_path)
    out = tmp_path / "summary.md"
    bench.summarize_profile(str(mp), str(tmp_path / "trace"), str(tmp_path / "fetch"), str(tmp_path / "write"),
                            str(out), "cmd")
    md = out.read_text()
    assert "FETCH_SIZE x 2.000 and WRITE_SIZE x 1.000" in md
    rows = _table(md)
    a = rows["kernelA<0>"]
    assert a[3] == "3 (expected 3)"
    assert float(a[4]) == pytest.approx(2000.0)              # avg us
    assert float(a[5]) == pytest.approx(4.0)                 # alg GB per launch
    assert float(a[6]) == pytest.approx(2000.0, rel=1e-3)    # alg GB/s
    gib = 1 << 30
    assert float(a[8]) == pytest.approx(3 * gib / 1e9, rel=1e-3)   # read: 1.5 GiB x 2
    assert float(a[9]) == pytest.approx(gib / 1e9, rel=1e-3)       # write: 1 GiB x 1
    assert float(a[11]) == pytest.approx((4 * gib / 1e9) / 4.0, rel=1e-2)
    b = rows["kernelB"]                                       # select "last": the second dispatch
    assert float(b[8]) == pytest.approx(2 * 0.25 * gib * 2 / 1e9, rel=1e-3)
    assert md.rstrip().endswith("kernel_source_sha256_16: " + "b" * 16)


def test_headline_summary_takes_the_timed_dispatches(tmp_path):
    kern = "wd::dslash_column_kernel<0, false, 1>"
    # 4 autotuning dispatches of 9 ms, then warmup 1 + steps 3 timed dispatches of 2.5 ms
    trace, stats, t0 = [], [], 0
    for i, dur in enumerate([9_000_000] * 4 + [2_500_000] * 4):
        trace.append({"Dispatch_Id": i + 1, "Kernel_Name": f"void {kern}(wd::ChunkTable<1>, int)",
                      "Start_Timestamp": t0, "End_Timestamp": t0 + dur})
        t0 += dur
    _write_csv(str(tmp_path / "tr" / "x_kernel_trace.csv"), trace)
    _write_csv(str(tmp_path / "tr" / "x_kernel_stats.csv"),
               [{"Name": f"void {kern}(wd::ChunkTable<1>, int)", "Calls": 8, "TotalDurationNs": 46_000_000,
                 "AverageNs": 5_750_000, "Percentage": 100.0, "MinNs": 2_500_000, "MaxNs": 9_000_000,
                 "StdDev": 0.0}])
    line = {"steps": 3, "warmup": 1, "roofline": {"kernel": kern, "alg_bytes_per_site": 1216,
                                                  "alg_bytes_per_launch": 1216 * 1000},
            "config": {"sites": 1000}, "extra": {"f64": {"launch": {"order": 3}}}}
    log = tmp_path / "b.log"
    log.write_text("[bench] FP64: 2.5000 ms/apply, 400.0 apps/s\n" + json.dumps(line) + "\n")
    out = tmp_path / "h.md"
    bench.summarize_headline(str(tmp_path / "tr"), str(log), str(out), "cmd")
    md = out.read_text()
    assert "the last 4 of 8" in md and "average 2500.0 us" in md
    assert f"kernel_source_sha256_16: {bench.kernel_hash()}" in md


def test_committed_summaries_match_their_own_format():
    """The committed kernel-suite summary parses into rows; when its hashes match the sources, the bench's
    lookups return the FP64 stencil's counted bytes."""
    path = os.path.join(bench.ROOT, bench.KERNELS_PROFILE)
    md = open(path).read()
    rows = _table(md)
    assert "dslash_column_kernel<0, false, 1>" in rows
    if f"kernel_source_sha256_16: {bench.kernel_hash()}" in md:
        t = bench.traffic_from_profile()
        r = rows["dslash_column_kernel<0, false, 1>"]
        assert t == pytest.approx((float(r[8]) + float(r[9])) * 1e9)
    if f"sources_sha256_16: {bench.all_sources_hash()}" in md:
        assert "dslash_column_kernel<0, false, 1>" in bench.kernel_profile_rows()


def test_solve_summary_takes_the_marked_window(tmp_path):
    """Dispatches before the second-to-last FP32 stencil marker (operator setup, autotuning, an earlier marker)
    and after the last one are left out; the window's kernels are summed per role."""
    seq = [("void wd::dslash_column_kernel<1, false, 1>(wd::ChunkTable<1>, int)", 5_000),     # autotune-time marker
           ("void wd::parity_kernel<2, false, 0, true, true, 2, 4>(wd::ParityTable)", 7_000),  # before the window
           ("void wd::dslash_column_kernel<1, false, 1>(wd::ChunkTable<1>, int)", 5_000),     # first marker
           ("void wd::(anonymous namespace)::parity_kernel<2, false, 0, true, true, 2, 4>(wd::(anonymous namespace)::ParityTable)", 3_000),
           ("void wd::parity_kernel<2, false, 2, true, false, 2, 4>(wd::ParityTable)", 3_000),
           ("void wd::parity_column_kernel<0, false, 0, true, true, 2, 2, 4>(wd::ParityTable)", 6_000),
           ("void wd::k_site_mdot<2>(int)", 2_000),
           ("void wd::k_mdot_all<double2, 8>(int)", 1_000),
           ("void wd::dslash_column_kernel<0, false, 1>(wd::ChunkTable<1>, int)", 4_000),
           ("void other_kernel(int)", 1_000),
           ("void wd::dslash_column_kernel<1, false, 1>(wd::ChunkTable<1>, int)", 5_000)]     # last marker
    trace, t0 = [], 0
    for i, (name, dur) in enumerate(seq):
        dur *= 1000                                             # microseconds -> milliseconds
        trace.append({"Dispatch_Id": i + 1, "Kernel_Name": name, "Start_Timestamp": t0, "End_Timestamp": t0 + dur})
        t0 += dur + 1_000
    _write_csv(str(tmp_path / "tr" / "x_kernel_trace.csv"), trace)
    log = tmp_path / "s.log"
    log.write_text("[bench] solve-profile: mixed on S, 12 RHS in waves of 4: 1.000 s, 120 outer applications of S, "
                   "708 FP16S ones\n")
    out = tmp_path / "s.md"
    bench.summarize_solve(str(tmp_path / "tr"), str(log), str(out), "cmd")
    md = out.read_text()
    roles = {}
    for line in md.splitlines():
        c = [x.strip() for x in line.split("|")]
        if len(c) == 5 and c[2].replace(".", "").isdigit() and c[3].endswith("%"):
            roles[c[1]] = float(c[2])
    assert "7 dispatches" in md
    assert roles["FP16S S, inner GMRES (parity kernels)"] == pytest.approx(6e-3)
    assert roles["FP64 parity kernels: outer S, prepare, reconstruct, true residual"] == pytest.approx(6e-3)
    assert roles["inner vector kernels (FP16S basis)"] == pytest.approx(2e-3)
    assert roles["outer vector kernels (FP64 basis)"] == pytest.approx(1e-3)
    assert roles["other"] == pytest.approx(5e-3)         # the FP64 full-lattice stencil is no role of this solve
    assert "| `wd::parity_kernel<2, false, 0, true, true, 2, 4>` | 1 |" in md
