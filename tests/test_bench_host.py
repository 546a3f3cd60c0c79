"""Host logic of bench.py that needs no GPU: the HBM-traffic figure from
counter runs, the kernel-trace summaries, and the refusal of more than one
GPU."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

STEP = "void lf::(anonymous namespace)::k_step<false>(lf::StepArgs)"
TYPED = "void lf::(anonymous namespace)::k_step<true>(lf::StepArgs)"
COPY = "__amd_rocclr_copyBuffer"


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def _counters(d, counter, per_kernel, grid=None):
    """per_kernel: name -> values, or name -> [(grid size, value), ...]."""
    rows = []
    for name, values in per_kernel.items():
        for v in values:
            g, v = v if isinstance(v, tuple) else (grid or bench._c3_step_grid(), v)
            rows.append([name, g, counter, v])
    _write(os.path.join(d, "run_counter_collection.csv"),
           ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"], rows)


def test_counter_summary_scales_by_the_copy_probe(tmp_path):
    """FETCH_SIZE and WRITE_SIZE of the scalar step kernel only (not the
    typed instance, and only its launches over the C3 mesh), each scaled so
    that the copy probe reads its known size."""
    kib = 1024
    other = bench._c3_step_grid(7)  # launches on another mesh do not count
    _counters(tmp_path / "f", "FETCH_SIZE",
              {STEP: [100.0, 300.0, (other, 7e9)], TYPED: [9e9]})
    _counters(tmp_path / "w", "WRITE_SIZE", {STEP: [50.0, 50.0, (other, 7e9)]})
    probe_mib = 1
    _counters(tmp_path / "cf", "FETCH_SIZE", {COPY: [512.0]})  # half of 1 MiB: scale 2
    _counters(tmp_path / "cw", "WRITE_SIZE", {COPY: [1024.0]})  # scale 1
    out = tmp_path / "c.json"
    bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                             str(tmp_path / "cw"), probe_mib, str(out))
    d = json.load(open(out))
    assert d["launches"] == [2, 2]
    assert d["fetch_scale"] == 2.0 and d["write_scale"] == 1.0
    assert d["hbm_read_bytes_per_launch"] == 200.0 * kib * 2.0
    assert d["hbm_write_bytes_per_launch"] == 50.0 * kib
    assert d["hbm_bytes_per_launch"] == 200.0 * kib * 2.0 + 50.0 * kib
    assert d["kernel_src_sha"] == bench.kernel_source_sha()


def _bench_line(step_us):
    return json.dumps({"metric": bench.METRIC, "config": {"step_kernel_us": step_us}})


def test_trace_summaries(tmp_path):
    """The step kernel's line and the agreement sentence; the post-processing
    of the last job split at its first dual-mesh kernel (with the fills
    before it), ending before the first library kernel."""
    tr = tmp_path / "trace"
    _write(str(tr / "run_kernel_stats.csv"),
           ["Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage"],
           [[STEP, 8000, 97900, 95700, 106700, 94.4],
            ["void lf::k_lloyd_accum(int)", 4, 2129000, 2124000, 2135000, 1.0]])
    seq = ["k_step<false>", "k_lloyd_accum", "k_lloyd_hits",  # an earlier job
           "k_step<false>", "k_lloyd_accum", "k_lloyd_hits", "k_lloyd_hits",
           "k_fill64", "k_dual_pairs", "k_bitonic", "k_bitonic", "k_orient_level",
           "at::native::fill", "k_copy_probe"]
    rows, t = [], 0
    for n in seq:
        name = n if n.startswith("at::") else f"void lf::{n}(int)"
        rows.append([name, t, t + 1000])
        t += 2000
    _write(str(tr / "run_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           rows)
    (tmp_path / "plain.json").write_text("log line\n" + _bench_line(98.7) + "\n")
    (tmp_path / "traced.json").write_text(_bench_line(102.5) + "\n")
    out = tmp_path / "out"
    out.mkdir()
    bench.summarize_trace(str(tr), str(tmp_path / "plain.json"), str(tmp_path / "traced.json"),
                          str(out))
    step = (out / "k_step_c3_trace.md").read_text()
    assert "| k_step<false> | 8000 | 97.9 | 95.7 | 106.7 | 94.40% |" in step
    assert "(97.9 us over 8000 launches)" in step and "102.5 us" in step and "98.7 us" in step
    post = (out / "post_c3_trace.md").read_text()
    assert "## Lloyd re-seed: 3 launches, 0.00 ms" in post
    assert "## dual mesh: 5 launches" in post
    assert "| k_lloyd_hits | 2 | 2.0 |" in post
    assert "k_fill64 | 1 |" in post.split("## dual mesh")[1]
    assert "at::native" not in post and "k_copy_probe" not in post


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_instruction_summary(tmp_path):
    """Per-wavefront counts over the last dispatches of the scalar step
    kernel, and the VALU issue time they imply."""
    d = tmp_path / "sq"
    rows = []
    for waves in [10.0, 40968.0, 40968.0]:  # the first is not among the last 2
        for name, v in [("SQ_WAVES", waves), ("SQ_INSTS_VALU", 1000.0 * waves),
                        ("SQ_INSTS_SALU", 500.0 * waves), ("SQ_INSTS_BRANCH", 300.0 * waves),
                        ("SQ_THREAD_CYCLES_VALU", 0.5 * 64 * 1000.0 * waves),
                        ("SQ_ACTIVE_INST_VALU", 1010.0 * waves), ("SQ_WAVE_CYCLES", 6000.0 * waves),
                        ("SQ_WAIT_INST_ANY", 1400.0 * waves)]:
            rows.append([STEP, name, v])
            rows.append([TYPED, name, 7 * v])
    _write(str(d / "run_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"],
           rows)
    out = tmp_path / "instr.md"
    bench.summarize_instructions(str(d), str(out), last=2)
    text = out.read_text()
    assert "| VALU instructions | 1,000 |" in text and "| SALU instructions | 500 |" in text
    assert "| active lanes per VALU instruction | 50.0% |" in text
    assert "| wavefront lifetime (SQ_WAVE_CYCLES, 4-cycle units) | 6,000 |" in text
    issue = 1000 * 40968 * 4 / 1024 / 2400
    assert f"= {issue:.1f} us per launch" in text


def test_cpu_baseline_legs():
    """The CPU baseline's three legs (one thread, every thread, one batch mesh
    per thread) on a small mesh and a small batch, with a tiny time budget."""
    import numpy as np
    from paper_1804_09152_amd import inputs as I
    mesh, seeds = I.config_c2(level=3, n_seeds=16, seed=1)
    items = I.batch_tori(4, nv_hi=2e3, s_hi=16)
    out = bench.cpu_baseline(mesh, seeds, 0.2, items, max_steps=8)
    assert out["kind"] == "oracle" and out["cores"] >= 1 and out["value"] > 0
    assert out["single_thread"]["cores"] == 1 and out["single_thread"]["value"] > 0
    b = out["batch_one_mesh_per_thread"]
    assert b["value"] > 0 and b["cores"] == out["cores"]


def test_batch_summary(tmp_path):
    """Per-vertex comparison of the batched and the single-mesh step: each
    mesh's launches picked by grid size, the wide-row kernel right after a
    step launch added to it, counters per wavefront, bytes scaled as the
    committed copy-probe factors."""
    WIDE = "void lf::(anonymous namespace)::k_wide<false>(lf::StepArgs)"
    g3, g4 = bench._grid_of(1000), bench._grid_of(4000)
    stats = {"entries_per_row": 1.4, "layers_per_neighbourhood": 2.0, "overflow_rows": 10,
             "rows_reading_overflow": 70, "neighbourhood_hist_1_to_8_9plus": [5, 4, 1, 0, 0, 0, 0, 0, 0]}
    probe = {"c3": {"grid": g3, "n_v": 1000, "cells": 10, **stats},
             "c4": {"grid": g4, "n_v": 4000, "cells": 50, **dict(stats, overflow_rows=80)}}
    (tmp_path / "probe.json").write_text("log line\n" + json.dumps(probe) + "\n")
    # trace: C3 launches of 10 us; C4 launches of 30 us, each followed by a 5 us k_wide
    rows, t = [], 0
    for name, grid, dur in [(STEP, g3, 10), (STEP, g3, 10), (STEP, g4, 30), (WIDE, 64 * 2048, 5),
                            (STEP, g4, 30), (WIDE, 64 * 2048, 5)]:
        rows.append([name, grid, t, t + dur * 1000])
        t += 100000
    _write(str(tmp_path / "t" / "run_kernel_trace.csv"),
           ["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"], rows)
    for d, counters in (("s", {"SQ_WAVES": 2.0, "SQ_INSTS_VALU": 2000.0, "SQ_INSTS_SALU": 1000.0}),
                        ("f", {"FETCH_SIZE": 100.0}), ("w", {"WRITE_SIZE": 50.0})):
        _write(str(tmp_path / d / "run_counter_collection.csv"),
               ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"],
               [[STEP, g, k, v * (1 if g == g3 else 4)] for g in (g3, g4) for k, v in counters.items()])
    out = tmp_path / "b.md"
    bench.summarize_batch(str(tmp_path / "probe.json"), str(tmp_path / "s"), str(tmp_path / "t"),
                          str(tmp_path / "f"), str(tmp_path / "w"), str(out))
    text = out.read_text()
    assert "| step (us; of which k_wide, the rows touching more than 8 layers) | 10.0 (0.0) | 35.0 (5.0) |" in text
    assert "| us per million vertices | 10000.0 | 8750.0 |" in text
    assert "| VALU instructions per wavefront | 1,000 | 1,000 |" in text
    cal = json.load(open(os.path.join(bench.ROOT, "profiles", "k_step_c3_counters.json")))
    b3 = (100 * 1024 * cal["fetch_scale"] + 50 * 1024 * cal["write_scale"]) / 1000
    assert f"| HBM bytes per vertex | {b3:.0f} | {b3:.0f} |" in text
    assert "hold 2.0 times more overflow rows per vertex" in text
