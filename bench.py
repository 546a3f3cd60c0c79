#!/usr/bin/env python3
"""Benchmark of the layered-field hot path on one MI355X.

Workload (one bench "step" = one whole job; the single-mesh roofline
configuration): icosphere level 9 (2,621,442
vertices, 5,242,880 triangles) radially displaced by 8 random real spherical
harmonics (max amplitude 0.2), cotangent operator, 16,384 seeds; the fields
are initialised from the seeds, advanced by 2,000 explicit Euler steps,
labelled, re-seeded once (Lloyd) and turned into a dual mesh.  Inputs are
resident in HBM before the timed region.

Prints one JSON line: field nnz-updates/s (sum over steps of the rows-of-
interest sizes divided by wall time), the step kernel's roofline (algorithmic
bytes per launch over its event-timed duration, against 8 TB/s), and the
FP64 CPU oracle timed on a bounded sample of the same job.  More objects
in the same line:

* "copy_roof": a measured 1 GiB device-to-device copy (read + write bytes
  over time), the practical HBM roof, and the step's achieved bandwidth as a
  fraction of it.
* "c2": jittered icosphere level 7 (163,842 vertices), 1,024 seeds,
  cotangent operator, 1,000 steps + 5 Lloyd rounds + labels + dual mesh.
* "typed": the same mesh and seeds with per-pair coefficients over 1, 8 and
  64 layer types; mean step-kernel time of each against the scalar step.
* "batch": 256 torus grids of uneven size (vertex counts log-uniform in
  [1e3, 1e5], seed counts log-uniform in [8, 512]), graph operator, 500 steps
  + labels each, advanced as one batch and, on the same GPU, one mesh at a
  time; nnz-updates/s of both.
* "serving": a Poisson stream of tessellation jobs on jittered icospheres of
  levels 5-9 (64 * 4^(level-5) seeds, cotangent operator, 1,000 steps + 3
  Lloyd rounds + labels + dual mesh each) through the continuous-batching
  server; p50/p99 latency from arrival to results in host memory, jobs/s.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "field nnz-updates/sec and % HBM peak per step; p50/p99 job latency batched"
# The step kernel is timed with start/stop events on every TIMING_EVERY-th
# launch of the timed region (events cost a few microseconds of wall time
# per timed launch); 17 is prime to the 256-step chunks, so the sampled
# launches cycle through every position of a chunk.
TIMING_EVERY = 17


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for name in ("lf_step.hip", "lf_internal.h"):
        with open(os.path.join(ROOT, "paper_1804_09152_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(alg_bytes_per_launch: float):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary, or None when it was taken on other kernel sources."""
    p = os.path.join(ROOT, "profiles", "k_step_c3_counters.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_src_sha") != kernel_source_sha():
        return None
    return d.get("hbm_bytes_per_launch")


def _counter_means(d: str, kernel: str, grid: int = 0):
    """Mean per dispatch of each counter of `kernel` in a rocprofv3 CSV folder
    (only the dispatches of that grid size, when grid > 0)."""
    import csv
    import glob
    acc = {}
    for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(fn)):
            if kernel in r["Kernel_Name"] and (grid <= 0 or int(r["Grid_Size"]) == grid):
                acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}


def _c3_step_grid(level: int = 9) -> int:
    """Threads in one step-kernel launch on the C3 mesh (64-row slices, the
    slice count rounded up to a multiple of 8 dies)."""
    n_v = 10 * 4 ** level + 2
    slices = (n_v + 63) // 64
    return 64 * 8 * ((slices + 7) // 8)


def summarize_counters(fetch_dir, write_dir, copyf_dir, copyw_dir, probe_mib, out_path):
    """HBM bytes per step-kernel launch from FETCH_SIZE / WRITE_SIZE runs,
    each scaled by what the same counter reads for a device copy of known
    size (the copy probe of this script)."""
    probe = probe_mib * (1 << 20)
    cf, _ = _counter_means(copyf_dir, "copyBuffer")
    cw, _ = _counter_means(copyw_dir, "copyBuffer")
    kf, nf = _counter_means(fetch_dir, "k_step<false>", _c3_step_grid())
    kw, nw = _counter_means(write_dir, "k_step<false>", _c3_step_grid())
    f_scale = probe / (cf["FETCH_SIZE"] * 1024)
    w_scale = probe / (cw["WRITE_SIZE"] * 1024)
    fetch = kf["FETCH_SIZE"] * 1024 * f_scale
    write = kw["WRITE_SIZE"] * 1024 * w_scale
    d = {"kernel": "k_step", "kernel_src_sha": kernel_source_sha(),
         "fetch_size_kib_per_launch": kf["FETCH_SIZE"], "write_size_kib_per_launch": kw["WRITE_SIZE"],
         "launches": [nf["FETCH_SIZE"], nw["WRITE_SIZE"]],
         "copy_probe_bytes": probe, "fetch_scale": f_scale, "write_scale": w_scale,
         "hbm_read_bytes_per_launch": fetch, "hbm_write_bytes_per_launch": write,
         "hbm_bytes_per_launch": fetch + write}
    with open(out_path, "w") as fh:
        json.dump(d, fh, indent=1)
    md = os.path.splitext(out_path)[0] + ".md"
    if os.path.exists(md):  # the per-launch table of the summary next to it
        text = open(md).read()
        i, j = text.index("Calibration:"), text.index("| algorithmic bytes")
        table = (f"Calibration: a {probe_mib // 1024} GiB device-to-device copy reads FETCH_SIZE = "
                 f"{cf['FETCH_SIZE']:,.0f} KiB and WRITE_SIZE =\n{cw['WRITE_SIZE']:,.0f} KiB per "
                 f"dispatch, so FETCH_SIZE is scaled by {f_scale:.1f} and WRITE_SIZE by "
                 f"{w_scale:.1f}.\n\n"
                 "| per launch (mean of 2,000 steps of one job) | value |\n|---|---|\n"
                 f"| FETCH_SIZE | {d['fetch_size_kib_per_launch']:,.0f} KiB → "
                 f"{d['hbm_read_bytes_per_launch'] / 1e6:.0f} MB read |\n"
                 f"| WRITE_SIZE | {d['write_size_kib_per_launch']:,.0f} KiB → "
                 f"{d['hbm_write_bytes_per_launch'] / 1e6:.0f} MB written |\n"
                 f"| HBM traffic | {d['hbm_bytes_per_launch'] / 1e6:.0f} MB |\n")
        with open(md, "w") as fh:
            fh.write(text[:i] + table + text[j:])
    print(json.dumps(d))


def state_probe(level: int, seeds_n: int, warm: int, steps: int):
    """C3 job advanced `warm` steps from its seeds, then `steps` more (for
    per-dispatch counters of the step kernel in a mid-job state)."""
    import paper_1804_09152_amd as lfb
    from paper_1804_09152_amd import inputs as I
    import torch
    lfb.load()
    mesh, seeds = I.config_c3(level=level, n_seeds=seeds_n)
    ctx = lfb.Context(0)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, lfb.LF_OP_COTAN)
    f = lfb.Fields(m, seeds)
    f.step(warm)
    torch.cuda.synchronize()
    log(f"state probe: {warm} steps done")
    f.step(steps)
    torch.cuda.synchronize()
    log(f"state probe: {steps} more steps done")
    f.close()
    m.close()


def _row_stats(rp, col, faces, n_v, inline: int = 3):
    """Entries per row, layers per row neighbourhood (the row and its mesh
    neighbours: the slots the step's merge fills), and whether the
    neighbourhood holds a row longer than the `inline` entries a fixed-width
    row keeps (an overflow row) -- of one mesh's fields."""
    import numpy as np
    import scipy.sparse as sp
    F = np.asarray(faces, np.int64)
    r = np.concatenate([F[:, 0], F[:, 1], F[:, 2], F[:, 1], F[:, 2], F[:, 0], np.arange(n_v)])
    c = np.concatenate([F[:, 1], F[:, 2], F[:, 0], F[:, 0], F[:, 1], F[:, 2], np.arange(n_v)])
    A = sp.csr_matrix((np.ones(r.size, np.float32), (r, c)), shape=(n_v, n_v))
    ncol = int(col.max()) + 1 if col.size else 1
    U = sp.csr_matrix((np.ones(col.size, np.float32), col, rp), shape=(n_v, ncol))
    N = (A @ U).tocsr()
    nnz = np.diff(rp)
    reads_ovf = (A @ (nnz > inline).astype(np.float32)) > 0
    return nnz, np.diff(N.indptr), reads_ovf


def _state_stats(parts) -> dict:
    """Row statistics over (entries, layers per neighbourhood, reads an
    overflow row) arrays of one or more meshes."""
    import numpy as np
    nnz = np.concatenate([p[0] for p in parts])
    uni = np.concatenate([p[1] for p in parts])
    ovf = np.concatenate([p[2] for p in parts])
    return {"entries_per_row": float(nnz.mean()), "layers_per_neighbourhood": float(uni.mean()),
            "overflow_rows": int((nnz > 3).sum()), "rows_reading_overflow": int(ovf.sum()),
            "neighbourhood_hist_1_to_8_9plus": [int((uni == q).sum()) for q in range(1, 9)]
            + [int((uni >= 9).sum())]}


def _grid_of(n_rows: int) -> int:
    """Threads in one step-kernel launch over n_rows rows."""
    slices = (n_rows + 63) // 64
    return 64 * 8 * ((slices + 7) // 8)


def batch_probe(n_meshes: int, steps: int):
    """The C3 job at steps 1,000-1,000+steps and the C4 batch at steps
    250-250+steps (for per-dispatch counters of the step kernel on both), then
    the row statistics of both states on the host (one JSON line)."""
    import numpy as np
    import paper_1804_09152_amd as lfb
    from paper_1804_09152_amd import inputs as I
    import torch
    lfb.load()
    ctx = lfb.Context(0)
    out = {}
    mesh, seeds = I.config_c3()
    m = lfb.Mesh(ctx, mesh.V, mesh.F, lfb.LF_OP_COTAN)
    f = lfb.Fields(m, seeds)
    f.step(1000)
    torch.cuda.synchronize()
    f.step(steps)
    torch.cuda.synchronize()
    log("batch probe: C3 done")
    rp, col, _ = f.export()
    out["c3"] = {"grid": _grid_of(mesh.n_v), "n_v": int(mesh.n_v), "cells": int(seeds.size),
                 **_state_stats([_row_stats(rp, col, mesh.F, mesh.n_v)])}
    f.close()
    m.close()
    items = I.batch_tori(n_meshes)
    B = lfb.Batch(ctx, [(mm.V, mm.F) for mm, _ in items], lfb.LF_OP_GRAPH, [sd for _, sd in items])
    B.step(250)
    torch.cuda.synchronize()
    B.step(steps)
    torch.cuda.synchronize()
    log("batch probe: C4 done")
    parts = []
    for q, (mm, _) in enumerate(items):
        rp, col, _ = B.export(q)
        parts.append(_row_stats(rp, col, mm.F, mm.n_v))
    n_v = int(sum(mm.n_v for mm, _ in items))
    out["c4"] = {"grid": _grid_of(n_v), "n_v": n_v, "cells": int(sum(sd.size for _, sd in items)),
                 **_state_stats(parts)}
    B.close()
    print(json.dumps(out), flush=True)


def summarize_batch(probe_json: str, pmc_dir: str, trace_dir: str, fetch_dir: str, write_dir: str,
                    out_path: str, last: int = 10):
    """Per-vertex cost of the batched step against the single-mesh step, from
    the runs of batch_probe: kernel time (trace), instructions (SQ counters),
    HBM bytes (FETCH_SIZE x 2 + WRITE_SIZE, the copy-probe scale factors of
    k_step_c3_counters.json) and the row statistics."""
    import csv
    import glob
    probe = json.loads(open(probe_json).read().strip().splitlines()[-1])
    cal = json.load(open(os.path.join(ROOT, "profiles", "k_step_c3_counters.json")))

    def per_grid(d, grid):
        acc = {}
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(fn)):
                if "k_step<false>" in r["Kernel_Name"] and int(r["Grid_Size"]) == grid:
                    acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        return {k: sum(v[-last:]) / len(v[-last:]) for k, v in acc.items()}

    trace = sorted(csv.DictReader(open(os.path.join(trace_dir, "run_kernel_trace.csv"))),
                   key=lambda r: int(r["Start_Timestamp"]))

    def trace_us(grid):
        """Mean of the last launches of the step kernel over `grid` threads,
        and of the wide-row kernel launched right after each of them."""
        step, wide = [], []
        for q, r in enumerate(trace):
            if "k_step<false>" in r["Kernel_Name"] and int(r["Grid_Size_X"]) == grid:
                step.append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
                nxt = trace[q + 1] if q + 1 < len(trace) else None
                wide.append(int(nxt["End_Timestamp"]) - int(nxt["Start_Timestamp"])
                            if nxt is not None and "k_wide<false>" in nxt["Kernel_Name"] else 0)
        return (sum(step[-last:]) / len(step[-last:]) / 1e3,
                sum(wide[-last:]) / len(wide[-last:]) / 1e3)

    rows = {}
    for key in ("c3", "c4"):
        p = probe[key]
        g = p["grid"]
        sq, fe, wr = per_grid(pmc_dir, g), per_grid(fetch_dir, g), per_grid(write_dir, g)
        us_step, us_wide = trace_us(g)
        us = us_step + us_wide
        waves = sq["SQ_WAVES"]
        rows[key] = {
            "n_v": p["n_v"], "cells": p["cells"], "us": us, "us_wide": us_wide,
            "us_per_mv": us / (p["n_v"] / 1e6),
            "ovf": p["overflow_rows"], "reads_ovf": p["rows_reading_overflow"],
            "waves": waves, "valu": sq["SQ_INSTS_VALU"] / waves, "salu": sq["SQ_INSTS_SALU"] / waves,
            "valu_us": sq["SQ_INSTS_VALU"] * 4 / 1024 / 2.4e3,
            "bytes_per_v": (fe["FETCH_SIZE"] * 1024 * cal["fetch_scale"]
                            + wr["WRITE_SIZE"] * 1024 * cal["write_scale"]) / p["n_v"],
            "epr": p["entries_per_row"], "lpn": p["layers_per_neighbourhood"],
            "hist": p["neighbourhood_hist_1_to_8_9plus"]}
    c3, c4 = rows["c3"], rows["c4"]
    fr = lambda h: " / ".join(f"{100 * x / sum(h):.0f}%" for x in h)
    lines = [
        "# Step kernel per vertex: C4 batch against the C3 mesh", "",
        "Commands (one MI355X, from the repository root; each a run of its own):", "", "```",
        "cd /tmp && export TMPDIR=/tmp",
        "python3 <repo>/bench.py --batch-probe 10 > <probe.json>",
        "rocprofv3 --kernel-trace --output-format csv -d <t> -o run -- python3 <repo>/bench.py --batch-probe 10",
        "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU --output-format csv -d <s> -o run -- "
        "python3 <repo>/bench.py --batch-probe 10",
        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <f> -o run -- python3 <repo>/bench.py --batch-probe 10",
        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <w> -o run -- python3 <repo>/bench.py --batch-probe 10",
        "python3 <repo>/bench.py --batch-summary <probe.json> <s> <t> <f> <w>",
        "```", "",
        "C3: icosphere level 9, 16,384 seeds, cotangent operator, steps 1,000-1,010.  C4: 256 torus",
        "grids (vertices and seeds log-uniform), graph operator, one batch, steps 250-260.  Means over",
        f"the last {last} dispatches of each; HBM bytes scaled as in k_step_c3_counters.md.", "",
        "| per launch | C3 | C4 batch |", "|---|---|---|",
        f"| vertices | {c3['n_v']:,} | {c4['n_v']:,} |",
        f"| cells (vertices per cell) | {c3['cells']:,} ({c3['n_v'] / c3['cells']:.0f}) | "
        f"{c4['cells']:,} ({c4['n_v'] / c4['cells']:.0f}) |",
        f"| step (us; of which k_wide, the rows touching more than 8 layers) | {c3['us']:.1f} "
        f"({c3['us_wide']:.1f}) | {c4['us']:.1f} ({c4['us_wide']:.1f}) |",
        f"| us per million vertices | {c3['us_per_mv']:.1f} | {c4['us_per_mv']:.1f} |",
        f"| entries of U per row | {c3['epr']:.2f} | {c4['epr']:.2f} |",
        f"| layers per row neighbourhood (mean) | {c3['lpn']:.2f} | {c4['lpn']:.2f} |",
        f"| rows whose neighbourhood holds 1 / 2 / ... / 8 / 9+ layers | {fr(c3['hist'])} | "
        f"{fr(c4['hist'])} |",
        f"| rows whose neighbourhood holds 9+ layers (stepped by k_wide) | {c3['hist'][-1]:,} | "
        f"{c4['hist'][-1]:,} |",
        f"| overflow rows (more than 3 entries) / rows reading one | {c3['ovf']:,} / "
        f"{c3['reads_ovf']:,} | {c4['ovf']:,} / {c4['reads_ovf']:,} |",
        f"| VALU instructions per wavefront | {c3['valu']:,.0f} | {c4['valu']:,.0f} |",
        f"| SALU instructions per wavefront | {c3['salu']:,.0f} | {c4['salu']:,.0f} |",
        f"| VALU issue (us; 4 cycles, 1,024 SIMDs, 2.4 GHz) | {c3['valu_us']:.1f} | {c4['valu_us']:.1f} |",
        f"| HBM bytes per vertex | {c3['bytes_per_v']:.0f} | {c4['bytes_per_v']:.0f} |", "",
        f"Per vertex the batched step costs {c4['us_per_mv'] / c3['us_per_mv']:.2f} times the C3 "
        f"step.  Its wavefronts issue {c4['valu'] / c3['valu']:.2f} times the VALU instructions",
        f"and move {c4['bytes_per_v'] / c3['bytes_per_v']:.2f} times the HBM bytes per vertex; VALU "
        f"issue is {100 * c3['valu_us'] / c3['us']:.0f}% of the C3 step and "
        f"{100 * c4['valu_us'] / (c4['us'] - c4['us_wide']):.0f}% of the batched step kernel.",
        f"The difference is latency: k_wide ({100 * c4['us_wide'] / c4['us']:.0f}% of the batched "
        "step) runs one wavefront per row whose",
        "neighbourhood holds 9+ layers, a chain of dependent loads, and the batch's small meshes "
        "with many seeds",
        f"hold {c4['ovf'] / c4['n_v'] / (c3['ovf'] / c3['n_v']):.1f} times more overflow rows per "
        "vertex (a row reading one waits one more dependent load round).", ""]
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines))
    print(json.dumps(rows))


def summarize_instructions(pmc_dir: str, out_path: str, last: int = 10):
    """Per-wavefront instruction counts of the step kernel over its last
    `last` dispatches, and the VALU issue time they imply."""
    import collections
    import csv
    import glob
    per = collections.defaultdict(list)
    for fn in glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(fn)):
            if "k_step<false>" in r["Kernel_Name"]:
                per[r["Counter_Name"]].append(float(r["Counter_Value"]))
    m = {k: sum(v[-last:]) / len(v[-last:]) for k, v in per.items()}
    waves = m["SQ_WAVES"]
    valu, salu = m["SQ_INSTS_VALU"] / waves, m["SQ_INSTS_SALU"] / waves
    lanes = m["SQ_THREAD_CYCLES_VALU"] / (m["SQ_INSTS_VALU"] * 64)
    simds, ghz = 1024, 2.4
    issue_us = valu * waves * 4 / simds / (ghz * 1e3)
    lines = ["# Instructions of the step kernel: C3 job, mid-job state", "",
             "Commands (one MI355X, from the repository root):", "", "```",
             "cd /tmp && export TMPDIR=/tmp",
             "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_THREAD_CYCLES_VALU "
             "SQ_INSTS_BRANCH SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VALU SQ_WAVE_CYCLES \\",
             "    --output-format csv -d <out> -o run -- python3 <repo>/bench.py --state-probe 10",
             "python3 <repo>/bench.py --instr-summary <out>",
             "```", "",
             f"Step 1,000 to 1,010 of the C3 job (icosphere level 9, 16,384 seeds); means over "
             f"the last {last} dispatches.", "",
             "| per wavefront | value |", "|---|---|",
             f"| wavefronts per launch | {waves:,.0f} |",
             f"| VALU instructions | {valu:,.0f} |",
             f"| SALU instructions | {salu:,.0f} |",
             f"| branch instructions | {m['SQ_INSTS_BRANCH'] / waves:,.0f} |",
             f"| active lanes per VALU instruction | {lanes:.1%} |", "",
             f"| VALU busy (SQ_ACTIVE_INST_VALU, 4-cycle units) | {m['SQ_ACTIVE_INST_VALU'] / waves:,.0f} |",
             f"| wavefront lifetime (SQ_WAVE_CYCLES, 4-cycle units) | {m['SQ_WAVE_CYCLES'] / waves:,.0f} |",
             f"| waiting on an instruction's issue (SQ_WAIT_INST_ANY) | {m['SQ_WAIT_INST_ANY'] / waves:,.0f} |",
             "",
             f"VALU issue: {valu:,.0f} instructions x {waves:,.0f} wavefronts x 4 cycles / "
             f"{simds:,} SIMDs / {ghz} GHz = {issue_us:.1f} us per launch; the step's time is in "
             "k_step_c3_trace.md.", ""]
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines))
    print(json.dumps({"valu_per_wave": valu, "salu_per_wave": salu, "waves": waves,
                      "lanes": lanes, "valu_issue_us": issue_us}))


def _kname(name: str) -> str:
    import re
    m = re.search(r"(k_[A-Za-z0-9_]+(<[a-z]+>)?|__amd_rocclr_[A-Za-z]+)", name)
    return m.group(1) if m else name.split("(")[0][:40]


def summarize_trace(trace_dir: str, plain_json: str, traced_json: str, out_dir: str):
    """Writes the kernel-trace summaries of the C3 job (step kernel and the
    post-processing of the last job) from a rocprofv3 --kernel-trace --stats
    run of `bench.py --no-c2 --no-batch --no-graphs --no-serve --no-typed --no-cpu-baseline`, next
    to the bench lines of that run and of a plain run."""
    import collections
    import csv
    stats = list(csv.DictReader(open(os.path.join(trace_dir, "run_kernel_stats.csv"))))
    plain = json.loads(open(plain_json).read().strip().splitlines()[-1])
    traced = json.loads(open(traced_json).read().strip().splitlines()[-1])
    cmd = ["```", "cd /tmp && export TMPDIR=/tmp",
           "rocprofv3 --kernel-trace --stats --output-format csv -d <out> -o run -- \\",
           "    python3 <repo>/bench.py --no-c2 --no-batch --no-graphs --no-serve --no-typed "
           "--no-cpu-baseline",
           "python3 <repo>/bench.py --trace-summary <out> <plain bench line> <traced bench line>",
           "```"]
    lines = ["# Kernel trace: C3 job (bench.py C3 section)", "",
             "Commands (on one MI355X, from the repository root):", "", *cmd, "",
             "Workload: icosphere level 9 (2,621,442 vertices) displaced by 8 spherical harmonics, "
             "cotangent", "operator, 16,384 seeds; 1 warm-up + 3 timed jobs of 2,000 steps + "
             "labels + Lloyd + dual mesh.", "",
             "| kernel | calls | avg (us) | min (us) | max (us) | share |",
             "|---|---|---|---|---|---|"]
    for r in stats[:14]:
        lines.append(f"| {_kname(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f}% |")
    step = next(r for r in stats if "k_step<false>" in r["Name"])
    lines += ["", f"The step kernel's mean ({float(step['AverageNs']) / 1e3:.1f} us over "
              f"{step['Calls']} launches) agrees with the event-timed",
              f"`config.step_kernel_us` of the bench line of the same run "
              f"({traced['config']['step_kernel_us']:.1f} us under the",
              f"profiler) and of the plain bench run ({plain['config']['step_kernel_us']:.1f} us)."]
    with open(os.path.join(out_dir, "k_step_c3_trace.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    # the post-processing of the last timed job: from its Lloyd accumulation
    # to the last kernel of its dual mesh (before the copy-roof probe)
    rows = sorted(csv.DictReader(open(os.path.join(trace_dir, "run_kernel_trace.csv"))),
                  key=lambda r: int(r["Start_Timestamp"]))
    first = max(i for i, r in enumerate(rows) if _kname(r["Kernel_Name"]) == "k_lloyd_accum")
    seg = rows[first:]
    stop = next((i for i, r in enumerate(seg) if "at::native" in r["Kernel_Name"]), len(seg))
    seg = seg[:stop]
    while seg and not _kname(seg[-1]["Kernel_Name"]).startswith("k_"):
        seg.pop()
    d0 = next(i for i, r in enumerate(seg) if _kname(r["Kernel_Name"]) == "k_dual_pairs")
    while d0 > 0 and _kname(seg[d0 - 1]["Kernel_Name"]) in ("k_fill64",
                                                            "__amd_rocclr_fillBufferAligned"):
        d0 -= 1
    lines = ["# Kernel trace: post-processing of one C3 job (Lloyd re-seed, dual mesh)", "",
             "From the same run as `k_step_c3_trace.md` (commands there): the kernels after the "
             "last", "job's 2,000 steps, split at the first dual-mesh kernel; GPU kernel times.", ""]
    for title, part in (("Lloyd re-seed", seg[:d0]), ("dual mesh", seg[d0:])):
        busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in part)
        lines += [f"## {title}: {len(part)} launches, {busy / 1e6:.2f} ms of kernel time", "",
                  "| kernel | calls | total (us) |", "|---|---|---|"]
        agg = collections.defaultdict(lambda: [0, 0])
        for r in part:
            a = agg[_kname(r["Kernel_Name"])]
            a[0] += 1
            a[1] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        for n, (c, t) in sorted(agg.items(), key=lambda x: -x[1][1])[:14]:
            lines.append(f"| {n} | {c} | {t / 1e3:.1f} |")
        lines.append("")
    with open(os.path.join(out_dir, "post_c3_trace.md"), "w") as fh:
        fh.write("\n".join(lines))


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(mesh, seeds, seconds: float, batch_items=None, max_steps: int = 200):
    """The FP64 oracle on the host: the same job from its seeds on one thread
    and on every host thread (rows in blocks, identical results), and the
    batch workload with one mesh per thread.  Each leg stops at the first
    chunk that ends past `seconds`; rates are rows-of-interest entries per
    second of wall time (operator builds excluded)."""
    import threading

    import oracle
    oracle.build()
    threads = oracle.host_threads()
    P = oracle.default_params()
    log("cpu baseline: oracle operator")
    L = oracle.operator(mesh.V, mesh.F, 1)

    def single_mesh(th, chunk):
        U = oracle.init(mesh.n_v, seeds)
        skel, n = 0, 0
        t0 = time.perf_counter()
        while n < max_steps:
            U, info = oracle.run(L, U, seeds.size, P, chunk, threads=th)
            skel += info["skel_total"]
            n += chunk
            if time.perf_counter() - t0 >= seconds:
                break
        return skel, n, time.perf_counter() - t0

    sk1, n1, dt1 = single_mesh(1, 1)
    log(f"cpu baseline: one thread, {n1} steps in {dt1:.1f} s")
    skm, nm, dtm = single_mesh(threads, 4)
    log(f"cpu baseline: {threads} threads, {nm} steps in {dtm:.1f} s")
    out = {"value": skm / dtm, "unit": "nnz-updates/s", "cores": threads, "kind": "oracle",
           "sample": (f"first {nm} Euler steps of the same job from its seeds, FP64 C oracle, "
                      f"rows in {threads} blocks on {threads} threads (results identical to one "
                      f"thread), operator build excluded ({dtm:.1f} s)"),
           "single_thread": {"value": sk1 / dt1, "cores": 1,
                             "sample": f"first {n1} Euler steps, one thread ({dt1:.1f} s)"},
           "host_cpu": _cpu_model(), "host_threads": os.cpu_count()}
    if batch_items:
        # one mesh per thread: the batch's meshes in order, each its own
        # oracle run of `bsteps` steps, until the time is up
        bsteps = 50
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:  # operator builds, not timed
            ops = list(ex.map(lambda it: oracle.operator(it[0].V, it[0].F, 0), batch_items))
        lock = threading.Lock()
        state = {"next": 0, "skel": 0, "meshes": 0}
        t0 = time.perf_counter()

        def worker():
            while True:
                with lock:
                    k = state["next"]
                    if k >= len(batch_items) or time.perf_counter() - t0 >= seconds:
                        return
                    state["next"] = k + 1
                bm, bs = batch_items[k]
                _, info = oracle.run(ops[k], oracle.init(bm.n_v, bs), bs.size, P, bsteps)
                with lock:
                    state["skel"] += info["skel_total"]
                    state["meshes"] += 1

        ts = [threading.Thread(target=worker) for _ in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        dtb = time.perf_counter() - t0
        log(f"cpu baseline: batch, {state['meshes']} meshes x {bsteps} steps in {dtb:.1f} s")
        out["batch_one_mesh_per_thread"] = {
            "value": state["skel"] / dtb, "cores": threads,
            "sample": (f"the first {state['meshes']} meshes of the batch workload, {bsteps} Euler "
                       f"steps each from their seeds, one mesh per thread on {threads} threads, "
                       f"operator builds excluded ({dtb:.1f} s)")}
    return out


def copy_roof(mib: int = 1024, reps: int = 10):
    """Measured device-to-device copy bandwidth (read + write bytes / time),
    the practical HBM roof next to the vendor peak."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    b.synchronize()
    gbs = 2 * n * 4 * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del x, y
    return gbs


def run_c2(lfb, I, steps: int, rounds: int, jobs: int):
    """C2: jittered icosphere level 7 (163,842 vertices), 1,024 seeds,
    cotangent operator, `steps` steps + `rounds` x (Lloyd re-seed,
    re-initialise, `steps` steps) + labels + dual mesh, inputs resident."""
    import torch
    mesh, seeds = I.config_c2()
    ctx = lfb.Context(0)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, lfb.LF_OP_COTAN)
    f = lfb.Fields(m, seeds)
    dev = torch.device("cuda", 0)
    lab = torch.empty(mesh.n_v, dtype=torch.int32, device=dev)

    def job():
        f.reset(seeds)
        f.step(steps)
        for _ in range(rounds):
            s, _ = f.lloyd_reseed()
            f.reset(s)
            f.step(steps)
        lfb.lf_labels(f.h, lab)
        f.dual_mesh(0.25)

    job()  # warm-up
    torch.cuda.synchronize()
    sk0 = f.stats()["skeleton_total"]
    f.timing(TIMING_EVERY)
    t0 = time.perf_counter()
    for _ in range(jobs):
        job()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, n = f.timing(0)
    skel = f.stats()["skeleton_total"] - sk0
    f.close()
    m.close()
    log(f"c2: {wall / jobs * 1e3:.1f} ms per job")
    return {"workload": (f"jittered icosphere level 7 (163,842 vertices), 1024 seeds, cotangent "
                         f"operator, {steps} steps + {rounds} Lloyd rounds + labels + dual mesh"),
            "value": skel / wall, "unit": "nnz-updates/s", "ms_per_job": wall / jobs * 1e3,
            "jobs": jobs, "step_kernel_us": ms / max(n, 1) * 1e3}


def run_typed(lfb, m, seeds, type_counts=(1, 8, 64), warm: int = 200, timed: int = 400):
    """Per-pair coefficients on the C3 mesh: each layer draws one of T types
    (seeded), the T x T table is symmetric around the scalar defaults (a =
    0.04, w uniform in [0.15, 0.25], e = 1).  Mean step-kernel time (every
    launch event-timed) over `timed` steps after `warm` steps from the seeds,
    for the scalar step and each T."""
    import numpy as np
    res = {}
    for n_t in (0,) + tuple(type_counts):
        f = lfb.Fields(m, seeds)
        if n_t:
            rng = np.random.default_rng(n_t)
            tab = np.empty((n_t, n_t, 3))
            tab[..., 0] = 0.04
            tab[..., 1] = rng.uniform(0.15, 0.25, (n_t, n_t))
            tab[..., 2] = 1.0
            tab = 0.5 * (tab + tab.transpose(1, 0, 2))
            f.set_coefficients(rng.integers(0, n_t, seeds.size + 1).astype(np.int32), tab)
        f.step(warm)
        f.timing(1)
        f.step(timed)
        ms, n = f.timing(0)
        res[n_t] = ms / max(n, 1) * 1e3
        f.close()
    log("per-pair coefficients: " + ", ".join(f"T={t}: {v:.1f} us" for t, v in res.items()))
    return {"workload": (f"the C3 mesh and seeds, per-pair coefficients over T layer types, "
                         f"steps {warm}-{warm + timed} from the seeds"),
            "scalar_step_kernel_us": res[0],
            "step_kernel_us_by_types": {str(t): res[t] for t in type_counts}}


def run_batch(lfb, I, n_meshes: int, steps: int):
    import numpy as np
    import torch
    items = I.batch_tori(n_meshes)
    nv = [m.n_v for m, _ in items]
    log(f"batch: {n_meshes} meshes, {sum(nv)} vertices, {sum(s.size for _, s in items)} seeds")
    ctx = lfb.Context(0)
    dev = torch.device("cuda", 0)
    B = lfb.Batch(ctx, [(m.V, m.F) for m, _ in items], lfb.LF_OP_GRAPH, [s for _, s in items])
    lab = torch.empty(sum(nv), dtype=torch.int32, device=dev)
    # warm-up pass grows the storage to its working size, then the timed pass
    for rep in range(2):
        B.reset()
        sk0 = B.stats()["skeleton_total"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.step(steps)
        lfb.lf_labels(B.fh, lab)
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t0
        sk_b = B.stats()["skeleton_total"] - sk0
    B.close()
    log(f"batch: {t_b * 1e3:.1f} ms batched")
    solo = []
    for m, s in items:
        M = lfb.Mesh(ctx, m.V, m.F, lfb.LF_OP_GRAPH)
        solo.append((M, lfb.Fields(M, s),
                     torch.empty(m.n_v, dtype=torch.int32, device=dev)))
    for rep in range(2):
        sk0 = sum(f.stats()["skeleton_total"] for _, f, _ in solo)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _, f, lab1 in solo:
            f.reset(f.seeds())
            f.step(steps)
            lfb.lf_labels(f.h, lab1)
        torch.cuda.synchronize()
        t_s = time.perf_counter() - t0
        sk_s = sum(f.stats()["skeleton_total"] for _, f, _ in solo) - sk0
    log(f"batch: {t_s * 1e3:.1f} ms one mesh at a time")
    for M, f, _ in solo:
        f.close()
        M.close()
    return {
        "workload": (f"{n_meshes} torus grids, vertices log-uniform [1e3,1e5], seeds log-uniform "
                     f"[8,512], graph operator, {steps} steps + labels each"),
        "n_vertices": int(sum(nv)),
        "n_seeds": int(sum(s.size for _, s in items)),
        "batched_nnz_updates_per_s": sk_b / t_b,
        "batched_ms": t_b * 1e3,
        "one_at_a_time_nnz_updates_per_s": sk_s / t_s,
        "one_at_a_time_ms": t_s * 1e3,
        "speedup": t_s / t_b,
        "identical_work": bool(sk_b == sk_s),
    }


def run_graphs(lfb, I):
    """Step chunks launched one by one against chunks replayed from captured
    graphs: a jittered icosphere level 5 (10,242 vertices, 64 seeds) and
    level 7 (the c2 mesh), 1,024 steps each, and the 256-torus batch, 512
    steps; wall time of the step loop (results are identical)."""
    import torch
    ctx = lfb.Context(0)
    out = {"what": "wall ms of the step loop, launches one by one vs 256-step chunks from a graph"}

    def timed(fields, steps, reps=3):
        best = []
        for on in (False, True):
            fields.use_graphs(on)
            fields.step(256)  # captures (when on) and warms
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fields.step(steps)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            best.append(min(ts) * 1e3)
        fields.use_graphs(False)
        return {"launches_ms": best[0], "graphs_ms": best[1], "speedup": best[0] / best[1]}

    for lv, k in ((5, 64), (7, 1024)):
        mesh, seeds = I.config_c2(level=lv, n_seeds=k)
        m = lfb.Mesh(ctx, mesh.V, mesh.F, lfb.LF_OP_COTAN)
        f = lfb.Fields(m, seeds)
        out[f"icosphere{lv}_1024_steps"] = timed(f, 1024)
        log(f"graphs: icosphere {lv}: {out[f'icosphere{lv}_1024_steps']}")
        f.close()
        m.close()
    items = I.batch_tori(256)
    B = lfb.Batch(ctx, [(mm.V, mm.F) for mm, _ in items], lfb.LF_OP_GRAPH, [sd for _, sd in items])
    out["batch_512_steps"] = timed(B, 512, reps=2)
    log(f"graphs: batch: {out['batch_512_steps']}")
    B.close()
    return out


def _mono_ms() -> float:
    return time.clock_gettime(time.CLOCK_MONOTONIC) * 1e3


def run_serving(lfb, I, n_jobs: int, rates, steps: int, rounds: int, max_active: int,
                budget_gib: float, chunk: int = 64):
    """The serving stream at each offered rate, then the same jobs one at a
    time with the plain calls.  Latency runs from a job's Poisson arrival to
    its completion (the library's monotonic timestamps), so time the loop
    spends before submitting counts against the server."""
    import numpy as np
    jobs = I.serving_jobs(n_jobs, seed=0)
    base, inputs = {}, []
    for j in jobs:
        lv = j["level"]
        if lv not in base:
            base[lv] = I.icosphere(lv)
        rng = np.random.default_rng(j["seed"])
        m = I.jitter(base[lv], rng)
        inputs.append((m, I.seeds_uniform(m.n_v, j["n_seeds"], rng)))
    budget = int(budget_gib * (1 << 30))
    log(f"serving: {n_jobs} jobs, levels {np.bincount([j['level'] for j in jobs], minlength=10)[5:]}")
    S = lfb.Server(0, budget, max_active, chunk)
    wm, ws = inputs[0]  # one small job first: loads the kernels, warms the allocator
    w = S.submit(wm.V, wm.F, ws, 50, 1, True, lfb.LF_OP_COTAN)
    S.run()
    S.release(w)
    S.close()
    out = {"workload": (f"Poisson arrivals of {n_jobs} jobs, jittered icospheres levels 5-9, "
                        f"64*4^(level-5) seeds, cotangent operator, {steps} steps + {rounds} "
                        f"Lloyd rounds + labels + dual mesh each"),
           "max_active": max_active, "hbm_budget_gib": budget_gib, "steps_per_tick": chunk,
           "rates": []}
    for qps in rates:
        arrivals = np.cumsum(np.random.default_rng(1).exponential(1.0 / qps, n_jobs)) * 1e3
        S = lfb.Server(0, budget, max_active, chunk)
        ids = [None] * n_jobs
        t0 = _mono_ms()
        nxt, done = 0, 0
        while done < n_jobs:
            now = _mono_ms() - t0
            while nxt < n_jobs and arrivals[nxt] <= now:
                m, sd = inputs[nxt]
                ids[nxt] = S.submit(m.V, m.F, sd, steps, rounds, True, lfb.LF_OP_COTAN)
                nxt += 1
            q, a, done = S.poll()
            if q == 0 and a == 0 and nxt < n_jobs:
                time.sleep(max(0.0, min(1e-3, (arrivals[nxt] - (_mono_ms() - t0)) * 1e-3)))
        lat, qms, ends, nsteps = [], [], [], 0
        for k, i in enumerate(ids):
            r = S.result(i)
            sub, adm, fin = S.times(i)
            lat.append(fin - (t0 + arrivals[k]))
            qms.append(adm - (t0 + arrivals[k]))
            ends.append(fin - t0)
            nsteps += r["steps"]
            S.release(i)
        peak = S.memory()[1]
        ticks, launches = S.stats()
        S.close()
        lat = np.array(lat)
        wall = max(ends) * 1e-3
        log(f"serving at {qps} jobs/s: p50 {np.percentile(lat, 50):.1f} ms, "
            f"p99 {np.percentile(lat, 99):.1f} ms, {n_jobs / wall:.2f} jobs/s")
        out["rates"].append({
            "offered_jobs_per_s": qps, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_to_admission_ms": float(np.mean(qms)),
            "jobs_per_s": n_jobs / wall, "wall_s": wall, "euler_steps": int(nsteps),
            "peak_charged_gib": peak / (1 << 30), "ticks": ticks, "grouped_launches": launches,
            "arrivals_s": float(arrivals[-1] * 1e-3)})
    # one job at a time, back to back, with the plain calls (mesh, fields,
    # steps, Lloyd rounds, labels, dual mesh; results to host memory)
    ctx = lfb.Context(0)
    service = []
    for m, sd in inputs:
        t = _mono_ms()
        M = lfb.Mesh(ctx, m.V, m.F, lfb.LF_OP_COTAN)
        f = lfb.Fields(M, sd)
        f.step(steps)
        for _ in range(rounds):
            ns, _ = f.lloyd_reseed()
            f.reset(ns)
            f.step(steps)
        f.labels()
        f.seeds()
        f.dual_mesh(0.25)
        f.close()
        M.close()
        service.append(_mono_ms() - t)
    service = np.array(service)
    solo = {"jobs_per_s": n_jobs / (service.sum() * 1e-3), "mean_service_ms": float(service.mean())}
    # the same arrivals served first come first served by that one-at-a-time
    # solver (its measured service times)
    for r in out["rates"]:
        arrivals = np.cumsum(np.random.default_rng(1).exponential(1.0 / r["offered_jobs_per_s"],
                                                                 n_jobs)) * 1e3
        fin, lat = 0.0, []
        for a, sv in zip(arrivals, service):
            fin = max(fin, a) + sv
            lat.append(fin - a)
        r["one_at_a_time_p50_ms"] = float(np.percentile(lat, 50))
        r["one_at_a_time_p99_ms"] = float(np.percentile(lat, 99))
        r["one_at_a_time_jobs_per_s"] = n_jobs / (fin * 1e-3)
    out["one_at_a_time"] = solo
    log(f"serving: one at a time {solo['jobs_per_s']:.2f} jobs/s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed jobs")
    ap.add_argument("--warmup", type=int, default=1, help="untimed jobs")
    ap.add_argument("--euler-steps", type=int, default=2000)
    ap.add_argument("--level", type=int, default=9)
    ap.add_argument("--seeds", type=int, default=16384)
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-post", action="store_true", help="skip Lloyd and dual mesh")
    ap.add_argument("--batch-meshes", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--serve-jobs", type=int, default=200)
    ap.add_argument("--serve-qps", type=float, nargs="+", default=[4.0, 8.0])
    ap.add_argument("--serve-steps", type=int, default=1000)
    ap.add_argument("--serve-rounds", type=int, default=3)
    ap.add_argument("--serve-chunk", type=int, default=64, help="steps per job per server tick")
    ap.add_argument("--serve-active", type=int, default=16)
    ap.add_argument("--serve-budget-gib", type=float, default=4.0)
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-typed", action="store_true", help="skip the per-pair coefficient steps")
    ap.add_argument("--counters", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPYF_DIR", "COPYW_DIR"),
                    help="only summarize rocprofv3 FETCH_SIZE / WRITE_SIZE runs of the step "
                         "kernel and of the copy probe into profiles/k_step_c3_counters.json")
    ap.add_argument("--trace-summary", nargs=3, metavar=("TRACE_DIR", "PLAIN_JSON", "TRACE_JSON"),
                    help="only summarize a rocprofv3 kernel trace of the C3 section into "
                         "profiles/k_step_c3_trace.md and profiles/post_c3_trace.md")
    ap.add_argument("--state-probe", type=int, default=0, metavar="STEPS",
                    help="only advance the C3 job 1,000 steps, then STEPS more (for counters)")
    ap.add_argument("--batch-probe", type=int, default=0, metavar="STEPS",
                    help="only step the C3 job to 1,000 and the C4 batch to 250 steps, STEPS more "
                         "each (for counters), and print both states' row statistics")
    ap.add_argument("--batch-summary", nargs=5,
                    metavar=("PROBE_JSON", "PMC_DIR", "TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="only summarize the --batch-probe runs into profiles/k_step_c4_batch.md")
    ap.add_argument("--instr-summary", metavar="PMC_DIR",
                    help="only summarize a rocprofv3 SQ counter run of --state-probe into "
                         "profiles/k_step_c3_instructions.md")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB ten times (calibrates "
                         "the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.instr_summary:
        summarize_instructions(args.instr_summary,
                               os.path.join(ROOT, "profiles", "k_step_c3_instructions.md"))
        return
    if args.state_probe:
        state_probe(args.level, args.seeds, 1000, args.state_probe)
        return
    if args.batch_probe:
        batch_probe(args.batch_meshes, args.batch_probe)
        return
    if args.batch_summary:
        summarize_batch(*args.batch_summary,
                        out_path=os.path.join(ROOT, "profiles", "k_step_c4_batch.md"))
        return
    if args.trace_summary:
        summarize_trace(*args.trace_summary, out_dir=os.path.join(ROOT, "profiles"))
        return
    if args.counters:
        summarize_counters(*args.counters, probe_mib=1024,
                           out_path=os.path.join(ROOT, "profiles", "k_step_c3_counters.json"))
        return
    if args.copy_probe:
        import torch
        n = args.copy_probe * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(10):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": n * 4, "launches": 10}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; "
              "the step would shard by vertex rows with a one-ring halo exchange",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1804_09152_amd as lfb
    from paper_1804_09152_amd import inputs as I

    lfb.load()
    log("generating the mesh")
    mesh, seeds = I.config_c3(level=args.level, n_seeds=args.seeds)
    dev = torch.device("cuda", 0)
    ctx = lfb.Context(0)
    log("operator build")
    m = lfb.Mesh(ctx, mesh.V, mesh.F, lfb.LF_OP_COTAN)
    f = lfb.Fields(m, seeds)
    labels = torch.empty(mesh.n_v, dtype=torch.int32, device=dev)
    post = not args.no_post
    have_post = True

    def job():
        nonlocal have_post
        f.reset(seeds)
        f.step(args.euler_steps)
        lfb.lf_labels(f.h, labels)
        if post and have_post:
            try:
                f.lloyd_reseed()
                f.dual_mesh(0.25)
            except lfb.LFError as e:
                if e.status != 6:
                    raise
                have_post = False

    for w in range(args.warmup):
        log(f"warmup job {w}")
        job()
    torch.cuda.synchronize()
    st0 = f.stats()
    tin0, tout0 = f.traffic()
    f.timing(TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        log(f"timed job {k}")
        job()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_total, launches = f.timing(0)
    st1 = f.stats()
    tin1, tout1 = f.traffic()
    wall = t1 - t0
    skel = st1["skeleton_total"] - st0["skeleton_total"]
    n_v = mesh.n_v
    # the operator as CSR with its diagonal: 4 (n_v + 1) + 8 nnz(L)
    nnz_l = lfb.lf_mesh_operator(m.h)
    op_bytes = 4 * (n_v + 1) + 8 * nnz_l
    # per step: the operator, both row-pointer arrays, and the mean entries of
    # U_t and U_{t+1} over every step of the timed jobs
    steps_run = st1["steps"] - st0["steps"]
    per_launch_bytes = (op_bytes + 2 * 4 * (n_v + 1)
                        + 8 * ((tin1 - tin0) + (tout1 - tout0)) / max(steps_run, 1))
    avg_ms = ms_total / max(launches, 1)
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    traffic = traffic_from_profile(per_launch_bytes)
    out = {
        "metric": METRIC,
        "value": skel / wall,
        "unit": "nnz-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"icosphere level {args.level} displaced by 8 random spherical harmonics, "
                         f"cotangent operator, {args.seeds} seeds, {args.euler_steps} Euler steps"
                         + (" + labels + Lloyd re-seed + dual mesh" if (post and have_post)
                            else " + labels")),
            "n_vertices": n_v,
            "n_faces": mesh.n_f,
            "n_seeds": int(seeds.size),
            "euler_steps_per_job": args.euler_steps,
            "step_kernel_us": avg_ms * 1e3,
            "step_kernel_launches": steps_run,
            "step_kernel_launches_timed": launches,
            "mean_nnz_per_vertex": (tout1 - tout0) / max(steps_run, 1) / n_v,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
        },
    }
    f.close()
    roof = copy_roof()
    out["copy_roof"] = {"unit": "GB/s", "measured": roof, "frac_of_peak": roof / HBM_PEAK_GBS,
                        "step_achieved_frac": achieved / roof,
                        "what": "1 GiB device-to-device copy, read + write bytes"}
    log(f"copy roof: {roof:.0f} GB/s")
    if not args.no_typed:
        out["typed"] = run_typed(lfb, m, seeds)
    m.close()
    if not args.no_c2:
        out["c2"] = run_c2(lfb, I, 1000, 5, 3)
    if not args.no_batch:
        out["batch"] = run_batch(lfb, I, args.batch_meshes, args.batch_steps)
    if not args.no_graphs:
        out["graphs"] = run_graphs(lfb, I)
    if not args.no_serve:
        out["serving"] = run_serving(lfb, I, args.serve_jobs, args.serve_qps, args.serve_steps,
                                     args.serve_rounds, args.serve_active, args.serve_budget_gib,
                                     args.serve_chunk)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mesh, seeds, args.cpu_seconds,
                                           I.batch_tori(args.batch_meshes))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
