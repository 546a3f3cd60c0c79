"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np


def say(*a):
    """Print and flush before a GPU step so a failing run names its case."""
    print(*a, flush=True)
    sys.stdout.flush()


def f32(U):
    """Oracle CSR with values rounded to float32 (what the GPU receives)."""
    return (np.asarray(U[0], np.int64), np.asarray(U[1], np.int32),
            np.asarray(U[2], np.float32).astype(np.float64))


def gpu_load(fields, U):
    fields.load(np.asarray(U[0], np.int32), np.asarray(U[1], np.int32),
                np.asarray(U[2], np.float32))


def as_oracle(G):
    """GPU export (int32 ptr, int32 col, float32 val) -> oracle CSR triple."""
    return (np.asarray(G[0], np.int64), np.asarray(G[1], np.int32),
            np.asarray(G[2], np.float64))


def row_compare(G, O):
    """Row-wise comparison of two CSR triples with the same row count.
    Returns (pattern_equal[n_rows], max |dval| per row over equal-pattern rows)."""
    Pg, Cg, Vg = G
    Po, Co, Vo = O
    Pg = np.asarray(Pg, np.int64)
    Po = np.asarray(Po, np.int64)
    n = Pg.size - 1
    cg = np.diff(Pg)
    co = np.diff(Po)
    same = cg == co
    rows = np.nonzero(same)[0]
    lens = cg[rows]
    tot = int(lens.sum())
    start = np.cumsum(lens) - lens
    within = np.arange(tot) - np.repeat(start, lens)
    ig = np.repeat(Pg[rows], lens) + within
    io = np.repeat(Po[rows], lens) + within
    row_of = np.repeat(rows, lens)
    ceq = np.asarray(Cg)[ig] == np.asarray(Co)[io]
    pat = same.copy()
    pat[np.unique(row_of[~ceq])] = False
    diff = np.zeros(n)
    d = np.abs(np.asarray(Vg, np.float64)[ig] - np.asarray(Vo, np.float64)[io])
    np.maximum.at(diff, row_of, d)
    diff[~pat] = np.inf
    return pat, diff


def check_step(G, O, margin, guard=1e-5, tol=1e-5, max_guarded_frac=1e-2, what=""):
    """Bit-exact patterns and values within tol on every row whose oracle
    decisions are all further than `guard` from their thresholds."""
    pat, diff = row_compare(G, O)
    unguarded = margin >= guard
    bad = unguarded & ~pat
    assert not bad.any(), f"{what}: pattern differs on {bad.sum()} unguarded rows, e.g. {np.nonzero(bad)[0][:5]}"
    worst = diff[unguarded].max() if unguarded.any() else 0.0
    assert worst <= tol, f"{what}: max |dphi| {worst} > {tol}"
    assert (~unguarded).mean() <= max_guarded_frac, f"{what}: {(~unguarded).sum()} guarded rows"
    return {"guarded": int((~unguarded).sum()), "max_diff": float(worst),
            "guarded_mismatch": int((~pat & ~unguarded).sum())}
