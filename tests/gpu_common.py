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


def _row(C, V, P, i):
    return {int(c): float(v) for c, v in zip(C[P[i]:P[i + 1]], V[P[i]:P[i + 1]])}


def check_step(G, O, info, theta, guard=1e-5, tol=1e-5, max_skel_guarded_frac=1e-3, what=""):
    """One GPU step G against one oracle step O from the same float32 input.
    info: the oracle's per-row margins (margin: every discrete decision of
    the row; smargin: its rows-of-interest decisions alone).  Rows are
    checked by what their near-ties (decisions closer than `guard` to their
    threshold) can change:
      clear rows (margin >= guard): identical pattern, values within tol;
      rows whose only near-ties are prune / clamp decisions: the entries
        present on both sides within tol (a pruned entry is not renormalised
        away, and a clamp near zero moves the row sum by less than guard);
        an entry present on one side only holds a value within guard + tol of
        theta (of zero when theta = 0);
      rows with a near-tie in the rows of interest (a layer whose field
        Laplacian is within guard of zero may join or not, which changes n
        and every value of the row): a valid row (ascending layers, values
        in (0, 1], sum in [1 - 64 theta - tol, 1 + tol]); their fraction is
        bounded by max_skel_guarded_frac.
    Returns the counts of each kind."""
    margin, smargin = info["margin"], info["smargin"]
    pat, diff = row_compare(G, O)
    clear = margin >= guard
    skel_g = smargin < guard
    out_g = ~clear & ~skel_g
    bad = clear & ~pat
    assert not bad.any(), f"{what}: pattern differs on {bad.sum()} clear rows, e.g. {np.nonzero(bad)[0][:5]}"
    worst = diff[clear].max() if clear.any() else 0.0
    assert worst <= tol, f"{what}: max |dphi| {worst} > {tol}"
    Pg, Cg, Vg = (np.asarray(x) for x in G)
    Po, Co, Vo = (np.asarray(x) for x in O)
    for i in np.nonzero(out_g)[0]:
        a, b = _row(Cg, Vg, Pg, i), _row(Co, Vo, Po, i)
        for c in set(a) & set(b):
            assert abs(a[c] - b[c]) <= tol, f"{what}: row {i} layer {c}: {a[c]} vs {b[c]}"
        for c in set(a) ^ set(b):
            v = a.get(c, b.get(c))
            assert abs(v - theta) <= guard + tol, f"{what}: row {i} layer {c} kept on one side at {v}"
    for i in np.nonzero(skel_g)[0]:
        a = _row(Cg, Vg, Pg, i)
        cols = list(a)
        assert cols == sorted(cols) and all(0.0 < v <= 1.0 for v in a.values()), f"{what}: row {i}"
        if a:
            tot = sum(a.values())
            # at most 64 layers per row, each pruned below theta
            assert 1.0 - 64 * theta - tol <= tot <= 1.0 + tol, f"{what}: row {i} sums to {tot}"
    assert skel_g.mean() <= max_skel_guarded_frac, f"{what}: {skel_g.sum()} rows with a near-tie rows-of-interest decision"
    res = {"output_guarded": int(out_g.sum()), "skel_guarded": int(skel_g.sum()),
           "max_diff": float(worst), "guarded_mismatch": int((~pat & ~clear).sum()),
           "rows": int(margin.size)}
    say("check_step", what, res)
    return res
