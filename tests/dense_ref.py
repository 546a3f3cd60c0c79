"""Brute-force dense helpers used only to pin the oracle on tiny inputs.

Independent of oracle/ (different representation, different formulas):
  * the operator is built from face angles via arccos/tan instead of
    dot/cross products, into a dense matrix;
  * the field step uses dense Phi (n_r x n_v), the dense product
    L_t = Phi @ L.T, dense coefficient matrices, and evaluates the inner sum
    of Algorithm 1 through the alternate form of Section 4 (equation 15):
    sum_jk = 1/2 (A_L(j) - A_L(k)) + (W_Phi(j) - W_Phi(k)) with
    A_L = a L_t and W_Phi = w Phi restricted to the rows of interest.
"""
from __future__ import annotations

import math

import numpy as np


def dense_operator(V, F, op):
    n = V.shape[0]
    L = np.zeros((n, n))
    for f in F:
        for c in range(3):
            o, p, q = f[c], f[(c + 1) % 3], f[(c + 2) % 3]
            if op == 0:
                L[p, q] = 1.0
                L[q, p] = 1.0
            else:
                u = V[p] - V[o]
                v = V[q] - V[o]
                ang = math.acos(np.clip(u @ v / (np.linalg.norm(u) * np.linalg.norm(v)), -1, 1))
                L[p, q] += 0.5 / math.tan(ang)
                L[q, p] += 0.5 / math.tan(ang)
    L[np.diag_indices(n)] = 0.0
    L[np.diag_indices(n)] = -L.sum(1)
    return L


def torus_graph_operator(nx, ny):
    """Graph operator of `inputs.torus_grid(nx, ny)` in closed form, as CSR
    (int64 row pointers, int32 sorted columns, float64 values): each vertex
    (x, y) has the six neighbours (x +- 1, y), (x, y +- 1), (x + 1, y + 1),
    (x - 1, y - 1) (the grid squares are split along that diagonal) with
    weight 1, and -6 on the diagonal.  Built from the grid, not from faces,
    so that it can stand in for the operator at sizes where a face-by-face
    build is slow."""
    x, y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    x = x.ravel()
    y = y.ravel()
    offs = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1)]
    cols = np.stack([(x + dx) % nx + nx * ((y + dy) % ny) for dx, dy in offs], 1)
    vals = np.where(np.arange(7) == 0, -6.0, 1.0)[None, :].repeat(cols.shape[0], 0)
    order = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, 1)
    vals = np.take_along_axis(vals, order, 1)
    ptr = np.arange(0, 7 * cols.shape[0] + 1, 7, dtype=np.int64)
    return ptr, cols.ravel().astype(np.int32), vals.ravel()


def coefficient_matrices(n_s, p):
    """Dense a, w, e over n_s cells + base (last).  With p["types"] and
    p["table"] (n_types x n_types x 3), entry (j, l) comes from the table at
    the pair of types; otherwise one scalar per matrix.  Zero diagonals; in
    base_mode 0 no w against the base, and the base's e against a cell is the
    negated table entry."""
    n_r = n_s + 1
    off = 1.0 - np.eye(n_r)
    if p.get("types") is not None:
        t = np.asarray(p["types"], dtype=np.int64)
        tab = np.asarray(p["table"], dtype=float)
        n_t = int(round((tab.size // 3) ** 0.5))
        tab = tab.reshape(n_t, n_t, 3)
        A = tab[t[:, None], t[None, :], 0] * off
        W = tab[t[:, None], t[None, :], 1] * off
        E = tab[t[:, None], t[None, :], 2] * off
    else:
        A = p["a"] * off
        W = p["w"] * off
        E = p["e"] * off
    if p.get("base_mode", 0) == 0:
        W[n_s, :] = 0.0
        W[:, n_s] = 0.0
        E[n_s, :n_s] = -E[n_s, :n_s]
    return A, W, E


def dense_step(Phi, L, n_s, p):
    """One Jacobi step of Algorithm 1 on dense Phi (n_r x n_v).  Returns the
    new Phi and the per-vertex active-set sizes."""
    A, W, E = coefficient_matrices(n_s, p)
    Lt = Phi @ L.T
    out = np.zeros_like(Phi)
    sizes = np.zeros(Phi.shape[1], dtype=np.int64)
    for i in range(Phi.shape[1]):
        col = Phi[:, i]
        lt = Lt[:, i]
        rows = np.nonzero((col > 0) | ((col == 0) & (lt > 0)))[0]
        n = rows.size
        sizes[i] = n
        if n == 0:
            continue
        AS = A[np.ix_(rows, rows)]
        WS = W[np.ix_(rows, rows)]
        ES = E[np.ix_(rows, rows)]
        s = 0.5 * (AS @ lt[rows]) + WS @ col[rows]
        sum_jk = s[:, None] - s[None, :]
        band = ES * np.sqrt(np.outer(col[rows], col[rows]))
        d = (-(p["mu"] / n) * (sum_jk - band)).sum(axis=1)
        v = np.clip(col[rows] + d * p["dt"], 0.0, 1.0)
        tot = v.sum()
        if tot > 0:
            v = v / tot
            v[(v < p["theta"]) | (v <= 0)] = 0.0
            out[rows, i] = v
    return out, sizes


def closed_form_row(phi, lam, is_base, p):
    """Closed-form update of one vertex's active set (O(n) per vertex):
    with T = sum lam, P_C = sum of cell phi, R_C = sum of cell sqrt(phi),
    Q_j = a/2 (T - lam_j) + w (P_C - phi_j) [cells only],
    G_cell = e (R_C - sqrt phi_j) + e sqrt(phi_base), G_base = -e R_C,
    d_j = -(mu/n) (n Q_j - sum_k Q_k - sqrt(phi_j) G_j).  Returns v before
    clamping."""
    n = phi.size
    cell = ~is_base
    T = lam.sum()
    PC = phi[cell].sum()
    RC = np.sqrt(phi[cell]).sum()
    pb = np.sqrt(phi[is_base]).sum()
    Q = 0.5 * p["a"] * (T - lam) + np.where(cell, p["w"] * (PC - phi), 0.0)
    G = np.where(cell, p["e"] * (RC - np.sqrt(phi)) + p["e"] * pb, -p["e"] * RC)
    d = -(p["mu"] / n) * (n * Q - Q.sum() - np.sqrt(phi) * G)
    return phi + p["dt"] * d
