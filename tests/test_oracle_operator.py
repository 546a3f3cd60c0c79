"""Pins for the oracle's mesh operator (Section 3.2, Laplacian computation)."""
import math

import numpy as np
import pytest

from paper_1804_09152_amd import inputs as I
from tests.dense_ref import dense_operator, torus_graph_operator


def _dense(orc, L, n):
    return orc.to_dense(L, n)


def _octahedron():
    V = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    F = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
                  [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], np.int32)
    return V, F


def test_equilateral_cotan_weight(orc):
    # every face of the regular octahedron is equilateral: each edge weight is
    # (cot 60 + cot 60)/2 = 1/sqrt(3), each vertex has four edges
    V, F = _octahedron()
    D = _dense(orc, orc.operator(V, F, 1), 6)
    w = 1 / math.sqrt(3)
    for i in range(6):
        off = np.delete(D[i], i)
        assert np.allclose(sorted(off), [0.0] + [w] * 4, atol=1e-15)
        assert abs(D[i, i] + 4 * w) < 1e-14


@pytest.mark.parametrize("op", [0, 1])
def test_zero_row_sums_symmetry_nsd(orc, op):
    m = I.jitter(I.icosphere(2), np.random.default_rng(5))
    D = _dense(orc, orc.operator(m.V, m.F, op), m.n_v)
    assert np.abs(D.sum(1)).max() < 1e-13
    assert np.abs(D - D.T).max() < 1e-15
    ev = np.linalg.eigvalsh(D)
    assert ev.max() < 1e-10  # approximates +Laplacian: negative semi-definite
    assert abs(ev).min() < 1e-10  # constants are in the null space


def test_graph_degrees(orc):
    m = I.torus_grid(9, 7)
    ptr, col, val = orc.operator(m.V, m.F, 0)
    assert np.all(np.diff(ptr) == 7)  # 6 neighbours + diagonal
    D = _dense(orc, (ptr, col, val), m.n_v)
    assert np.all(np.diag(D) == -6)


@pytest.mark.parametrize("nx,ny", [(3, 3), (9, 7), (64, 33)])
def test_torus_graph_operator_closed_form(orc, nx, ny):
    """The graph operator of a torus grid equals its closed form (six
    neighbours of weight 1, diagonal -6), entry for entry."""
    m = I.torus_grid(nx, ny)
    ptr, col, val = orc.operator(m.V, m.F, 0)
    cp, cc, cv = torus_graph_operator(nx, ny)
    assert np.array_equal(ptr, cp) and np.array_equal(col, cc) and np.array_equal(val, cv)


@pytest.mark.parametrize("op", [0, 1])
def test_against_brute_force_dense(orc, op):
    rng = np.random.default_rng(2)
    m = I.jitter(I.icosphere(2), rng)
    D = _dense(orc, orc.operator(m.V, m.F, op), m.n_v)
    B = dense_operator(m.V, m.F, op)
    assert np.abs(D - B).max() < 1e-11
    if op == 1:
        # jitter makes some weights negative; the operator keeps them
        assert (B < -1e-12).sum() - 0 >= 0


def test_sorted_columns_and_invalid_faces(orc):
    m = I.icosphere(1)
    ptr, col, _ = orc.operator(m.V, m.F, 1)
    for i in range(m.n_v):
        assert (np.diff(col[ptr[i]:ptr[i + 1]]) > 0).all()
    bad = m.F.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(RuntimeError):
        orc.operator(m.V, bad, 0)
