"""Pins for the oracle's time step (Algorithm 1, equations (11)-(13)).

Each test checks the oracle against something other than itself: a hand
derivation, a brute-force dense implementation through the alternate sum of
equation (15), an algebraic closed form, or an invariant of the mathematics.
"""
import os

import numpy as np
import pytest

from paper_1804_09152_amd import inputs as I
from tests.dense_ref import closed_form_row, coefficient_matrices, dense_operator, dense_step

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _to_csr(D):
    """dense rows x cols -> CSR triple over the positive entries"""
    ptr = np.zeros(D.shape[0] + 1, np.int64)
    cols, vals = [], []
    for i in range(D.shape[0]):
        nz = np.nonzero(D[i] > 0)[0]
        cols.extend(nz)
        vals.extend(D[i, nz])
        ptr[i + 1] = len(cols)
    return ptr, np.array(cols, np.int32), np.array(vals, float)


def _xy(nx, v):
    return v % nx, v // nx


def test_golden_single_seed_first_step(orc):
    rows = {}
    for line in open(os.path.join(GOLDEN, "single_seed_step1.txt")):
        if line.strip() and not line.startswith("#"):
            role, c, b = line.split()
            rows[role] = (float(c), float(b))
    m = I.torus_grid(10, 10)
    L = orc.operator(m.V, m.F, 0)
    s = 0
    U = orc.step(L, orc.init(m.n_v, [s]), 1, orc.default_params())
    D = orc.to_dense(U, 2)
    nbr = [int(c) for c in L[1][L[0][s]:L[0][s + 1]] if c != s]
    assert len(nbr) == 6
    assert np.allclose(D[s], rows["seed"], atol=1e-14)
    for u in nbr:
        assert np.allclose(D[u], rows["neighbour"], atol=1e-14)
    far = [v for v in range(m.n_v) if v != s and v not in nbr]
    assert np.allclose(D[far], rows["far"], atol=0)


CASES = [
    ("torus6", lambda: I.torus_grid(6, 6), 0, 2),
    ("torus8", lambda: I.torus_grid(8, 8), 0, 3),
    ("torus12", lambda: I.torus_grid(12, 12), 0, 5),
    ("ico2_cot", lambda: I.jitter(I.icosphere(2), np.random.default_rng(3)), 1, 4),
]


@pytest.mark.parametrize("name,make,op,k", CASES)
@pytest.mark.parametrize("theta,base_mode", [(1e-3, 0), (0.0, 0), (1e-3, 1)])
def test_against_dense_algorithm(orc, name, make, op, k, theta, base_mode):
    """Teacher-forced for 50 steps: the oracle and the dense equation-(15)
    implementation take the same input every step; patterns must match
    exactly (outside rows with a decision within 1e-9 of its threshold) and
    values to 1e-12."""
    m = make()
    rng = np.random.default_rng(len(name) + k)
    seeds = I.seeds_uniform(m.n_v, k, rng)
    p = orc.default_params(theta=theta, base_mode=base_mode)
    L = orc.operator(m.V, m.F, op)
    Ld = dense_operator(m.V, m.F, op)
    U = orc.init(m.n_v, seeds)
    guarded = 0
    for t in range(50):
        Phi = orc.to_dense(U, k + 1).T
        Dn, sizes = dense_step(Phi, Ld, k, p)
        U2, info = orc.step(L, U, k, p, want_info=True)
        Do = orc.to_dense(U2, k + 1)
        ok = info["margin"] > 1e-9
        guarded += int((~ok).sum())
        assert np.array_equal(Do[ok] > 0, Dn.T[ok] > 0), f"pattern differs at step {t}"
        assert np.abs(Do[ok] - Dn.T[ok]).max() < 1e-12
        assert np.array_equal(info["skel"][ok], sizes[ok])
        U = U2
    assert guarded < 5 * m.n_v  # the guard is for rare near-ties only


def test_closed_form_identity(orc):
    """Random active sets, with and without the base: the literal triple loop
    of Algorithm 1 (inside the oracle) equals the O(n) closed form."""
    rng = np.random.default_rng(7)
    m = I.jitter(I.icosphere(2), rng)
    n_s = 6
    p = orc.default_params(theta=0.0)
    L = orc.operator(m.V, m.F, 1)
    Ld = orc.to_dense(L, m.n_v)
    for trial in range(20):
        # random sparse fields: every vertex gets 1-4 random layers
        D = np.zeros((m.n_v, n_s + 1))
        for i in range(m.n_v):
            cols = rng.choice(n_s + 1, size=rng.integers(1, 5), replace=False)
            D[i, cols] = rng.uniform(0.05, 1.0, cols.size)
        D /= D.sum(1, keepdims=True)
        U = _to_csr(D)
        U2, info = orc.step(L, U, n_s, p, want_info=True)
        Do = orc.to_dense(U2, n_s + 1)
        Lt = Ld @ D  # rows = vertices
        for i in range(m.n_v):
            S = np.nonzero((D[i] > 0) | ((D[i] == 0) & (Lt[i] > 0)))[0]
            v = closed_form_row(D[i, S], Lt[i, S], S == n_s, p)
            v = np.clip(v, 0, 1)
            if v.sum() > 0:
                v = v / v.sum()
            exp = np.zeros(n_s + 1)
            exp[S] = v
            assert np.abs(exp - Do[i]).max() < 1e-13


def test_constant_field_invariance(orc):
    """L 1 = 0: if every layer is spatially constant the field Laplacian
    vanishes and every vertex takes the same update."""
    m = I.jitter(I.icosphere(3), np.random.default_rng(1))
    for op in (0, 1):
        L = orc.operator(m.V, m.F, op)
        row = np.array([0.3, 0.0, 0.5, 0.2])  # cells 0..2 and base
        D = np.tile(row, (m.n_v, 1))
        U = _to_csr(D)
        for _ in range(5):
            U = orc.step(L, U, 3, orc.default_params())
            Do = orc.to_dense(U, 4)
            assert np.abs(Do - Do[0]).max() < 1e-14


def test_single_seed_floods_and_seedless_component_stays_base(orc):
    a = I.torus_grid(20, 20)
    b = I.torus_grid(10, 10)
    V = np.concatenate([a.V, b.V + 20.0])
    F = np.concatenate([a.F, b.F + a.n_v]).astype(np.int32)
    L = orc.operator(V, F, 0)
    U = orc.init(V.shape[0], [37])
    for _ in range(120):
        U = orc.step(L, U, 1, orc.default_params())
    D = orc.to_dense(U, 2)
    assert (D[: a.n_v, 0] == 1.0).all() and (D[: a.n_v, 1] == 0).all()
    assert (D[a.n_v:, 1] == 1.0).all() and (D[a.n_v:, 0] == 0).all()


def test_uniform_base_reading_cannot_grow(orc):
    """With the base as an ordinary layer, a one-vertex seed mirrors a
    one-vertex hole in the base and shrinks (base_mode 1)."""
    m = I.torus_grid(16, 16)
    L = orc.operator(m.V, m.F, 0)
    U = orc.init(m.n_v, [0])
    for _ in range(30):
        U = orc.step(L, U, 1, orc.default_params(base_mode=1))
    D = orc.to_dense(U, 2)
    assert (D[:, 0] > 0).sum() == 1 and D[0, 0] < 0.5


def _mirror_check(orc, nx, seeds_xy, vmap, cmap, steps=100):
    m = I.torus_grid(nx, nx)
    L = orc.operator(m.V, m.F, 0)
    seeds = np.array([x + nx * y for x, y in seeds_xy], np.int32)
    U = orc.init(m.n_v, seeds)
    k = len(seeds)
    perm_v = np.array([vmap(*_xy(nx, v)) for v in range(m.n_v)])
    for t in range(steps):
        U = orc.step(L, U, k, orc.default_params())
        D = orc.to_dense(U, k + 1)
        M = D[perm_v][:, cmap]
        assert np.array_equal(D > 0, M > 0), f"pattern asymmetric at step {t}"
        assert np.abs(D - M).max() < 1e-12


def test_mirror_symmetry_transpose(orc):
    nx = 16
    _mirror_check(orc, nx, [(2, 5), (5, 2), (10, 12), (12, 10), (7, 7)],
                  lambda x, y: y + nx * x, [1, 0, 3, 2, 4, 5])


def test_mirror_symmetry_point_reflection(orc):
    nx = 16
    _mirror_check(orc, nx, [(2, 5), (14, 11), (4, 12), (12, 4)],
                  lambda x, y: (-x) % nx + nx * ((-y) % nx), [1, 0, 3, 2, 4])


def test_front_speed_at_most_one_ring_per_step(orc):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    m = I.torus_grid(24, 24)
    L = orc.operator(m.V, m.F, 0)
    A = csr_matrix((np.ones(L[1].size), L[1], L[0]), shape=(m.n_v, m.n_v))
    dist = shortest_path(A, unweighted=True, indices=[0])[0]
    U = orc.init(m.n_v, [0])
    for t in range(1, 40):
        U = orc.step(L, U, 1, orc.default_params())
        D = orc.to_dense(U, 2)
        assert dist[D[:, 0] > 0].max() <= t


def test_bounds_and_partition_of_unity(orc):
    m, seeds = I.config_c2(level=3, n_seeds=24)
    L = orc.operator(m.V, m.F, 1)
    U = orc.init(m.n_v, seeds)
    p = orc.default_params()
    for _ in range(150):
        U, info = orc.step(L, U, 24, p, want_info=True)
        assert info["events"] == 0
        v = U[2]
        assert (v > 0).all() and (v <= 1).all() and (v >= p["theta"]).all()
        sums = np.add.reduceat(v, U[0][:-1])
        pruned = info["skel"] - np.diff(U[0])  # each pruned entry was below theta
        assert (sums <= 1 + 1e-14).all()
        assert (sums >= 1 - pruned * p["theta"] - 1e-14).all()


def test_band_term_ablation(orc):
    """Without the band term g (e = 0) the fields do not separate into a band
    (Figure 5): the squared sum stays near 1 and fewer vertices are shared."""
    m, seeds = I.config_c1()
    L = orc.operator(m.V, m.F, 0)
    res = {}
    for e in (1.0, 0.0):
        U = orc.init(m.n_v, seeds)
        U, _ = orc.run(L, U, 32, orc.default_params(e=e), 150)
        D = orc.to_dense(U, 33)
        res[e] = ((D ** 2).sum(1).mean(), U[0][-1] / m.n_v)
    assert res[0.0][0] > res[1.0][0] + 0.03
    assert res[0.0][1] < res[1.0][1]


def test_voronoi_agreement_c1(orc):
    """Labels after 200 steps agree with graph-distance Voronoi cells (the
    paper's planar comparison, Section 3.1) on vertices without a tie."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    m, seeds = I.config_c1()
    L = orc.operator(m.V, m.F, 0)
    U, info = orc.run(L, orc.init(m.n_v, seeds), 32, orc.default_params(), 200)
    assert info["events"] == 0
    lab, gap = orc.labels(U, 32)
    A = csr_matrix((np.ones(L[1].size), L[1], L[0]), shape=(m.n_v, m.n_v))
    A.setdiag(0)
    A.eliminate_zeros()
    Dd = shortest_path(A, unweighted=True, indices=seeds)
    s = np.sort(Dd, 0)
    tied = s[0] == s[1]
    vor = np.argmin(Dd, 0)
    assert (lab[~tied] == vor[~tied]).mean() >= 0.99
    assert (lab >= 0).all()


def test_row_blocks_give_the_same_step(orc):
    """The row-block (threaded) step equals the one-thread step bit for bit,
    also its margins and rows-of-interest sizes, on a jittered icosphere state
    with bands and junctions."""
    mesh, seeds = I.config_c2(level=5, n_seeds=64, seed=3)
    L = orc.operator(mesh.V, mesh.F, 1)
    p = orc.default_params()
    U = orc.run(L, orc.init(mesh.n_v, seeds), 64, p, 80)[0]
    A, ia = orc.step(L, U, 64, p, want_info=True)
    for t in (2, 5, 16):
        B, ib = orc.step(L, U, 64, p, want_info=True, threads=t)
        for x, y in zip(A, B):
            assert np.array_equal(x, y)
        assert np.array_equal(ia["margin"], ib["margin"]) and np.array_equal(ia["skel"], ib["skel"])
        # the rows-of-interest margin is part of the whole margin
        assert (ib["smargin"] >= ib["margin"]).all()
