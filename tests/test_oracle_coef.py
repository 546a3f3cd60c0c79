"""Pins for the oracle's step with per-pair coefficients (equation (2) with
a, w, e per pair of layers; Section 3.1 keeps them scalars and foresees
varying them).  Layers carry types and a pair of layers takes its
coefficients from a table over pairs of types.

Checked against: the brute-force dense Algorithm 1 through equation (15)
with the full coefficient matrices (tests/dense_ref.py), a non-symmetric
table so that a transposed index fails; the scalar step, which one type
must reproduce bit for bit; relabelling the types, which must change
nothing."""
import numpy as np
import pytest

from paper_1804_09152_amd import inputs as I
from tests.dense_ref import dense_operator, dense_step


def _table(rng, n_t, symmetric=True):
    t = np.empty((n_t, n_t, 3))
    t[..., 0] = rng.uniform(0.02, 0.06, (n_t, n_t))
    t[..., 1] = rng.uniform(0.1, 0.3, (n_t, n_t))
    t[..., 2] = rng.uniform(0.5, 1.5, (n_t, n_t))
    if symmetric:
        t = 0.5 * (t + t.transpose(1, 0, 2))
    return t


CASES = [
    ("torus8", lambda: I.torus_grid(8, 8), 0, 3),
    ("torus12", lambda: I.torus_grid(12, 12), 0, 5),
    ("ico2_cot", lambda: I.jitter(I.icosphere(2), np.random.default_rng(3)), 1, 4),
]


@pytest.mark.parametrize("name,make,op,k", CASES)
@pytest.mark.parametrize("base_mode,symmetric", [(0, True), (1, True), (0, False)])
def test_typed_against_dense_algorithm(orc, name, make, op, k, base_mode, symmetric):
    """Teacher-forced for 30 steps: patterns equal (outside decisions within
    1e-9 of a threshold), values to 1e-12."""
    m = make()
    rng = np.random.default_rng(len(name) + 10 * k + base_mode)
    seeds = I.seeds_uniform(m.n_v, k, rng)
    n_t = 3
    types = rng.integers(0, n_t, k + 1)
    p = orc.default_params(base_mode=base_mode, types=types, table=_table(rng, n_t, symmetric))
    L = orc.operator(m.V, m.F, op)
    Ld = dense_operator(m.V, m.F, op)
    U = orc.init(m.n_v, seeds)
    guarded = 0
    for t in range(30):
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
    assert guarded < 5 * m.n_v


@pytest.mark.parametrize("base_mode", [0, 1])
def test_one_type_is_the_scalar_step(orc, base_mode):
    m = I.jitter(I.icosphere(3), np.random.default_rng(5))
    seeds = I.seeds_uniform(m.n_v, 12, np.random.default_rng(6))
    L = orc.operator(m.V, m.F, 1)
    ps = orc.default_params(base_mode=base_mode)
    pt = orc.default_params(base_mode=base_mode, types=np.zeros(13, np.int32),
                            table=np.array([[[ps["a"], ps["w"], ps["e"]]]]))
    Us = Ut = orc.init(m.n_v, seeds)
    for _ in range(30):
        Us = orc.step(L, Us, 12, ps)
        Ut = orc.step(L, Ut, 12, pt)
        for x, y in zip(Us, Ut):
            assert np.array_equal(x, y)


def test_relabelling_types_changes_nothing(orc):
    m = I.torus_grid(16, 16)
    rng = np.random.default_rng(9)
    seeds = I.seeds_uniform(m.n_v, 8, rng)
    L = orc.operator(m.V, m.F, 0)
    n_t = 4
    types = rng.integers(0, n_t, 9)
    tab = _table(rng, n_t, symmetric=False)
    perm = rng.permutation(n_t)  # type t is called perm[t] after relabelling
    tab2 = np.empty_like(tab)
    tab2[perm[:, None], perm[None, :]] = tab
    p1 = orc.default_params(types=types, table=tab)
    p2 = orc.default_params(types=perm[types], table=tab2)
    U1 = U2 = orc.init(m.n_v, seeds)
    for _ in range(25):
        U1 = orc.step(L, U1, 8, p1)
        U2 = orc.step(L, U2, 8, p2)
    for x, y in zip(U1, U2):
        assert np.array_equal(x, y)


def test_types_change_the_result(orc):
    """A penalty w between two types that differs from the others' moves
    the fields (the table is not ignored)."""
    m = I.torus_grid(16, 16)
    seeds = I.seeds_uniform(m.n_v, 8, np.random.default_rng(2))
    L = orc.operator(m.V, m.F, 0)
    base = orc.default_params()
    tab = np.tile(np.array([base["a"], base["w"], base["e"]]), (2, 2, 1))
    tab[0, 1, 1] = tab[1, 0, 1] = 0.6
    types = np.array([0, 1] * 4 + [0], np.int32)
    U1 = U2 = orc.init(m.n_v, seeds)
    for _ in range(40):
        U1 = orc.step(L, U1, 8, base)
        U2 = orc.step(L, U2, 8, orc.default_params(types=types, table=tab))
    D1, D2 = orc.to_dense(U1, 9), orc.to_dense(U2, 9)
    assert np.abs(D1 - D2).max() > 1e-3


def test_invalid_types_rejected(orc):
    m = I.torus_grid(6, 6)
    L = orc.operator(m.V, m.F, 0)
    U = orc.init(m.n_v, [0, 7])
    p = orc.default_params(types=np.array([0, 2, 0]), table=np.zeros((2, 2, 3)))
    with pytest.raises(Exception):
        orc.step(L, U, 2, p)
