"""Work-class ordering of the step's rows (interior rows first within
tiles, interior slices written without the merge): the fields, counters,
change measures and everything read from them are identical, bit for bit,
to a run that keeps the locality order."""
import numpy as np
import pytest

from paper_1804_09152_amd import inputs as I
from tests.gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_09152_amd as lfb
    lfb.load()
    yield lfb, lfb.Context(0)


def _same(a, b):
    for x, y in zip(a.export(), b.export()):
        assert np.array_equal(x, y)
    sa, sb = a.stats(), b.stats()
    for k in ("nnz", "skeleton_total", "steps", "empty_columns"):
        assert sa[k] == sb[k], k
    assert a.last_change() == b.last_change()
    assert np.array_equal(a.labels(), b.labels())


@pytest.mark.parametrize("level,k,every", [(6, 256, 512), (6, 256, 64), (7, 1024, 200)])
def test_reordered_steps_equal_locality_order(lf, level, k, every):
    lfb, ctx = lf
    mesh, seeds = I.config_c2(level=level, n_seeds=k, seed=3)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, lfb.LF_OP_COTAN)
    a, b = lfb.Fields(m, seeds), lfb.Fields(m, seeds)
    a.set_reorder(every)
    b.set_reorder(0)
    for n in (100, 300, 256, 190):
        say("reorder", level, k, every, n)
        a.step(n)
        b.step(n)
        _same(a, b)
    assert a.reorders() >= (1 if every > 300 else 2) and b.reorders() == 0
    # convergence stepping, import (teacher forcing) and post-processing on
    # the re-ordered fields
    assert a.step_until(300, 1e-2, 32) == b.step_until(300, 1e-2, 32)
    _same(a, b)
    G = b.export()
    a.load(*G)
    a.step(3)
    b.step(3)
    _same(a, b)
    sa, sta = a.lloyd_reseed()
    sb, stb = b.lloyd_reseed()
    assert np.array_equal(sa, sb) and np.array_equal(sta, stb)
    ta, (ra, ca) = a.dual_mesh(0.25)
    tb, (rb, cb) = b.dual_mesh(0.25)
    assert np.array_equal(ta, tb) and np.array_equal(ra, rb) and np.array_equal(ca, cb)
    # a reset keeps the order and moves the next re-ordering to 128 steps on
    a.reset(sa)
    b.reset(sa)
    a.step(400)
    b.step(400)
    _same(a, b)


def test_reordered_batch_and_typed(lf):
    """A batch (rows of many meshes in one order) and per-pair coefficients
    (the typed step instance) under re-ordering."""
    lfb, ctx = lf
    items = I.batch_tori(16, nv_hi=3e4, seed=4)
    mk = lambda: lfb.Batch(ctx, [(mm.V, mm.F) for mm, _ in items], lfb.LF_OP_GRAPH,
                           [sd for _, sd in items])
    A, B = mk(), mk()
    A.set_reorder(100)
    B.set_reorder(0)
    say("reorder batch")
    A.step(450)
    B.step(450)
    for q in range(len(items)):
        for x, y in zip(A.export(q), B.export(q)):
            assert np.array_equal(x, y)
        assert np.array_equal(A.labels(q), B.labels(q))
    A.close()
    B.close()
    mesh, seeds = I.config_c2(level=5, n_seeds=64, seed=6)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, lfb.LF_OP_COTAN)
    rng = np.random.default_rng(2)
    types = rng.integers(0, 3, seeds.size + 1).astype(np.int32)
    tab = rng.uniform(0.5, 1.5, (3, 3, 3)) * np.array([0.04, 0.2, 1.0])
    a, b = lfb.Fields(m, seeds), lfb.Fields(m, seeds)
    a.set_coefficients(types, tab)
    b.set_coefficients(types, tab)
    a.set_reorder(96)
    b.set_reorder(0)
    say("reorder typed")
    a.step(500)
    b.step(500)
    _same(a, b)
