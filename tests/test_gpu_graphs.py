"""Chunks of 256 steps replayed from captured HIP graphs against the same
steps launched one by one: identical fields and counters after every replay,
with eager chunks, storage growth (re-capture) and a batch in between."""
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
    assert a.stats() == b.stats()
    assert a.last_change() == b.last_change()


def test_graph_replays_equal_eager(lf):
    lfb, ctx = lf
    mesh, seeds = I.config_c2(level=5, n_seeds=64, seed=2)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, lfb.LF_OP_COTAN)
    a, b = lfb.Fields(m, seeds), lfb.Fields(m, seeds)
    a.use_graphs(True)
    for rep in range(4):
        say("graph replay", rep)
        a.step(256)
        b.step(256)
        _same(a, b)
        a.step(37)  # an eager chunk between replays moves the starting buffer
        b.step(37)
        _same(a, b)
    a.use_graphs(False)
    a.step(256)
    b.step(256)
    _same(a, b)


def test_graph_recaptured_after_growth(lf):
    """Dense seeds fill a small overflow area during a captured chunk: the
    chunk stops at the failed step, the area grows, the rest is replayed, and
    the next whole chunk is captured again over the new buffers."""
    lfb, ctx = lf
    mesh, seeds = I.config_c2(level=3, n_seeds=160, seed=5)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, lfb.LF_OP_COTAN)
    prm = lfb.default_params(capacity_hint=90)
    a, b = lfb.Fields(m, seeds, prm), lfb.Fields(m, seeds, prm)
    a.use_graphs(True)
    for rep in range(3):
        say("graph growth", rep)
        a.step(256)
        b.step(256)
        _same(a, b)
    assert a.stats()["grow_events"] > 0


def test_batch_graphs(lf):
    lfb, ctx = lf
    items = I.batch_tori(12, nv_hi=2e4)
    mk = lambda: lfb.Batch(ctx, [(mm.V, mm.F) for mm, _ in items], lfb.LF_OP_GRAPH,
                           [s for _, s in items])
    A, B = mk(), mk()
    A.use_graphs(True)
    say("batch graphs")
    for rep in range(2):
        A.step(256)
        B.step(256)
        for q in range(len(items)):
            for x, y in zip(A.export(q), B.export(q)):
                assert np.array_equal(x, y)
    A.close()
    B.close()
