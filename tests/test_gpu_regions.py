"""Fields from initial regions (Algorithm 1, first line: seeds and/or
initial regions) on the GPU against the FP64 oracle."""
import numpy as np
import pytest

from paper_1804_09152_amd import inputs as I
from tests.gpu_common import as_oracle, row_compare, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_09152_amd as lfb
    lfb.load()
    ctx = lfb.Context(0)
    yield lfb, ctx


def test_init_from_regions_is_exact(lf, orc):
    lfb, ctx = lf
    mesh, seeds = I.config_c1()
    ptr, verts = I.ring_regions(mesh, seeds)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, 0)
    f = lfb.Fields(m, regions=(ptr, verts))
    G = f.export()
    O = orc.init_regions(mesh.n_v, ptr, verts)
    assert np.array_equal(np.asarray(G[0], np.int64), O[0])
    assert np.array_equal(G[1], O[1]) and np.array_equal(G[2].astype(np.float64), O[2])
    assert np.array_equal(f.seeds(), verts[ptr[:-1]])


def test_one_ring_seeds_free_running(lf, orc):
    """1-ring seeds on C1: 150 float32 GPU steps against 150 float64 oracle
    steps, identical patterns and labels, fields within 1e-5."""
    lfb, ctx = lf
    mesh, seeds = I.config_c1()
    ptr, verts = I.ring_regions(mesh, seeds)
    P = orc.default_params()
    L = orc.operator(mesh.V, mesh.F, 0)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, 0)
    f = lfb.Fields(m, regions=(ptr, verts))
    U = orc.init_regions(mesh.n_v, ptr, verts)
    for chunk in range(5):
        say("1-ring seeds chunk", chunk)
        f.step(30)
        U, _ = orc.run(L, U, seeds.size, P, 30)
        pat, diff = row_compare(as_oracle(f.export()), U)
        assert pat.all(), f"pattern differs on {(~pat).sum()} rows"
        assert diff.max() <= 1e-5
    lab_o, gap = orc.labels(U, seeds.size)
    clear = gap > 1e-5
    assert np.array_equal(f.labels()[clear], lab_o[clear])


def test_regions_reset_and_invalid(lf, orc):
    lfb, ctx = lf
    mesh = I.torus_grid(20, 20)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, 0)
    ptr = np.array([0, 3, 5], np.int32)
    verts = np.array([10, 11, 30, 200, 201], np.int32)
    f = lfb.Fields(m, regions=(ptr, verts))
    f.step(5)
    f.reset_regions(ptr, verts)
    O = orc.init_regions(mesh.n_v, ptr, verts)
    G = f.export()
    assert np.array_equal(G[1], O[1])
    for bad in ((np.array([0, 3, 5]), np.array([10, 11, 30, 30, 201])),   # overlap
                (np.array([0, 0, 5]), np.array([10, 11, 30, 200, 201])),  # empty region
                (np.array([0, 3, 5]), np.array([10, 11, 30, 200, 400]))):  # out of range
        with pytest.raises(lfb.LFError):
            lfb.Fields(m, regions=bad)
    # a bad reset leaves the fields as they were
    f.step(3)
    before = f.export()
    with pytest.raises(lfb.LFError):
        f.reset_regions(np.array([0, 3, 5]), np.array([10, 11, 30, 30, 201]))
    after = f.export()
    assert all(np.array_equal(a, b) for a, b in zip(before, after))
