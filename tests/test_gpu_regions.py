"""Fields from seeds grown into rings and from initial regions (Algorithm 1,
first line: seeds and/or initial regions) on the GPU against the FP64
oracle."""
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


def _patches(mesh, seeds, rng):
    """Disjoint regions for the regions entry point: each seed with a random
    part of its neighbours that no earlier region took (any disjoint regions
    are valid input)."""
    nb = [set() for _ in range(mesh.n_v)]
    for a, b, c in mesh.F:
        nb[a] |= {int(b), int(c)}
        nb[b] |= {int(a), int(c)}
        nb[c] |= {int(a), int(b)}
    taken = set(int(s) for s in seeds)
    ptr, verts = [0], []
    for s in seeds:
        reg = [int(s)] + [v for v in sorted(nb[s]) if v not in taken and rng.random() < 0.7]
        taken |= set(reg)
        verts += reg
        ptr.append(len(verts))
    return np.array(ptr, np.int32), np.array(verts, np.int32)


@pytest.mark.parametrize("name,rings", [("c1", 1), ("c1", 2), ("ico5", 1), ("ico5", 3)])
def test_rings_init_is_exact(lf, orc, name, rings):
    """Seeds grown by rings on the GPU equal the oracle's breadth-first
    regions bit for bit; a reset grows the new seeds the same way."""
    lfb, ctx = lf
    if name == "c1":
        mesh, seeds = I.config_c1()
        op = 0
    else:
        mesh, seeds = I.config_c2(level=5, n_seeds=64, seed=2)
        op = 1
    say("rings init", name, rings)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, op)
    f = lfb.Fields(m, seeds, rings=rings)
    G = f.export()
    O = orc.init_rings(mesh.n_v, mesh.F, seeds, rings)
    assert np.array_equal(np.asarray(G[0], np.int64), O[0])
    assert np.array_equal(G[1], O[1]) and np.array_equal(G[2].astype(np.float64), O[2])
    assert np.array_equal(f.seeds(), seeds)
    f.step(7)
    s2 = np.roll(seeds, 1)
    f.reset(s2)
    O2 = orc.init_rings(mesh.n_v, mesh.F, s2, rings)
    assert np.array_equal(f.export()[1], O2[1])


def test_init_from_regions_is_exact(lf, orc):
    lfb, ctx = lf
    mesh, seeds = I.config_c1()
    ptr, verts = _patches(mesh, seeds, np.random.default_rng(5))
    m = lfb.Mesh(ctx, mesh.V, mesh.F, 0)
    f = lfb.Fields(m, regions=(ptr, verts))
    G = f.export()
    O = orc.init_regions(mesh.n_v, ptr, verts)
    assert np.array_equal(np.asarray(G[0], np.int64), O[0])
    assert np.array_equal(G[1], O[1]) and np.array_equal(G[2].astype(np.float64), O[2])
    assert np.array_equal(f.seeds(), verts[ptr[:-1]])


def test_one_ring_seeds_free_running(lf, orc):
    """1-ring seeds on C1 (grown by the library): 150 float32 GPU steps
    against 150 float64 oracle steps from the oracle's own 1-ring regions,
    identical patterns and labels, fields within 1e-5."""
    lfb, ctx = lf
    mesh, seeds = I.config_c1()
    P = orc.default_params()
    L = orc.operator(mesh.V, mesh.F, 0)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, 0)
    f = lfb.Fields(m, seeds, rings=1)
    U = orc.init_rings(mesh.n_v, mesh.F, seeds, 1)
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
