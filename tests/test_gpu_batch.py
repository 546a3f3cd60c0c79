"""Batches and the job server compute exactly what solo runs compute.

A batch is a disjoint union of meshes with per-mesh layer offsets and one
shared base layer, so every row sees the same operands in the same order as
in a solo run: fields and labels must be bit-identical.  The server runs each
job on its own stream with the solo entry points, so its seeds, labels and
dual-mesh triangles must be bit-identical to a solo sequence of the same
calls.  Solo runs are checked against the oracle in the other GPU tests."""
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
    ctx = lfb.Context(0)
    yield lfb, ctx


def _solo_fields(lfb, ctx, mesh, seeds, op, params, steps):
    M = lfb.Mesh(ctx, mesh.V, mesh.F, op)
    f = lfb.Fields(M, seeds, params)
    f.step(steps)
    return M, f


def _same_csr(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("op,cap", [(0, 0), (1, 0), (0, 1)])
def test_batch_equals_solo(lf, op, cap):
    lfb, ctx = lf
    items = I.batch_tori(8, seed=3, nv_lo=150, nv_hi=6000, s_lo=3, s_hi=80)
    # capacity_hint 1: a one-entry overflow area (grown if a row needs it)
    params = lfb.default_params(capacity_hint=cap) if cap else lfb.default_params()
    steps = 45
    say(f"batch op={op} cap={cap}: {[m.n_v for m, _ in items]} vertices")
    B = lfb.Batch(ctx, [(m.V, m.F) for m, _ in items], op, [s for _, s in items], params)
    B.step(steps)
    st = B.stats()
    assert st["steps"] == steps
    for k, (mesh, seeds) in enumerate(items):
        M, f = _solo_fields(lfb, ctx, mesh, seeds, op, params, steps)
        assert _same_csr(B.export(k), f.export()), f"mesh {k} fields differ from its solo run"
        assert np.array_equal(B.labels(k), f.labels()), f"mesh {k} labels differ"
        f.close()
        M.close()
    B.close()


def test_batch_of_one_and_counters(lf):
    lfb, ctx = lf
    mesh, seeds = I.config_c1()
    B = lfb.Batch(ctx, [(mesh.V, mesh.F)], 0, [seeds])
    B.step(30)
    M, f = _solo_fields(lfb, ctx, mesh, seeds, 0, None, 30)
    assert _same_csr(B.export(0), f.export())
    # counters of a batch of one are those of the solo run
    for k in ("nnz", "skeleton_total", "steps"):
        assert B.stats()[k] == f.stats()[k]


def test_batch_rejects_bad_input(lf):
    lfb, ctx = lf
    mesh, seeds = I.config_c1()
    bad = seeds.copy()
    bad[0] = mesh.n_v
    with pytest.raises(lfb.LFError):
        lfb.Batch(ctx, [(mesh.V, mesh.F), (mesh.V, mesh.F)], 0, [seeds, bad])
    with pytest.raises(lfb.LFError):
        lfb.Batch(ctx, [], 0, [])


def _solo_job(lfb, ctx, mesh, seeds, op, steps, rounds, dual, params):
    M = lfb.Mesh(ctx, mesh.V, mesh.F, op)
    f = lfb.Fields(M, seeds, params)
    f.step(steps)
    for _ in range(rounds):
        s, _ = f.lloyd_reseed()
        f.reset(s)
        f.step(steps)
    out = dict(labels=f.labels(), seeds=f.seeds())
    out["tris"] = f.dual_mesh(params.tau if params else 0.25)[0] if dual else np.zeros((0, 3), np.int32)
    f.close()
    M.close()
    return out


def _jobs():
    rng = np.random.default_rng(11)
    out = []
    t = I.torus_grid(24, 24)
    out.append((t, I.seeds_uniform(t.n_v, 6, rng), 0, 40, 0, False))
    m3 = I.jitter(I.icosphere(3), rng)
    out.append((m3, I.seeds_uniform(m3.n_v, 16, rng), 0, 60, 1, True))
    m4 = I.jitter(I.icosphere(4), rng)
    out.append((m4, I.seeds_uniform(m4.n_v, 32, rng), 1, 50, 2, True))
    t2 = I.torus_grid(40, 30)
    out.append((t2, I.seeds_uniform(t2.n_v, 20, rng), 0, 33, 0, True))
    out.append((m3, I.seeds_uniform(m3.n_v, 12, rng), 1, 0, 1, False))
    return out


@pytest.mark.parametrize("max_active,budget_mb,chunk", [(3, 12, 16), (8, 4096, 7), (1, 4096, 64)])
def test_server_equals_solo(lf, max_active, budget_mb, chunk):
    lfb, ctx = lf
    jobs = _jobs()
    say(f"server max_active={max_active} budget={budget_mb}MB chunk={chunk}")
    S = lfb.Server(0, budget_mb << 20, max_active, chunk)
    ids = [S.submit(m.V, m.F, s, steps, rounds, dual, op) for m, s, op, steps, rounds, dual in jobs]
    S.run()
    in_use, peak = S.memory()
    assert in_use == 0
    assert peak <= budget_mb << 20
    for i, (m, s, op, steps, rounds, dual) in zip(ids, jobs):
        r = S.result(i)
        ref = _solo_job(lfb, ctx, m, s, op, steps, rounds, dual, None)
        assert r["steps"] == steps * (rounds + 1)
        assert np.array_equal(r["seeds"], ref["seeds"]), f"job {i} seeds"
        assert np.array_equal(r["labels"], ref["labels"]), f"job {i} labels"
        assert np.array_equal(r["tris"], ref["tris"]), f"job {i} triangles"
        assert r["latency_ms"] >= r["queue_ms"] >= 0
        S.release(i)
    S.close()


def test_full_size_c4_batch_equals_solo(lf):
    """The benchmark's batch at full size (256 torus grids, 6.1 M vertices,
    graph operator, 500 steps): eight meshes spread over the batch, from the
    smallest to the largest, are bit-identical to their solo runs."""
    lfb, ctx = lf
    items = I.batch_tori(256)
    say("c4 batch", sum(m.n_v for m, _ in items), "vertices")
    B = lfb.Batch(ctx, [(m.V, m.F) for m, _ in items], 0, [s for _, s in items])
    B.step(500)
    order = np.argsort([m.n_v for m, _ in items])
    pick = sorted(set(int(order[k]) for k in np.linspace(0, len(items) - 1, 8).round().astype(int)))
    for k in pick:
        mesh, seeds = items[k]
        M, f = _solo_fields(lfb, ctx, mesh, seeds, 0, None, 500)
        assert _same_csr(B.export(k), f.export()), f"mesh {k} ({mesh.n_v} vertices) differs"
        assert np.array_equal(B.labels(k), f.labels())
        f.close()
        M.close()
    B.close()


def test_server_cancel(lf):
    """Cancelling an active job (after its first chunk is in flight) and a
    queued one: their memory is released, their results fail, and the other
    jobs compute exactly what they compute alone."""
    lfb, ctx = lf
    jobs = _jobs()[:3]
    S = lfb.Server(0, 4096 << 20, 1, 8)
    ids = [S.submit(m.V, m.F, s, steps, rounds, dual, op) for m, s, op, steps, rounds, dual in jobs]
    say("server cancel")
    S.poll()  # admits the first job and issues its first chunk
    S.cancel(ids[0])
    S.cancel(ids[2])
    assert S.memory()[0] == 0
    S.run()
    for i in (ids[0], ids[2]):
        with pytest.raises(lfb.LFError):
            S.result(i)
        S.release(i)
    m, s, op, steps, rounds, dual = jobs[1]
    r = S.result(ids[1])
    ref = _solo_job(lfb, ctx, m, s, op, steps, rounds, dual, None)
    assert np.array_equal(r["labels"], ref["labels"]) and np.array_equal(r["seeds"], ref["seeds"])
    assert np.array_equal(r["tris"], ref["tris"])
    with pytest.raises(lfb.LFError):
        S.cancel(ids[1])  # finished
    S.release(ids[1])
    assert S.memory()[0] == 0
    S.close()
