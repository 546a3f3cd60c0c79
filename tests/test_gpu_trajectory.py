"""GPU against the FP64 oracle on the workloads' own trajectories: the
icosphere level 7 job (1,000 free-running steps, five Lloyd rounds taken from
the oracle's seeds, dual mesh), the icosphere level 9 job (free-running steps
from its seeds, a teacher-forced step, re-seeding and dual mesh on the
oracle's state), meshes of the 256-torus batch, and jobs run by the server.
The oracle runs on every host thread (rows in blocks; results identical to
one thread)."""
import os

import numpy as np
import pytest

from paper_1804_09152_amd import inputs as I
from tests.gpu_common import as_oracle, check_step, f32, gpu_load, row_compare, say
from tests.test_gpu_post import _csr_pairs, check_dual

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def lf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_09152_amd as lfb
    lfb.load()
    yield lfb, lfb.Context(0)


def compare_free(G, U, lab_g, orc, n_s, what):
    """Free-running GPU fields G (float32) against the oracle's U (float64):
    identical patterns on every row, values within TOL, identical labels
    wherever the oracle's top-two gap exceeds TOL."""
    pat, diff = row_compare(as_oracle(G), U)
    assert pat.all(), f"{what}: pattern differs on {(~pat).sum()} rows, e.g. {np.nonzero(~pat)[0][:5]}"
    worst = float(diff.max())
    assert worst <= TOL, f"{what}: max |dphi| {worst}"
    lab_o, gap = orc.labels(U, n_s)
    clear = gap > TOL
    assert np.array_equal(lab_g[clear], lab_o[clear]), f"{what}: labels differ"
    say(what, f"max |dphi| {worst:.3g}, {int((~clear).sum())} tied labels")


def lloyd_compare(f, orc, mesh, U, seeds, what):
    """Re-seeding on the same float32 state: identical new seeds and
    statuses at every cell whose decisions are clear of ties."""
    Uf = f32(U)
    gpu_load(f, Uf)
    new_g, st_g = f.lloyd_reseed()
    new_o, st_o, mg = orc.lloyd(mesh.V, mesh.F, Uf, seeds)
    clear = mg > 1e-9
    assert clear.mean() > 0.99, f"{what}: {int((~clear).sum())} guarded cells"
    assert np.array_equal(new_g[clear], new_o[clear]), f"{what}: seeds differ"
    assert np.array_equal(st_g[clear], st_o[clear])
    say(what, f"{int((new_o != seeds).sum())} seeds moved, {int((~clear).sum())} guarded")
    return new_o


def dual_compare(f, orc, mesh, U, seeds, what):
    Uf = f32(U)
    gpu_load(f, Uf)
    tris, adj = f.dual_mesh(0.25)
    d = orc.dual_mesh(mesh.V, mesh.F, Uf, seeds, 0.25)
    assert _csr_pairs(*f.dual_matrix(0)) == _csr_pairs(*d["A_v"])
    assert _csr_pairs(*f.dual_matrix(1)) == _csr_pairs(*d["A_t"])
    pairs, state = f.dual_candidates()
    assert np.array_equal(pairs, d["cand"])
    clear = d["cand_margin"] > 1e-12
    assert np.array_equal(state[clear], d["cand_state"][clear])
    guarded = {(int(p), int(q)) for p, q in d["cand"][~clear]}
    differ = check_dual(tris, adj, d, guarded)
    say(what, f"{len(d['tri'])} triangles, {d['n_removed']} spurious removed, "
              f"{len(guarded)} guarded pairs, {differ} triangles differ")
    return d


def test_c2_job_against_oracle(lf, orc):
    """Icosphere level 7 (163,842 vertices), 1,024 seeds, cotangent
    operator: 1,000 free-running steps; then five Lloyd rounds, each
    re-seeded from the oracle's state on both sides (compared) and continued
    from the oracle's seeds for 1,000 free-running steps (compared); then the
    dual mesh of the final state."""
    lfb, ctx = lf
    mesh, seeds = I.config_c2()
    k = seeds.size
    th = orc.host_threads()
    P = orc.default_params()
    L = orc.operator(mesh.V, mesh.F, 1)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, lfb.LF_OP_COTAN)
    f = lfb.Fields(m, seeds)
    g = lfb.Fields(m, seeds)  # for the teacher-forced re-seeding and dual mesh
    say("c2 job: 1000 steps")
    U, _ = orc.run(L, orc.init(mesh.n_v, seeds), k, P, 1000, threads=th)
    f.step(1000)
    compare_free(f.export(), U, f.labels(), orc, k, "c2 t=1000")
    for r in range(5):
        seeds = lloyd_compare(g, orc, mesh, U, seeds, f"c2 Lloyd round {r + 1}")
        f.reset(seeds)
        U, _ = orc.run(L, orc.init(mesh.n_v, seeds), k, P, 1000, threads=th)
        f.step(1000)
        compare_free(f.export(), U, f.labels(), orc, k, f"c2 round {r + 1} t=1000")
    dual_compare(g, orc, mesh, U, seeds, "c2 dual mesh")


def test_c3_job_against_oracle(lf, orc):
    """Icosphere level 9 (2,621,442 vertices), 16,384 seeds, cotangent
    operator (the benchmark's job): 250 free-running steps from the seeds
    (the fields have spread over the whole surface and the entry count has
    settled), a teacher-forced step from the oracle's state, re-seeding and
    dual mesh on it."""
    lfb, ctx = lf
    mesh, seeds = I.config_c3()
    k = seeds.size
    th = orc.host_threads()
    P = orc.default_params()
    say("c3 job: operator")
    L = orc.operator(mesh.V, mesh.F, 1)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, lfb.LF_OP_COTAN)
    f = lfb.Fields(m, seeds)
    g = lfb.Fields(m, seeds)
    say("c3 job: 250 steps")
    U, _ = orc.run(L, orc.init(mesh.n_v, seeds), k, P, 250, threads=th)
    f.step(250)
    compare_free(f.export(), U, f.labels(), orc, k, "c3 t=250")
    Uf = f32(U)
    gpu_load(g, Uf)
    g.step(1)
    O, info = orc.step(L, Uf, k, P, want_info=True, threads=th)
    check_step(as_oracle(g.export()), O, info, P["theta"], what="c3 teacher-forced t=250")
    lloyd_compare(g, orc, mesh, U, seeds, "c3 Lloyd")
    d = dual_compare(g, orc, mesh, U, seeds, "c3 dual mesh")
    assert d["n_removed"] > 0  # the spurious-triangle rule fires on this state


@pytest.mark.skipif(os.environ.get("LF_LONG") != "1",
                    reason="2,000 oracle steps on 2.6 M vertices take about six minutes of host "
                           "time; run with LF_LONG=1")
def test_c3_full_job_against_oracle(lf, orc):
    """The benchmark's whole job, 2,000 free-running steps from the seeds,
    compared at steps 250, 1,000 and 2,000 with teacher-forced steps from the
    oracle's states there, then re-seeding and dual mesh at step 2,000."""
    lfb, ctx = lf
    mesh, seeds = I.config_c3()
    k = seeds.size
    th = orc.host_threads()
    P = orc.default_params()
    L = orc.operator(mesh.V, mesh.F, 1)
    m = lfb.Mesh(ctx, mesh.V, mesh.F, lfb.LF_OP_COTAN)
    f = lfb.Fields(m, seeds)
    g = lfb.Fields(m, seeds)
    U = orc.init(mesh.n_v, seeds)
    done = 0
    for t in (250, 1000, 2000):
        while done < t:  # the oracle in runs of 250 steps, each reported
            n = min(250, t - done)
            U, _ = orc.run(L, U, k, P, n, threads=th)
            f.step(n)
            done += n
            say(f"c3 full job: step {done} on both sides")
        compare_free(f.export(), U, f.labels(), orc, k, f"c3 t={t}")
        Uf = f32(U)
        gpu_load(g, Uf)
        g.step(1)
        O, info = orc.step(L, Uf, k, P, want_info=True, threads=th)
        check_step(as_oracle(g.export()), O, info, P["theta"], what=f"c3 teacher-forced t={t}")
    lloyd_compare(g, orc, mesh, U, seeds, "c3 Lloyd at 2000")
    dual_compare(g, orc, mesh, U, seeds, "c3 dual mesh at 2000")


def test_c4_batch_meshes_against_oracle(lf, orc):
    """The 256-torus batch (6.1 M vertices, graph operator) stepped 500 times
    as one field object: eight meshes from the smallest to the largest
    against their own oracle runs."""
    lfb, ctx = lf
    items = I.batch_tori(256)
    P = orc.default_params()
    say("c4 batch against the oracle")
    B = lfb.Batch(ctx, [(mm.V, mm.F) for mm, _ in items], lfb.LF_OP_GRAPH, [s for _, s in items])
    B.step(500)
    order = np.argsort([mm.n_v for mm, _ in items])
    pick = sorted(set(int(order[q]) for q in np.linspace(0, len(items) - 1, 8).round().astype(int)))
    th = orc.host_threads()
    for q in pick:
        mesh, seeds = items[q]
        L = orc.operator(mesh.V, mesh.F, 0)
        U, _ = orc.run(L, orc.init(mesh.n_v, seeds), seeds.size, P, 500, threads=th)
        compare_free(B.export(q), U, B.labels(q), orc, seeds.size,
                     f"batch mesh {q} ({mesh.n_v} vertices, {seeds.size} seeds)")
    B.close()


def _oracle_job(orc, mesh, seeds, steps, rounds, th):
    """The server's recipe on the oracle: steps, then rounds x (re-seed,
    re-initialise, steps), labels, dual mesh.  Returns None if a re-seeding
    decision was a near-tie (the float32 run may then take the other seed)."""
    P = orc.default_params()
    L = orc.operator(mesh.V, mesh.F, 1)
    U, _ = orc.run(L, orc.init(mesh.n_v, seeds), seeds.size, P, steps, threads=th)
    for _ in range(rounds):
        seeds, _, mg = orc.lloyd(mesh.V, mesh.F, U, seeds)
        if (mg <= 1e-9).any():
            return None
        U, _ = orc.run(L, orc.init(mesh.n_v, seeds), seeds.size, P, steps, threads=th)
    return U, seeds, orc.dual_mesh(mesh.V, mesh.F, U, seeds, 0.25)


def test_served_jobs_against_oracle(lf, orc):
    """Jobs run by the server side by side (their steps in shared launches)
    against the oracle running each job's recipe alone: final seeds, labels
    and dual triangles."""
    lfb, ctx = lf
    th = orc.host_threads()
    jobs = []
    for lv, seed in ((5, 3), (5, 4), (6, 5)):
        rng = np.random.default_rng(seed)
        mesh = I.jitter(I.icosphere(lv), rng)
        jobs.append((mesh, I.seeds_uniform(mesh.n_v, 64 * 4 ** (lv - 5), rng)))
    steps, rounds = 400, 2
    S = lfb.Server(0, 8 << 30, 8, 64)
    say("served jobs against the oracle")
    ids = [S.submit(mm.V, mm.F, s, steps, rounds, True, lfb.LF_OP_COTAN) for mm, s in jobs]
    S.run()
    ticks, launches = S.stats()
    assert launches < sum(steps * (rounds + 1) for _ in jobs)  # steps shared launches
    compared = 0
    for i, (mesh, seeds) in zip(ids, jobs):
        r = S.result(i)
        ref = _oracle_job(orc, mesh, seeds, steps, rounds, th)
        if ref is None:
            say("job", i, "has a near-tie re-seeding decision; not compared")
            continue
        U, s_o, d = ref
        assert np.array_equal(r["seeds"], s_o), f"job {i} seeds"
        lab_o, gap = orc.labels(U, seeds.size)
        clear = gap > TOL
        assert np.array_equal(r["labels"][clear], lab_o[clear]), f"job {i} labels"
        if (d["cand_margin"] > 1e-12).all():
            tg = {tuple(sorted(int(x) for x in t)) for t in r["tris"]}
            to = {tuple(sorted(int(x) for x in t)) for t in d["tri"]}
            assert tg == to, f"job {i} triangles"
        compared += 1
        S.release(i)
    assert compared >= 2
    S.close()
