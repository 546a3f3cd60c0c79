"""Input generators: counts, closedness, seeds (no method arithmetic here)."""
import numpy as np

from paper_1804_09152_amd import inputs as I


def _euler(m):
    e = np.concatenate([m.F[:, [0, 1]], m.F[:, [1, 2]], m.F[:, [2, 0]]])
    k = e[:, 0].astype(np.int64) * m.n_v + e[:, 1]
    assert np.unique(k).size == k.size  # consistently oriented, no duplicate faces
    # closed: every directed edge has its reverse
    rk = e[:, 1].astype(np.int64) * m.n_v + e[:, 0]
    assert np.isin(rk, k).all()
    return m.n_v - k.size // 2 + m.n_f


def test_torus_counts_and_topology():
    m = I.torus_grid(64, 64)
    assert (m.n_v, m.n_f) == (4096, 8192)
    assert _euler(m) == 0


def test_icosphere_counts_and_topology():
    for level in range(4):
        m = I.icosphere(level)
        assert m.n_v == 10 * 4 ** level + 2 and m.n_f == 20 * 4 ** level
        assert _euler(m) == 2
        assert np.allclose(np.linalg.norm(m.V, axis=1), 1.0)


def test_config_sizes():
    m, s = I.config_c1()
    assert m.n_v == 4096 and s.size == 32 and np.unique(s).size == 32
    m, s = I.config_c2(level=3, n_seeds=16)
    assert m.n_v == 642 and np.unique(s).size == 16


def test_sh_displacement_amplitude():
    m = I.sh_displace(I.icosphere(3), np.random.default_rng(1))
    r = np.linalg.norm(m.V, axis=1)
    assert abs(np.abs(r - 1.0).max() - 0.2) < 1e-12


def test_synthetic_state_rows():
    m, s = I.config_c2(level=3, n_seeds=16)
    ptr, col, val = I.synthetic_state(m, s, np.random.default_rng(0))
    assert ptr[-1] == col.size == val.size
    sums = np.add.reduceat(val, ptr[:-1])
    assert np.allclose(sums, 1.0) and (val > 0).all()
    for i in range(m.n_v):
        c = col[ptr[i]:ptr[i + 1]]
        assert (np.diff(c) > 0).all() and c.max() <= 16


def test_batch_and_jobs():
    b = I.batch_tori(8, seed=3)
    assert len(b) == 8 and all(1 <= s.size <= m.n_v for m, s in b)
    jobs = I.serving_jobs(10)
    assert all(j["n_seeds"] == 64 * 4 ** (j["level"] - 5) for j in jobs)
