"""Seeded synthetic inputs: meshes, seed vertices and field states.

This module is the only code shared by the HIP path and the FP64 oracle, and it
holds none of the method's arithmetic: no operator, no field update, no
labelling, no Lloyd step and no dual-mesh logic.  It only produces the inputs
the method starts from (a closed triangle mesh and distinct seed vertices), plus
a plausible mid-run field matrix used to drive one-step comparisons at full
size.

The paper's own meshes (scans and artist models of 54k to 21.4M triangles,
Section 7, Table 2) are not available; closed tori and icospheres of the same
vertex counts stand in for them.  Every generator takes a seed and is fully
deterministic.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Mesh",
    "torus_grid",
    "icosphere",
    "jitter",
    "sh_displace",
    "seeds_uniform",
    "config_c1",
    "config_c2",
    "config_c3",
    "batch_tori",
    "serving_jobs",
    "synthetic_state",
    "morton_order",
    "permute_mesh",
]


@dataclasses.dataclass
class Mesh:
    """A closed triangle mesh.  V: float64 (n_v, 3); F: int32 (n_f, 3)."""

    V: np.ndarray
    F: np.ndarray
    name: str = ""

    @property
    def n_v(self) -> int:
        return int(self.V.shape[0])

    @property
    def n_f(self) -> int:
        return int(self.F.shape[0])


def torus_grid(nx: int, ny: int, R: float = 3.0, r: float = 1.0) -> Mesh:
    """Regular triangulated torus with nx*ny vertices, vertex id = x + nx*y.

    Faces are (a,b,c) and (a,c,d) with a=(x,y), b=(x+1,y), c=(x+1,y+1),
    d=(x,y+1), indices taken modulo the grid.  The grid is embedded in R^3 as a
    ring torus (major radius R, minor radius r) so that geometric stages have
    positions to work with; the graph operator ignores them.
    """
    x, y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    x = x.ravel()
    y = y.ravel()
    th = 2.0 * np.pi * x / nx
    ph = 2.0 * np.pi * y / ny
    V = np.stack([(R + r * np.cos(ph)) * np.cos(th),
                  (R + r * np.cos(ph)) * np.sin(th),
                  r * np.sin(ph)], axis=1).astype(np.float64)

    def vid(xx, yy):
        return (xx % nx) + nx * (yy % ny)

    a = vid(x, y)
    b = vid(x + 1, y)
    c = vid(x + 1, y + 1)
    d = vid(x, y + 1)
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 0)
    # interleave so that the two triangles of a grid square are adjacent ids
    F = F.reshape(2, -1, 3).transpose(1, 0, 2).reshape(-1, 3)
    return Mesh(V, F.astype(np.int32), f"torus{nx}x{ny}")


_ICO_V = None


def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    F = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    return V, F


def icosphere(level: int) -> Mesh:
    """Unit icosphere: icosahedron, `level` rounds of 4-way midpoint subdivision,
    vertices pushed back to the unit sphere after every round.

    n_v = 10*4^level + 2, n_f = 20*4^level.  New (midpoint) vertices are
    appended after the old ones, in order of their sorted edge keys.
    """
    V, F = _icosahedron()
    for _ in range(level):
        nv = V.shape[0]
        e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], 0)
        e.sort(axis=1)
        key = e[:, 0] * nv + e[:, 1]
        uk, inv = np.unique(key, return_inverse=True)
        a = uk // nv
        b = uk % nv
        M = 0.5 * (V[a] + V[b])
        M /= np.linalg.norm(M, axis=1, keepdims=True)
        mid = (nv + inv).reshape(3, -1)  # midpoints of edges (0,1), (1,2), (2,0)
        m01, m12, m20 = mid[0], mid[1], mid[2]
        v0, v1, v2 = F[:, 0], F[:, 1], F[:, 2]
        F = np.concatenate([np.stack([v0, m01, m20], 1), np.stack([v1, m12, m01], 1),
                            np.stack([v2, m20, m12], 1), np.stack([m01, m12, m20], 1)], 0)
        V = np.concatenate([V, M], 0)
    return Mesh(V.astype(np.float64), F.astype(np.int32), f"icosphere{level}")


def mean_edge_length(mesh: Mesh) -> float:
    V, F = mesh.V, mesh.F
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], 0)
    return float(np.linalg.norm(V[e[:, 0]] - V[e[:, 1]], axis=1).mean())


def jitter(mesh: Mesh, rng: np.random.Generator, rel: float = 0.1) -> Mesh:
    """Add i.i.d. N(0, (rel * mean edge length)^2) noise to every coordinate."""
    s = rel * mean_edge_length(mesh)
    V = mesh.V + rng.normal(0.0, s, size=mesh.V.shape)
    return Mesh(V, mesh.F.copy(), mesh.name + "_jit")


def _real_sh(l: int, m: int, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Real spherical harmonic of degree l, order m (theta polar, phi azimuth)."""
    from scipy.special import sph_harm_y
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    Y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2.0) * (-1) ** m * np.real(Y)
    return math.sqrt(2.0) * (-1) ** m * np.imag(Y)


def sh_displace(mesh: Mesh, rng: np.random.Generator, k: int = 8, lmax: int = 4,
                amplitude: float = 0.2) -> Mesh:
    """Radial displacement r = 1 + sum_k c_k Y_{l_k m_k}, l_k ~ U{1..lmax},
    m_k ~ U{-l..l}, c_k ~ U(-1, 1), the sum rescaled so max |sum| = amplitude.
    Vertices are assumed to lie on the unit sphere."""
    V = mesh.V
    theta = np.arccos(np.clip(V[:, 2], -1.0, 1.0))
    phi = np.arctan2(V[:, 1], V[:, 0])
    s = np.zeros(V.shape[0])
    for _ in range(k):
        l = int(rng.integers(1, lmax + 1))
        m = int(rng.integers(-l, l + 1))
        c = float(rng.uniform(-1.0, 1.0))
        s += c * _real_sh(l, m, theta, phi)
    s *= amplitude / max(np.abs(s).max(), 1e-300)
    return Mesh(V * (1.0 + s)[:, None], mesh.F.copy(), mesh.name + "_sh")


def seeds_uniform(n_v: int, k: int, rng: np.random.Generator) -> np.ndarray:
    """k distinct seed vertices drawn uniformly without replacement."""
    return rng.choice(n_v, size=k, replace=False).astype(np.int32)


def morton_order(V: np.ndarray, bits: int = 10) -> np.ndarray:
    """Permutation that sorts vertices along a 3D Morton (Z-order) curve."""
    lo = V.min(0)
    span = np.maximum(V.max(0) - lo, 1e-300)
    q = np.clip(((V - lo) / span * ((1 << bits) - 1)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(V.shape[0], dtype=np.int64)
    for b in range(bits):
        for d in range(3):
            code |= ((q[:, d] >> b) & 1) << (3 * b + d)
    return np.argsort(code, kind="stable")


def permute_mesh(mesh: Mesh, order: np.ndarray) -> tuple[Mesh, np.ndarray]:
    """Relabel vertices so that new id k is old vertex order[k].
    Returns the mesh and the old->new map."""
    inv = np.empty_like(order)
    inv[order] = np.arange(order.size)
    return Mesh(mesh.V[order], inv[mesh.F].astype(np.int32), mesh.name + "_perm"), inv


# --- the five workloads --------------------------------------------------------

def config_c1():
    """64x64 torus grid, graph operator, 32 seeds from default_rng(0)."""
    mesh = torus_grid(64, 64)
    seeds = seeds_uniform(mesh.n_v, 32, np.random.default_rng(0))
    return mesh, seeds


def config_c2(level: int = 7, n_seeds: int = 1024, seed: int = 0):
    """Jittered icosphere (level 7: 163,842 vertices), 1,024 seeds.
    Jitter draws first, then the seeds, from one default_rng(seed) stream."""
    rng = np.random.default_rng(seed)
    mesh = jitter(icosphere(level), rng)
    seeds = seeds_uniform(mesh.n_v, n_seeds, rng)
    return mesh, seeds


def config_c3(level: int = 9, n_seeds: int = 16384, seed: int = 0):
    """Icosphere (level 9: 2,621,442 vertices) displaced by 8 random real
    spherical harmonics of degree 1..4 (max amplitude 0.2), 16,384 seeds."""
    rng = np.random.default_rng(seed)
    mesh = sh_displace(icosphere(level), rng)
    seeds = seeds_uniform(mesh.n_v, n_seeds, rng)
    return mesh, seeds


def batch_tori(count: int = 256, seed: int = 0, nv_lo: float = 1e3, nv_hi: float = 1e5,
               s_lo: float = 8, s_hi: float = 512):
    """Uneven batch: vertex counts log-uniform in [nv_lo, nv_hi] (nx = round(sqrt
    n_v), ny = round(n_v/nx)), seed counts round(log-uniform[s_lo, s_hi])."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        nv = math.exp(rng.uniform(math.log(nv_lo), math.log(nv_hi)))
        nx = max(3, int(round(math.sqrt(nv))))
        ny = max(3, int(round(nv / nx)))
        k = int(round(math.exp(rng.uniform(math.log(s_lo), math.log(s_hi)))))
        mesh = torus_grid(nx, ny)
        k = min(k, mesh.n_v)
        out.append((mesh, seeds_uniform(mesh.n_v, k, rng)))
    return out


def serving_jobs(count: int, seed: int = 0, levels=(5, 6, 7, 8, 9)):
    """Job descriptions for the serving stream: level ~ U{levels}, jittered
    icosphere, 64 * 4^(level-5) seeds (about 160 vertices per cell)."""
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(count):
        level = int(rng.choice(levels))
        jobs.append({"id": j, "level": level, "n_seeds": 64 * 4 ** (level - 5),
                     "seed": int(rng.integers(0, 2 ** 31 - 1))})
    return jobs


def synthetic_state(mesh: Mesh, seeds: np.ndarray, rng: np.random.Generator,
                    band: float = 0.35, base_frac: float = 0.3, k: int = 3):
    """A plausible mid-run field matrix U (n_v x (n_s+1), CSR, rows = vertices,
    last column = base layer) for one-step comparisons.

    Built only from Euclidean nearest-seed assignment: each vertex takes its
    nearest seed's layer with weight 1; up to k-1 further seeds whose distance
    is within (1 + band) of the nearest get a weight in [0.2, 0.9] (bands and
    junctions); in a random fraction of the cells (still "growing") half the
    vertices also keep some base layer.  Rows are normalised to sum 1,
    columns ascending.  Returns (rowptr int64, col int32, val float64).
    """
    from scipy.spatial import cKDTree
    n_v = mesh.n_v
    n_s = int(seeds.size)
    k = max(1, min(k, n_s))
    dist, idx = cKDTree(mesh.V[seeds]).query(mesh.V, k=k)
    dist = np.asarray(dist, dtype=np.float64).reshape(n_v, k)
    idx = np.asarray(idx, dtype=np.int64).reshape(n_v, k)
    w = rng.uniform(0.2, 0.9, size=(n_v, k))
    w[:, 0] = 1.0
    keep = np.ones((n_v, k), dtype=bool)
    keep[:, 1:] = (dist[:, 1:] - dist[:, :1]) < band * np.maximum(dist[:, :1], 1e-12)
    growing = rng.random(n_s) < base_frac
    has_base = growing[idx[:, 0]] & (dist[:, 0] > 0) & (rng.random(n_v) < 0.5)
    bw = rng.uniform(0.05, 0.9, size=n_v)
    cols = np.concatenate([np.where(keep, idx, n_s + 1), np.where(has_base, n_s, n_s + 1)[:, None]], 1)
    vals = np.concatenate([np.where(keep, w, 0.0), np.where(has_base, bw, 0.0)[:, None]], 1)
    order = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, 1)
    vals = np.take_along_axis(vals, order, 1)
    vals /= vals.sum(1, keepdims=True)
    valid = cols <= n_s
    rowptr = np.zeros(n_v + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(valid.sum(1))
    return rowptr, cols[valid].astype(np.int32), vals[valid]
