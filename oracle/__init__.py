"""FP64 CPU oracle, Python side (ctypes over liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg load this package; the library and its binding never do.
It shares no code with the HIP path.  Functions return plain numpy arrays; a
field matrix is the CSR triple (ptr int64, col int32, val float64) with rows
= vertices and columns = cells 0..n_s-1 then the base layer n_s.

Parity status of each function (what pins it, see tests/test_oracle_*.py):
  operator   pinned: zero row sums, symmetry, degrees, equilateral weight
             1/sqrt(3), negative semi-definiteness, brute-force dense build.
  init       pinned: definition.
  step       pinned: brute-force dense Algorithm 1 on tiny meshes, closed-form
             identity, constant-field invariance, flooding, mirror symmetry,
             front speed, partition of unity, bounds.  With per-pair
             coefficients: brute-force dense Algorithm 1 with the typed
             coefficient matrices, one type equal to the scalar step bit for
             bit, invariance under relabelling the types.
  labels     pinned: definition on hand-built rows; Voronoi agreement.
  change     pinned: hand-computed two-step example (golden file), zero for a
             constant field and for a step onto itself.
  run_until  pinned: convergence reached on a lattice of seeds, later steps
             change nothing; Delta-t insensitivity (Section 7): labels after
             convergence agree across time steps 1 to 5.  Reading: with the
             theta prune the values can end in a period-2 oscillation of size
             about theta (entries near theta appear and vanish), and the first
             steps from seeds are quiet too (first-ring values are pruned), so
             convergence is a whole quiet chunk: labels and tau pattern fixed,
             values moving by at most eps (above that oscillation).
  init_regions pinned: single-vertex regions reproduce init(seeds); a
             region's vertices all start in its layer.
  init_rings pinned: rings = 0 is init(seeds); on the regular torus grid an
             isolated seed's regions hold 1, 7 and 19 vertices for 0, 1, 2
             rings (the triangular lattice's hexagonal rings); a vertex between
             two seeds goes to the lower index, a seed next to a lower seed
             keeps itself; the nearest seed wins over a lower index.
  lloyd      pinned: hand-built single-cell cases with known centroids and hit
             faces, a miss keeps the seed, collision rule cases.
  dual_mesh  pinned: hand-built adjacency cases, regular lattice on a torus
             (every dual vertex of degree 6, Euler characteristic 0), sphere
             case (Euler characteristic 2) against the convex hull of seeds;
             spurious-triangle removal (Section 5.2): six octahedral cells plus
             a small cell in one octant, whose known dual is the octahedron
             with the covered face replaced by the fan around the small cell
             (one triangle removed), and no removal without a cell of degree 3.
  step(threads > 1) pinned: identical, bit for bit, to the one-thread step
             (rows are independent; blocks joined in row order).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, IEEE arithmetic)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-fopenmp",
                               "-o", _SO, src, "-lm"])
    return _SO


class Params(C.Structure):
    _fields_ = [("w", C.c_double), ("a", C.c_double), ("e", C.c_double), ("mu", C.c_double),
                ("dt", C.c_double), ("theta", C.c_double), ("base_mode", C.c_int32),
                ("n_types", C.c_int32), ("types", C.POINTER(C.c_int32)),
                ("tab", C.POINTER(C.c_double))]


class _Dual(C.Structure):
    _fields_ = [("av_ptr", C.POINTER(C.c_int64)), ("av_col", C.POINTER(C.c_int32)),
                ("at_ptr", C.POINTER(C.c_int64)), ("at_col", C.POINTER(C.c_int32)),
                ("ad_ptr", C.POINTER(C.c_int64)), ("ad_col", C.POINTER(C.c_int32)),
                ("n_cand", C.c_int64), ("cand", C.POINTER(C.c_int32)),
                ("cand_state", C.POINTER(C.c_int32)), ("cand_margin", C.POINTER(C.c_double)),
                ("n_tri", C.c_int64), ("tri", C.POINTER(C.c_int32)),
                ("n_removed", C.c_int64), ("n_conflict", C.c_int64),
                ("n_nonmanifold", C.c_int64)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = C.CDLL(_SO)
        P = C.c_void_p
        lib.orc_free.argtypes = [P]
        lib.orc_operator.argtypes = [C.c_int32, P, C.c_int32, P, C.c_int32, P,
                                     C.POINTER(P), C.POINTER(P)]
        lib.orc_init.argtypes = [C.c_int32, P, C.c_int32, P, C.POINTER(P), C.POINTER(P)]
        lib.orc_init_rings.argtypes = [C.c_int32, C.c_int32, P, P, C.c_int32, C.c_int32, P,
                                       C.POINTER(P), C.POINTER(P)]
        lib.orc_step.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, P, C.POINTER(Params),
                                 P, C.POINTER(P), C.POINTER(P), P, P, P]
        lib.orc_step_threads.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, P,
                                         C.POINTER(Params), P, C.POINTER(P), C.POINTER(P), P, P,
                                         P, P, C.c_int32]
        lib.orc_labels.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P]
        lib.orc_lloyd.argtypes = [C.c_int32, P, C.c_int32, P, C.c_int32, P, P, P, P, P, P, P]
        lib.orc_dual_mesh.argtypes = [C.c_int32, P, C.c_int32, P, C.c_int32, P, P, P, P,
                                      C.c_double, C.POINTER(_Dual)]
        lib.orc_dual_free.argtypes = [C.POINTER(_Dual)]
        lib.orc_run_threads.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, P,
                                        C.POINTER(Params), C.c_int32, C.c_int32, P,
                                        C.POINTER(P), C.POINTER(P), P, P]
        for f in ("orc_operator", "orc_init", "orc_init_rings", "orc_step", "orc_step_threads", "orc_run_threads",
                  "orc_labels",
                  "orc_lloyd", "orc_dual_mesh"):
            getattr(lib, f).restype = C.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def _take(ptr, n, dtype):
    """Copy n elements out of a malloc'd C array and free it."""
    lib = _load()
    if n:
        arr = np.ctypeslib.as_array(C.cast(ptr, C.POINTER(np.ctypeslib.as_ctypes_type(dtype))),
                                    shape=(n,)).copy()
    else:
        arr = np.zeros(0, dtype=dtype)
    lib.orc_free(ptr)
    return arr


def default_params(**kw) -> dict:
    """Constants of the complete reading: w = 0.2 with a = w/5 (the paper's
    ratio of 5), e = 1, mu = 0.1, dt = 5 (Section 7), theta = 1e-3.
    Optional per-pair coefficients: types (int, one per layer, the base
    last) and table (n_types x n_types x 3: a, w, e of a pair of types)."""
    p = dict(w=0.2, a=0.04, e=1.0, mu=0.1, dt=5.0, theta=1e-3, base_mode=0)
    p.update(kw)
    return p


def _params(p: dict) -> Params:
    prm = Params(p["w"], p["a"], p["e"], p["mu"], p["dt"], p["theta"], int(p.get("base_mode", 0)), 0,
                 None, None)
    if p.get("types") is not None:
        types = np.ascontiguousarray(p["types"], dtype=np.int32)
        tab = np.ascontiguousarray(p["table"], dtype=np.float64)
        n_t = int(round(math.sqrt(tab.size // 3)))
        if tab.size != 3 * n_t * n_t:
            raise ValueError("table must hold n_types x n_types x 3 values")
        prm.n_types = n_t
        prm.types = types.ctypes.data_as(C.POINTER(C.c_int32))
        prm.tab = tab.ctypes.data_as(C.POINTER(C.c_double))
        prm._keep = (types, tab)  # the arrays live as long as the struct
    return prm


def _mesh(V, F):
    V = np.ascontiguousarray(V, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    return V, F


def operator(V, F, op: int):
    """Mesh Laplacian with diagonal (CSR, float64).  op 0 graph, 1 cotangent."""
    lib = _load()
    V, F = _mesh(V, F)
    n_v = V.shape[0]
    ptr = np.zeros(n_v + 1, dtype=np.int64)
    cp, vp = C.c_void_p(), C.c_void_p()
    _check(lib.orc_operator(n_v, _p(V), F.shape[0], _p(F), op, _p(ptr), C.byref(cp), C.byref(vp)),
           "operator")
    nnz = int(ptr[-1])
    return ptr, _take(cp, nnz, np.int32), _take(vp, nnz, np.float64)


def init(n_v: int, seeds):
    lib = _load()
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    ptr = np.zeros(n_v + 1, dtype=np.int64)
    cp, vp = C.c_void_p(), C.c_void_p()
    _check(lib.orc_init(n_v, _p(seeds), seeds.size, _p(ptr), C.byref(cp), C.byref(vp)), "init")
    return ptr, _take(cp, n_v, np.int32), _take(vp, n_v, np.float64)


def host_threads() -> int:
    """Threads for the row-block oracle: the host's CPUs, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def init_rings(n_v: int, F, seeds, rings: int):
    """Seeds grown by `rings` edge-rings: nearest seed, ties to the lowest
    index (breadth-first search from every seed)."""
    lib = _load()
    F = np.ascontiguousarray(F, dtype=np.int32)
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    ptr = np.zeros(n_v + 1, dtype=np.int64)
    cp, vp = C.c_void_p(), C.c_void_p()
    _check(lib.orc_init_rings(n_v, F.shape[0], _p(F), _p(seeds), seeds.size, rings, _p(ptr),
                              C.byref(cp), C.byref(vp)), "init_rings")
    return ptr, _take(cp, n_v, np.int32), _take(vp, n_v, np.float64)


def step(L, U, n_s: int, params: dict, want_info: bool = False, threads: int = 1):
    """One time step.  L, U: CSR triples.  Returns U' (and info dict with
    margin, smargin (rows-of-interest decisions only), skel, events).
    threads > 1 splits the rows into blocks run in parallel; the result is
    the same for any thread count."""
    lib = _load()
    Lp, Lc, Lv = (np.ascontiguousarray(L[0], np.int64), np.ascontiguousarray(L[1], np.int32),
                  np.ascontiguousarray(L[2], np.float64))
    Up, Uc, Uv = (np.ascontiguousarray(U[0], np.int64), np.ascontiguousarray(U[1], np.int32),
                  np.ascontiguousarray(U[2], np.float64))
    n_v = Lp.size - 1
    Op = np.zeros(n_v + 1, dtype=np.int64)
    margin = np.zeros(n_v, dtype=np.float64)
    smargin = np.zeros(n_v, dtype=np.float64)
    skel = np.zeros(n_v, dtype=np.int32)
    ev = np.zeros(1, dtype=np.int64)
    prm = _params(params)
    cp, vp = C.c_void_p(), C.c_void_p()
    rc = lib.orc_step_threads(n_v, n_s, _p(Lp), _p(Lc), _p(Lv), _p(Up), _p(Uc), _p(Uv),
                              C.byref(prm), _p(Op), C.byref(cp), C.byref(vp), _p(margin),
                              _p(smargin), _p(skel), _p(ev), int(threads))
    _check(rc, "step")
    nnz = int(Op[-1])
    out = (Op, _take(cp, nnz, np.int32), _take(vp, nnz, np.float64))
    if want_info:
        return out, {"margin": margin, "smargin": smargin, "skel": skel, "events": int(ev[0])}
    return out


def run(L, U, n_s: int, params: dict, steps: int, record=None, threads: int = 1):
    """Free-running steps; record(t, U) is called after every step if given
    (without it the steps loop in C)."""
    if record is None:
        lib = _load()
        Lp, Lc, Lv = (np.ascontiguousarray(L[0], np.int64), np.ascontiguousarray(L[1], np.int32),
                      np.ascontiguousarray(L[2], np.float64))
        Up, Uc, Uv = (np.ascontiguousarray(U[0], np.int64), np.ascontiguousarray(U[1], np.int32),
                      np.ascontiguousarray(U[2], np.float64))
        n_v = Lp.size - 1
        Op = np.zeros(n_v + 1, dtype=np.int64)
        sk = np.zeros(1, dtype=np.int64)
        ev = np.zeros(1, dtype=np.int64)
        prm = _params(params)
        cp, vp = C.c_void_p(), C.c_void_p()
        _check(lib.orc_run_threads(n_v, n_s, _p(Lp), _p(Lc), _p(Lv), _p(Up), _p(Uc), _p(Uv),
                                   C.byref(prm), int(steps), int(threads), _p(Op), C.byref(cp),
                                   C.byref(vp), _p(sk), _p(ev)), "run")
        nnz = int(Op[-1])
        out = (Op, _take(cp, nnz, np.int32), _take(vp, nnz, np.float64))
        return out, {"skel_total": int(sk[0]), "events": int(ev[0])}
    skel_total = 0
    events = 0
    for t in range(steps):
        U, info = step(L, U, n_s, params, want_info=True, threads=threads)
        skel_total += int(info["skel"].sum())
        events += info["events"]
        if record is not None:
            record(t + 1, U)
    return U, {"skel_total": skel_total, "events": events}


def change(U_old, U_new, n_s: int, tau: float = 0.25):
    """Change made by a step, from its definition: the number of rows whose
    label (argmax over the cell layers, lowest layer on ties, -1 for none)
    or whose set of layers at or above tau (Phibar, Section 5.1) differs,
    and max |U_new(i,l) - U_old(i,l)| over every (vertex, layer) pair
    (absent entries are 0).  Plain row loop."""
    Po, Co, Vo = U_old
    Pn, Cn, Vn = U_new

    def label(r):
        best, bv = -1, 0.0
        for c in sorted(r):
            if c < n_s and (best < 0 or r[c] > bv):
                best, bv = c, r[c]
        return best

    changed, dmax = 0, 0.0
    for i in range(len(Po) - 1):
        a = {int(c): float(v) for c, v in zip(Co[Po[i]:Po[i + 1]], Vo[Po[i]:Po[i + 1]])}
        b = {int(c): float(v) for c, v in zip(Cn[Pn[i]:Pn[i + 1]], Vn[Pn[i]:Pn[i + 1]])}
        if (label(a) != label(b)
                or {c for c in a if a[c] >= tau} != {c for c in b if b[c] >= tau}):
            changed += 1
        for c in set(a) | set(b):
            dmax = max(dmax, abs(b.get(c, 0.0) - a.get(c, 0.0)))
    return changed, dmax


def run_until(L, U, n_s: int, params: dict, max_steps: int, eps: float, check_every: int,
              tau: float = 0.25):
    """Steps until converged, the rule of the library's lf_step_until: steps
    run in chunks of check_every; the fields have converged at the end of the
    first whole chunk in which no step changed any row (label or tau
    pattern) and no value moved by more than eps.  Returns (U, steps_done,
    converged_at (1-based, 0 if none), per-step (changed, dmax))."""
    done, conv, hist = 0, 0, []
    while done < max_steps and not conv:
        m = min(check_every, max_steps - done)
        quiet = m == check_every
        for _ in range(m):
            U1 = step(L, U, n_s, params)
            c = change(U, U1, n_s, tau)
            hist.append(c)
            quiet = quiet and c[0] == 0 and c[1] <= eps
            U = U1
        done += m
        if quiet:
            conv = done
    return U, done, conv, hist


def init_regions(n_v: int, region_ptr, region_vertices):
    """Initial fields from initial regions (Algorithm 1, first line: "seeds
    and/or initial regions"): U(v, k) = 1 for every vertex v of region k,
    U(v, base) = 1 for every other vertex; regions must be disjoint."""
    n_s = len(region_ptr) - 1
    owner = np.full(n_v, n_s, dtype=np.int32)
    for k in range(n_s):
        for v in region_vertices[region_ptr[k]:region_ptr[k + 1]]:
            if owner[v] != n_s:
                raise ValueError("regions overlap")
            owner[v] = k
    return np.arange(n_v + 1, dtype=np.int64), owner, np.ones(n_v)


def labels(U, n_s: int):
    lib = _load()
    Up, Uc, Uv = (np.ascontiguousarray(U[0], np.int64), np.ascontiguousarray(U[1], np.int32),
                  np.ascontiguousarray(U[2], np.float64))
    n_v = Up.size - 1
    lab = np.zeros(n_v, dtype=np.int32)
    gap = np.zeros(n_v, dtype=np.float64)
    _check(lib.orc_labels(n_v, n_s, _p(Up), _p(Uc), _p(Uv), _p(lab), _p(gap)), "labels")
    return lab, gap


def lloyd(V, F, U, seeds):
    """One re-seeding.  Returns (new seeds, status, margin)."""
    lib = _load()
    V, F = _mesh(V, F)
    Up, Uc, Uv = (np.ascontiguousarray(U[0], np.int64), np.ascontiguousarray(U[1], np.int32),
                  np.ascontiguousarray(U[2], np.float64))
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    n_s = seeds.size
    out = np.zeros(n_s, dtype=np.int32)
    st = np.zeros(n_s, dtype=np.int32)
    mg = np.zeros(n_s, dtype=np.float64)
    _check(lib.orc_lloyd(V.shape[0], _p(V), F.shape[0], _p(F), n_s, _p(Up), _p(Uc), _p(Uv),
                         _p(seeds), _p(out), _p(st), _p(mg)), "lloyd")
    return out, st, mg


def dual_mesh(V, F, U, seeds, tau: float = 0.25) -> dict:
    lib = _load()
    V, F = _mesh(V, F)
    Up, Uc, Uv = (np.ascontiguousarray(U[0], np.int64), np.ascontiguousarray(U[1], np.int32),
                  np.ascontiguousarray(U[2], np.float64))
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    n_s = seeds.size
    d = _Dual()
    _check(lib.orc_dual_mesh(V.shape[0], _p(V), F.shape[0], _p(F), n_s, _p(Up), _p(Uc), _p(Uv),
                             _p(seeds), tau, C.byref(d)), "dual_mesh")

    def csr(pp, cc):
        ptr = np.ctypeslib.as_array(pp, shape=(n_s + 1,)).copy()
        col = np.ctypeslib.as_array(cc, shape=(max(int(ptr[-1]), 1),))[: int(ptr[-1])].copy()
        return ptr, col

    res = {
        "A_v": csr(d.av_ptr, d.av_col),
        "A_t": csr(d.at_ptr, d.at_col),
        "A_d": csr(d.ad_ptr, d.ad_col),
        "n_removed": int(d.n_removed),
        "n_conflict": int(d.n_conflict),
        "n_nonmanifold": int(d.n_nonmanifold),
    }
    nc = int(d.n_cand)
    res["cand"] = (np.ctypeslib.as_array(d.cand, shape=(2 * nc,)).reshape(nc, 2).copy()
                   if nc else np.zeros((0, 2), np.int32))
    res["cand_state"] = np.ctypeslib.as_array(d.cand_state, shape=(nc,)).copy() if nc else np.zeros(0, np.int32)
    res["cand_margin"] = np.ctypeslib.as_array(d.cand_margin, shape=(nc,)).copy() if nc else np.zeros(0)
    nt = int(d.n_tri)
    res["tri"] = (np.ctypeslib.as_array(d.tri, shape=(3 * nt,)).reshape(nt, 3).copy()
                  if nt else np.zeros((0, 3), np.int32))
    lib.orc_dual_free(C.byref(d))
    return res


def to_dense(U, n_cols: int) -> np.ndarray:
    """CSR triple -> dense (rows x n_cols) float64 array (small cases only)."""
    ptr, col, val = U
    n = ptr.size - 1
    D = np.zeros((n, n_cols))
    for i in range(n):
        D[i, col[ptr[i]:ptr[i + 1]]] = val[ptr[i]:ptr[i + 1]]
    return D
