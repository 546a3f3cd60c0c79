"""Python binding of liblf.so, the gfx950 layered-field library.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  The functions `lf_*` mirror the C ABI in include/lf.h one to
one (same names, same arguments, a handle in place of an out-pointer);
`Context`, `Mesh` and `Fields` are small owners of those handles.  PyTorch
provides device memory (tensors passed by data_ptr) and streams.

There is no fallback: if liblf.so is missing or fails to load, every call
raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os

import numpy as np

__all__ = ["LFError", "load", "Context", "Mesh", "Batch", "Fields", "Server", "default_params",
           "LF_OP_GRAPH", "LF_OP_COTAN"]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblf.so")
LF_OP_GRAPH = 0
LF_OP_COTAN = 1
_STATUS = {0: "LF_OK", 1: "LF_EINVAL", 2: "LF_ENOMEM", 3: "LF_EDEVICE", 4: "LF_ECAPACITY",
           5: "LF_EBUSY", 6: "LF_ENOSYS"}


class LFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class lf_params(C.Structure):
    _fields_ = [("w", C.c_double), ("a", C.c_double), ("e", C.c_double), ("mu", C.c_double),
                ("dt", C.c_double), ("theta", C.c_double), ("tau", C.c_double),
                ("base_mode", C.c_int32), ("pad_", C.c_int32), ("capacity_hint", C.c_int64)]


class lf_job(C.Structure):
    _fields_ = [("V", C.c_void_p), ("F", C.c_void_p), ("seeds", C.c_void_p),
                ("n_v", C.c_int32), ("n_f", C.c_int32), ("n_s", C.c_int32), ("op", C.c_int32),
                ("steps", C.c_int32), ("lloyd_rounds", C.c_int32), ("dual_mesh", C.c_int32),
                ("pad_", C.c_int32), ("params", lf_params), ("conv_eps", C.c_double),
                ("conv_every", C.c_int32), ("n_types", C.c_int32),
                ("layer_types", C.c_void_p), ("table", C.c_void_p)]


EXPORTS = [
    "lf_last_error", "lf_params_default", "lf_ctx_create", "lf_ctx_destroy", "lf_mesh_create",
    "lf_mesh_destroy", "lf_mesh_operator", "lf_fields_create", "lf_fields_destroy",
    "lf_fields_reset", "lf_fields_create_rings", "lf_fields_create_regions", "lf_fields_reset_regions", "lf_fields_seeds", "lf_fields_set_coefficients", "lf_step", "lf_sync", "lf_fields_use_graphs", "lf_fields_set_reorder", "lf_fields_reorders", "lf_fields_export",
    "lf_fields_import", "lf_labels", "lf_step_until", "lf_last_change", "lf_lloyd_reseed", "lf_lloyd", "lf_dual_mesh", "lf_dual_matrix",
    "lf_dual_candidates", "lf_stats", "lf_traffic", "lf_step_timing", "lf_step_async",
    "lf_batch_create", "lf_batch_destroy", "lf_batch_fields", "lf_batch_export", "lf_batch_labels",
    "lf_server_create", "lf_server_destroy", "lf_server_submit", "lf_server_poll", "lf_server_cancel",
    "lf_server_result", "lf_server_release", "lf_server_memory", "lf_server_times",
    "lf_server_stats",
]

_lib = None
_exiting = False


def _at_exit():
    # handles still alive at interpreter exit are left to the process
    # teardown: the HIP runtime may already be shutting down
    global _exiting
    _exiting = True


atexit.register(_at_exit)


def load(path: str | None = None):
    """Load liblf.so (no build, no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise LFError(6, f"{p} is missing: build it with python -m paper_1804_09152_amd.build")
    # torch ships its own HIP runtime; importing it first makes liblf.so bind
    # to that same runtime instead of loading a second one
    import torch  # noqa: F401
    lib = C.CDLL(p)
    V, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    PV = C.POINTER(C.c_void_p)
    sig = {
        "lf_last_error": (C.c_char_p, []),
        "lf_params_default": (None, [C.POINTER(lf_params)]),
        "lf_ctx_create": (C.c_int, [I32, V, PV]),
        "lf_ctx_destroy": (C.c_int, [V]),
        "lf_mesh_create": (C.c_int, [V, V, I32, V, I32, I32, PV]),
        "lf_mesh_destroy": (C.c_int, [V]),
        "lf_mesh_operator": (C.c_int, [V, V, V, V, V, I32]),
        "lf_fields_create": (C.c_int, [V, V, I32, C.POINTER(lf_params), PV]),
        "lf_fields_destroy": (C.c_int, [V]),
        "lf_fields_reset": (C.c_int, [V, V]),
        "lf_fields_create_rings": (C.c_int, [V, V, I32, I32, C.POINTER(lf_params), PV]),
        "lf_fields_create_regions": (C.c_int, [V, V, V, I32, C.POINTER(lf_params), PV]),
        "lf_fields_reset_regions": (C.c_int, [V, V, V]),
        "lf_fields_seeds": (C.c_int, [V, V]),
        "lf_fields_set_coefficients": (C.c_int, [V, I32, V, V]),
        "lf_step": (C.c_int, [V, I32]),
        "lf_step_until": (C.c_int, [V, I32, D, I32, V, V]),
        "lf_last_change": (C.c_int, [V, V, V]),
        "lf_sync": (C.c_int, [V]),
        "lf_fields_use_graphs": (C.c_int, [V, I32]),
        "lf_fields_set_reorder": (C.c_int, [V, I32, I32, I32]),
        "lf_fields_reorders": (C.c_int, [V, V]),
        "lf_fields_export": (C.c_int, [V, V, V, V, V, I32]),
        "lf_fields_import": (C.c_int, [V, I64, V, V, V, I32]),
        "lf_labels": (C.c_int, [V, V, I32]),
        "lf_lloyd_reseed": (C.c_int, [V, V, V]),
        "lf_lloyd": (C.c_int, [V, I32, I32, V]),
        "lf_dual_mesh": (C.c_int, [V, D, V, V, V, V, V]),
        "lf_dual_matrix": (C.c_int, [V, I32, V, V, V]),
        "lf_dual_candidates": (C.c_int, [V, V, V, V]),
        "lf_stats": (C.c_int, [V, V, V, V, V, V]),
        "lf_traffic": (C.c_int, [V, V, V]),
        "lf_step_timing": (C.c_int, [V, I32, V, V]),
        "lf_step_async": (C.c_int, [V, I32]),
        "lf_batch_create": (C.c_int, [V, I32, V, V, V, V, I32, V, V, C.POINTER(lf_params), PV]),
        "lf_batch_destroy": (C.c_int, [V]),
        "lf_batch_fields": (C.c_int, [V, PV]),
        "lf_batch_export": (C.c_int, [V, I32, V, V, V, V]),
        "lf_batch_labels": (C.c_int, [V, I32, V]),
        "lf_server_create": (C.c_int, [I32, I64, I32, I32, PV]),
        "lf_server_destroy": (C.c_int, [V]),
        "lf_server_submit": (C.c_int, [V, C.POINTER(lf_job), V]),
        "lf_server_poll": (C.c_int, [V, V, V, V]),
        "lf_server_cancel": (C.c_int, [V, I64]),
        "lf_server_result": (C.c_int, [V, I64, V, V, V, V, V, V, V]),
        "lf_server_release": (C.c_int, [V, I64]),
        "lf_server_memory": (C.c_int, [V, V, V]),
        "lf_server_times": (C.c_int, [V, I64, V, V, V]),
        "lf_server_stats": (C.c_int, [V, V, V]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise LFError(rc, load().lf_last_error().decode())


def _ptr(a):
    """numpy array or torch tensor -> (address, is_device)"""
    if a is None:
        return None, 0
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data, 0
    assert a.is_contiguous()
    return a.data_ptr(), int(a.is_cuda)


def _addr(x):
    return C.byref(x)


def default_params(**kw) -> lf_params:
    p = lf_params()
    load().lf_params_default(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# ---- C ABI, one wrapper per entry point ------------------------------------------

def lf_ctx_create(device: int = 0, stream=None):
    h = C.c_void_p()
    _check(load().lf_ctx_create(device, stream, C.byref(h)))
    return h


def lf_ctx_destroy(ctx):
    _check(load().lf_ctx_destroy(ctx))


def lf_mesh_create(ctx, V: np.ndarray, F: np.ndarray, op: int):
    V = np.ascontiguousarray(V, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    h = C.c_void_p()
    _check(load().lf_mesh_create(ctx, V.ctypes.data, V.shape[0], F.ctypes.data, F.shape[0], op,
                                 C.byref(h)))
    return h


def lf_mesh_destroy(mesh):
    _check(load().lf_mesh_destroy(mesh))


def lf_mesh_operator(mesh, rowptr=None, col=None, val=None):
    nnz = C.c_int64()
    pr, d = _ptr(rowptr)
    pc, _ = _ptr(col)
    pv, _ = _ptr(val)
    _check(load().lf_mesh_operator(mesh, C.byref(nnz), pr, pc, pv, d))
    return nnz.value


def lf_fields_create(mesh, seeds, params: lf_params | None = None):
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    h = C.c_void_p()
    _check(load().lf_fields_create(mesh, seeds.ctypes.data, seeds.size,
                                   C.byref(params) if params is not None else None, C.byref(h)))
    return h


def lf_fields_create_rings(mesh, seeds, rings: int, params: lf_params | None = None):
    s = np.ascontiguousarray(seeds, np.int32)
    out = C.c_void_p()
    _check(load().lf_fields_create_rings(mesh, s.ctypes.data, s.size, rings,
                                         C.byref(params) if params is not None else None,
                                         C.byref(out)))
    return out


def lf_fields_create_regions(mesh, region_ptr, region_vertices, params: lf_params | None = None):
    rp = np.ascontiguousarray(region_ptr, dtype=np.int32)
    rv = np.ascontiguousarray(region_vertices, dtype=np.int32)
    h = C.c_void_p()
    _check(load().lf_fields_create_regions(mesh, rp.ctypes.data, rv.ctypes.data, rp.size - 1,
                                           C.byref(params) if params is not None else None,
                                           C.byref(h)))
    return h


def lf_fields_reset_regions(f, region_ptr, region_vertices):
    rp = np.ascontiguousarray(region_ptr, dtype=np.int32)
    rv = np.ascontiguousarray(region_vertices, dtype=np.int32)
    _check(load().lf_fields_reset_regions(f, rp.ctypes.data, rv.ctypes.data))


def lf_fields_destroy(f):
    _check(load().lf_fields_destroy(f))


def lf_fields_reset(f, seeds):
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    _check(load().lf_fields_reset(f, seeds.ctypes.data))


def lf_fields_seeds(f, out: np.ndarray):
    _check(load().lf_fields_seeds(f, out.ctypes.data))


def lf_fields_set_coefficients(f, layer_types=None, table=None):
    """Per-pair coefficients: layer_types int32[n_s+1] (the base last),
    table float64[n_types, n_types, 3] (a, w, e); None clears them."""
    if layer_types is None:
        _check(load().lf_fields_set_coefficients(f, 0, None, None))
        return
    types = np.ascontiguousarray(layer_types, dtype=np.int32)
    tab = np.ascontiguousarray(table, dtype=np.float64)
    if tab.ndim != 3 or tab.shape[0] != tab.shape[1] or tab.shape[2] != 3:
        raise LFError(1, "table must have shape (n_types, n_types, 3)")
    _check(load().lf_fields_set_coefficients(f, tab.shape[0], types.ctypes.data, tab.ctypes.data))


def lf_step(f, n_steps: int):
    _check(load().lf_step(f, n_steps))


def lf_step_until(f, max_steps: int, eps: float, check_every: int):
    """Returns (steps_done, converged_at)."""
    a, b = C.c_int64(), C.c_int64()
    _check(load().lf_step_until(f, max_steps, eps, check_every, C.byref(a), C.byref(b)))
    return a.value, b.value


def lf_last_change(f):
    """Returns (changed_rows, max_delta) of the last completed step."""
    a, b = C.c_int64(), C.c_double()
    _check(load().lf_last_change(f, C.byref(a), C.byref(b)))
    return a.value, b.value


def lf_sync(f):
    _check(load().lf_sync(f))


def lf_fields_export(f, rowptr=None, col=None, val=None):
    nnz = C.c_int64()
    pr, d = _ptr(rowptr)
    pc, _ = _ptr(col)
    pv, _ = _ptr(val)
    _check(load().lf_fields_export(f, C.byref(nnz), pr, pc, pv, d))
    return nnz.value


def lf_fields_import(f, rowptr, col, val):
    pr, d = _ptr(rowptr)
    pc, _ = _ptr(col)
    pv, _ = _ptr(val)
    _check(load().lf_fields_import(f, int(col.shape[0]), pr, pc, pv, d))


def lf_labels(f, out):
    p, d = _ptr(out)
    _check(load().lf_labels(f, p, d))


def lf_lloyd_reseed(f, seeds_out: np.ndarray, status: np.ndarray | None = None):
    _check(load().lf_lloyd_reseed(f, seeds_out.ctypes.data,
                                  status.ctypes.data if status is not None else None))


def lf_dual_mesh(f, tau: float, tris=None, adj_rowptr=None, adj_col=None):
    n_tri = C.c_int64()
    nnz = C.c_int64()
    _check(load().lf_dual_mesh(f, tau, C.byref(n_tri), _ptr(tris)[0], C.byref(nnz),
                               _ptr(adj_rowptr)[0], _ptr(adj_col)[0]))
    return n_tri.value, nnz.value


def lf_dual_matrix(f, which: int, rowptr=None, col=None):
    nnz = C.c_int64()
    _check(load().lf_dual_matrix(f, which, C.byref(nnz), _ptr(rowptr)[0], _ptr(col)[0]))
    return nnz.value


def lf_dual_candidates(f, pairs=None, state=None):
    n = C.c_int64()
    _check(load().lf_dual_candidates(f, C.byref(n), _ptr(pairs)[0], _ptr(state)[0]))
    return n.value


def lf_stats(f):
    v = [C.c_int64() for _ in range(5)]
    _check(load().lf_stats(f, *[C.byref(x) for x in v]))
    return dict(zip(["nnz", "skeleton_total", "steps", "empty_columns", "grow_events"],
                    [x.value for x in v]))


def lf_traffic(f):
    a, b = C.c_int64(), C.c_int64()
    _check(load().lf_traffic(f, C.byref(a), C.byref(b)))
    return a.value, b.value


def lf_step_timing(f, enable: int):
    ms = C.c_double()
    n = C.c_int64()
    _check(load().lf_step_timing(f, enable, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def lf_batch_create(ctx, meshes, op: int, seeds, params: lf_params | None = None):
    """meshes: list of (V float64 (n,3), F int32 (m,3)); seeds: list of int32."""
    n = len(meshes)
    Vs = [np.ascontiguousarray(V, np.float64) for V, _ in meshes]
    Fs = [np.ascontiguousarray(F, np.int32) for _, F in meshes]
    Ss = [np.ascontiguousarray(s, np.int32) for s in seeds]
    Vp = (C.c_void_p * n)(*[v.ctypes.data for v in Vs])
    Fp = (C.c_void_p * n)(*[f.ctypes.data for f in Fs])
    Sp = (C.c_void_p * n)(*[s.ctypes.data for s in Ss])
    nv = np.array([v.shape[0] for v in Vs], np.int32)
    nf = np.array([f.shape[0] for f in Fs], np.int32)
    ns = np.array([s.size for s in Ss], np.int32)
    h = C.c_void_p()
    _check(load().lf_batch_create(ctx, n, Vp, nv.ctypes.data, Fp, nf.ctypes.data, op, Sp,
                                  ns.ctypes.data,
                                  C.byref(params) if params is not None else None, C.byref(h)))
    return h


def lf_batch_destroy(b):
    _check(load().lf_batch_destroy(b))


def lf_batch_fields(b):
    h = C.c_void_p()
    _check(load().lf_batch_fields(b, C.byref(h)))
    return h


def lf_batch_export(b, mesh: int, rowptr=None, col=None, val=None):
    nnz = C.c_int64()
    _check(load().lf_batch_export(b, mesh, C.byref(nnz), _ptr(rowptr)[0], _ptr(col)[0],
                                  _ptr(val)[0]))
    return nnz.value


def lf_batch_labels(b, mesh: int, out: np.ndarray):
    _check(load().lf_batch_labels(b, mesh, out.ctypes.data))


def lf_server_create(device: int, hbm_budget: int, max_active: int, chunk: int):
    h = C.c_void_p()
    _check(load().lf_server_create(device, hbm_budget, max_active, chunk, C.byref(h)))
    return h


def lf_server_destroy(s):
    _check(load().lf_server_destroy(s))


def lf_server_submit(s, job: lf_job):
    i = C.c_int64()
    _check(load().lf_server_submit(s, C.byref(job), C.byref(i)))
    return i.value


def lf_server_poll(s):
    q, a, d = C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().lf_server_poll(s, C.byref(q), C.byref(a), C.byref(d)))
    return q.value, a.value, d.value


def lf_server_result(s, job_id: int, seeds=None, labels=None, tris=None):
    """Returns (n_tri, latency_ms, queue_ms, steps)."""
    nt, lat, qu, st = C.c_int64(), C.c_double(), C.c_double(), C.c_int64()
    _check(load().lf_server_result(s, job_id, _ptr(seeds)[0], _ptr(labels)[0], C.byref(nt),
                                   _ptr(tris)[0], C.byref(lat), C.byref(qu), C.byref(st)))
    return nt.value, lat.value, qu.value, st.value


def lf_server_release(s, job_id: int):
    _check(load().lf_server_release(s, job_id))


def lf_server_memory(s):
    a, b = C.c_int64(), C.c_int64()
    _check(load().lf_server_memory(s, C.byref(a), C.byref(b)))
    return a.value, b.value


# ---- owners ----------------------------------------------------------------------

class Context:
    """A library context on one GPU, running on a torch stream (default: the
    current stream of `device`)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.torch_stream = stream
        self.device = device
        self.h = lf_ctx_create(device, C.c_void_p(stream.cuda_stream))

    def close(self):
        if self.h:
            lf_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    def __init__(self, ctx: Context, V, F, op: int):
        self.ctx = ctx
        self.n_v = int(V.shape[0])
        self.n_f = int(F.shape[0])
        self.h = lf_mesh_create(ctx.h, V, F, op)

    def operator(self):
        """Operator with diagonal as host CSR (rowptr, col, val float32)."""
        nnz = lf_mesh_operator(self.h)
        rp = np.zeros(self.n_v + 1, np.int32)
        col = np.zeros(nnz, np.int32)
        val = np.zeros(nnz, np.float32)
        lf_mesh_operator(self.h, rp, col, val)
        return rp, col, val

    def close(self):
        if self.h:
            lf_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent meshes stepped together; results per mesh in its own
    numbering."""

    def __init__(self, ctx: Context, meshes, op: int, seeds, params: lf_params | None = None):
        self.ctx = ctx
        self.n_v = [int(V.shape[0]) for V, _ in meshes]
        self.n_s = [int(np.asarray(s).size) for s in seeds]
        self.h = lf_batch_create(ctx.h, meshes, op, seeds, params)
        self.fh = lf_batch_fields(self.h)

    def step(self, n: int = 1):
        lf_step(self.fh, n)

    def reset(self):
        """Back to the initial fields of every mesh (seeds kept)."""
        s = np.zeros(sum(self.n_s), np.int32)
        lf_fields_seeds(self.fh, s)
        lf_fields_reset(self.fh, s)

    def export(self, m: int):
        nnz = lf_batch_export(self.h, m)
        rp = np.zeros(self.n_v[m] + 1, np.int32)
        col = np.zeros(nnz, np.int32)
        val = np.zeros(nnz, np.float32)
        lf_batch_export(self.h, m, rp, col, val)
        return rp, col, val

    def set_coefficients(self, layer_types=None, table=None):
        """Per-pair coefficients over the batch's layers (cells of mesh 0,
        mesh 1, ..., then the shared base)."""
        lf_fields_set_coefficients(self.fh, layer_types, table)

    def labels(self, m: int):
        out = np.zeros(self.n_v[m], np.int32)
        lf_batch_labels(self.h, m, out)
        return out

    def stats(self):
        return lf_stats(self.fh)

    def timing(self, enable: int = -1):
        return lf_step_timing(self.fh, enable)

    def use_graphs(self, on: bool = True):
        _check(load().lf_fields_use_graphs(self.fh, int(bool(on))))

    def set_reorder(self, every: int, tile_rows: int = 4096, classes: int = 4):
        _check(load().lf_fields_set_reorder(self.fh, int(every), int(tile_rows), int(classes)))

    def close(self):
        if self.h:
            lf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching job loop on one GPU (see lf_server_* in lf.h)."""

    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, max_active: int = 8,
                 chunk: int = 64):
        self.h = lf_server_create(device, hbm_budget, max_active, chunk)
        self.shape = {}

    def submit(self, V, F, seeds, steps: int, lloyd_rounds: int = 0, dual_mesh: bool = False,
               op: int = LF_OP_GRAPH, params: lf_params | None = None, conv_eps: float = 0.0,
               conv_every: int = 16, layer_types=None, table=None) -> int:
        V = np.ascontiguousarray(V, np.float64)
        F = np.ascontiguousarray(F, np.int32)
        S = np.ascontiguousarray(seeds, np.int32)
        j = lf_job()
        j.V, j.F, j.seeds = V.ctypes.data, F.ctypes.data, S.ctypes.data
        j.n_v, j.n_f, j.n_s, j.op = V.shape[0], F.shape[0], S.size, op
        j.steps, j.lloyd_rounds, j.dual_mesh = steps, lloyd_rounds, int(bool(dual_mesh))
        j.params = params if params is not None else default_params()
        j.conv_eps, j.conv_every = conv_eps, conv_every
        if layer_types is not None:  # copied by the server during submit
            T = np.ascontiguousarray(layer_types, np.int32)
            tab = np.ascontiguousarray(table, np.float64)
            if tab.ndim != 3 or tab.shape[0] != tab.shape[1] or tab.shape[2] != 3 or T.size != S.size + 1:
                raise LFError(1, "layer_types must hold n_s + 1 types, table (n_types, n_types, 3)")
            j.n_types, j.layer_types, j.table = tab.shape[0], T.ctypes.data, tab.ctypes.data
        i = lf_server_submit(self.h, j)
        self.shape[i] = (V.shape[0], S.size)
        return i

    def poll(self):
        return lf_server_poll(self.h)

    def run(self, sleep_s: float = 0.0):
        """Polls until every submitted job has finished."""
        import time
        while True:
            q, a, _ = self.poll()
            if q == 0 and a == 0:
                return
            if sleep_s:
                time.sleep(sleep_s)

    def result(self, job_id: int):
        """dict(seeds, labels, tris, latency_ms, queue_ms, steps)."""
        n_v, n_s = self.shape[job_id]
        nt, _, _, _ = lf_server_result(self.h, job_id)
        seeds = np.zeros(n_s, np.int32)
        labels = np.zeros(n_v, np.int32)
        tris = np.zeros((nt, 3), np.int32)
        nt, lat, qu, st = lf_server_result(self.h, job_id, seeds, labels, tris)
        return dict(seeds=seeds, labels=labels, tris=tris, latency_ms=lat, queue_ms=qu, steps=st)

    def cancel(self, job_id: int):
        _check(load().lf_server_cancel(self.h, job_id))

    def release(self, job_id: int):
        lf_server_release(self.h, job_id)
        self.shape.pop(job_id, None)

    def memory(self):
        return lf_server_memory(self.h)

    def times(self, job_id: int):
        """(submit, admit, done) on the monotonic clock, ms."""
        v = [C.c_double() for _ in range(3)]
        _check(load().lf_server_times(self.h, job_id, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def stats(self):
        """(ticks, grouped step launches)."""
        v = [C.c_int64() for _ in range(2)]
        _check(load().lf_server_stats(self.h, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def close(self):
        if self.h:
            lf_server_destroy(self.h)
            self.h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


class Fields:
    def __init__(self, mesh: Mesh, seeds=None, params: lf_params | None = None, regions=None,
                 rings: int = 0):
        """From seeds (int32 vertex ids; grown by `rings` rings), or from
        initial regions given as (region_ptr, region_vertices)."""
        self.mesh = mesh
        if rings:
            self.n_s = int(np.asarray(seeds).size)
            self.h = lf_fields_create_rings(mesh.h, seeds, rings, params)
        elif regions is not None:
            rp, rv = regions
            self.n_s = int(np.asarray(rp).size) - 1
            self.h = lf_fields_create_regions(mesh.h, rp, rv, params)
        else:
            self.n_s = int(np.asarray(seeds).size)
            self.h = lf_fields_create(mesh.h, seeds, params)

    def reset_regions(self, region_ptr, region_vertices):
        lf_fields_reset_regions(self.h, region_ptr, region_vertices)

    def set_coefficients(self, layer_types=None, table=None):
        """Per-pair a, w, e from layer types and a type-pair table; None
        returns to the scalar constants."""
        lf_fields_set_coefficients(self.h, layer_types, table)

    def step(self, n: int = 1):
        lf_step(self.h, n)

    def step_async(self, n: int = 1):
        """Enqueue the first min(n, 256) steps and return; the next call on
        these fields (sync, export, ...) completes all n."""
        _check(load().lf_step_async(self.h, int(n)))

    def sync(self):
        _check(load().lf_sync(self.h))

    def use_graphs(self, on: bool = True):
        _check(load().lf_fields_use_graphs(self.h, int(bool(on))))

    def set_reorder(self, every: int, tile_rows: int = 4096, classes: int = 4):
        _check(load().lf_fields_set_reorder(self.h, int(every), int(tile_rows), int(classes)))

    def reorders(self) -> int:
        n = C.c_int64()
        _check(load().lf_fields_reorders(self.h, C.byref(n)))
        return n.value

    def step_until(self, max_steps: int, eps: float = 1e-2, check_every: int = 32):
        return lf_step_until(self.h, max_steps, eps, check_every)

    def last_change(self):
        return lf_last_change(self.h)

    def reset(self, seeds):
        lf_fields_reset(self.h, seeds)

    def seeds(self):
        out = np.zeros(self.n_s, np.int32)
        lf_fields_seeds(self.h, out)
        return out

    def export(self):
        """Host CSR (rowptr int32, col int32, val float32)."""
        nnz = lf_fields_export(self.h)
        rp = np.zeros(self.mesh.n_v + 1, np.int32)
        col = np.zeros(nnz, np.int32)
        val = np.zeros(nnz, np.float32)
        lf_fields_export(self.h, rp, col, val)
        return rp, col, val

    def export_device(self):
        import torch
        nnz = lf_fields_export(self.h)
        dev = torch.device("cuda", self.mesh.ctx.device)
        rp = torch.empty(self.mesh.n_v + 1, dtype=torch.int32, device=dev)
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)[:nnz]
        val = torch.empty(max(nnz, 1), dtype=torch.float32, device=dev)[:nnz]
        lf_fields_export(self.h, rp, col, val)
        return rp, col, val

    def load(self, rowptr, col, val):
        lf_fields_import(self.h, np.ascontiguousarray(rowptr, np.int32) if isinstance(rowptr, np.ndarray) else rowptr,
                         np.ascontiguousarray(col, np.int32) if isinstance(col, np.ndarray) else col,
                         np.ascontiguousarray(val, np.float32) if isinstance(val, np.ndarray) else val)

    def labels(self):
        out = np.zeros(self.mesh.n_v, np.int32)
        lf_labels(self.h, out)
        return out

    def lloyd(self, rounds: int, steps_per_round: int):
        """rounds x (re-seed, re-initialise, steps_per_round steps); the
        final seeds."""
        seeds = np.zeros(self.n_s, np.int32)
        _check(load().lf_lloyd(self.h, rounds, steps_per_round, seeds.ctypes.data))
        return seeds

    def lloyd_reseed(self):
        seeds = np.zeros(self.n_s, np.int32)
        status = np.zeros(self.n_s, np.int32)
        lf_lloyd_reseed(self.h, seeds, status)
        return seeds, status

    def dual_mesh(self, tau: float = 0.25):
        n_tri, nnz = lf_dual_mesh(self.h, tau)
        tris = np.zeros((n_tri, 3), np.int32)
        rp = np.zeros(self.n_s + 1, np.int32)
        col = np.zeros(nnz, np.int32)
        lf_dual_mesh(self.h, tau, tris, rp, col)
        return tris, (rp, col)

    def dual_matrix(self, which: int):
        nnz = lf_dual_matrix(self.h, which)
        rp = np.zeros(self.n_s + 1, np.int32)
        col = np.zeros(nnz, np.int32)
        lf_dual_matrix(self.h, which, rp, col)
        return rp, col

    def dual_candidates(self):
        n = lf_dual_candidates(self.h)
        pairs = np.zeros((n, 2), np.int32)
        state = np.zeros(n, np.int32)
        lf_dual_candidates(self.h, pairs, state)
        return pairs, state

    def stats(self):
        return lf_stats(self.h)

    def timing(self, enable: int = -1):
        return lf_step_timing(self.h, enable)

    def traffic(self):
        return lf_traffic(self.h)

    def close(self):
        if self.h:
            lf_fields_destroy(self.h)
            self.h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass
