"""The C-ABI library loads and exports every entry point include/lf.h
declares (no GPU needed, no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lf_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ["lf_ctx_create", "lf_mesh_create", "lf_fields_create", "lf_step", "lf_labels",
              "lf_lloyd_reseed", "lf_dual_mesh", "lf_fields_export", "lf_fields_import"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1804_09152_amd as lfb
    if not os.path.exists(lfb.LIB_PATH):
        pytest.skip("liblf.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(lfb.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(lfb.EXPORTS) == _declared()


def test_params_default_without_gpu():
    import paper_1804_09152_amd as lfb
    if not os.path.exists(lfb.LIB_PATH):
        pytest.skip("liblf.so not built")
    p = lfb.default_params()
    assert (p.w, p.a, p.e, p.mu, p.dt, p.theta, p.tau) == (0.2, 0.04, 1.0, 0.1, 5.0, 1e-3, 0.25)


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_1804_09152_amd as lfb
    saved = lfb._lib
    lfb._lib = None
    try:
        with pytest.raises(lfb.LFError):
            lfb.load(str(tmp_path / "nope.so"))
    finally:
        lfb._lib = saved


def test_server_host_logic_without_gpu():
    """Queueing, budget check and result states touch no GPU until a poll."""
    import numpy as np
    import paper_1804_09152_amd as lfb
    from paper_1804_09152_amd import inputs as I
    if not os.path.exists(lfb.LIB_PATH):
        pytest.skip("liblf.so not built")
    mesh = I.torus_grid(16, 16)
    seeds = np.array([0, 40, 200], np.int32)
    with pytest.raises(lfb.LFError) as e:
        lfb.Server(0, 0, 1, 1)
    assert e.value.status == 1
    S = lfb.Server(0, 8 << 20, 2, 8)
    i = S.submit(mesh.V, mesh.F, seeds, steps=10)
    big = I.torus_grid(200, 200)
    with pytest.raises(lfb.LFError) as e:
        S.submit(big.V, big.F, seeds, steps=10)
    assert e.value.status == 2  # alone above the budget
    with pytest.raises(lfb.LFError) as e:
        lfb.lf_server_result(S.h, i)
    assert e.value.status == 5  # queued, not finished
    with pytest.raises(lfb.LFError) as e:
        lfb.lf_server_release(S.h, i)
    assert e.value.status == 5
    with pytest.raises(lfb.LFError) as e:
        lfb.lf_server_result(S.h, 12345)
    assert e.value.status == 1
    j = S.submit(mesh.V, mesh.F, seeds, steps=10)
    S.cancel(j)  # a queued job leaves the queue; no GPU needed
    with pytest.raises(lfb.LFError) as e:
        S.result(j)
    assert e.value.status == 1
    S.release(j)
    with pytest.raises(lfb.LFError):
        S.cancel(j)  # unknown now
    with pytest.raises(lfb.LFError):  # layer types for n_s + 1 layers, a square table
        S.submit(mesh.V, mesh.F, seeds, steps=10, layer_types=np.zeros(3, np.int32),
                 table=np.zeros((2, 2, 3)))
    assert S.memory() == (0, 0)
    S.close()  # queued jobs are dropped
