"""The C-ABI library loads and exports every entry point include/esrk.h
declares; argument validation needs no GPU (CPU only, no compute calls)."""
import ctypes as C
import os
import subprocess

import pytest

from paper_2003_08831_amd import esrk


def test_library_exports_declared_symbols():
    L = esrk.load()
    names = esrk.declared_symbols()
    assert "esrk_step" in names and "esrk_local_relaxation_solve" in names
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", esrk.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_status_strings():
    L = esrk.load()
    for code in range(8):
        assert L.esrk_status_str(code)


@pytest.mark.parametrize("field,value,expect", [
    ("dim", 4, 1), ("dim", 0, 1), ("deg", 0, 1), ("deg", 9, 1), ("gas_gamma", 1.0, 1),
    ("precision", 3, 1), ("tableau", 5, 7),
])
def test_create_rejects_bad_config(field, value, expect):
    cfg = esrk.make_config(2, 3, (4, 4), (0, 0), (1, 1))
    setattr(cfg, field, value)
    h = C.c_void_p()
    assert esrk.load().esrk_create(C.byref(cfg), C.byref(h)) == expect
    assert not h.value


def test_create_rejects_empty_mesh_and_null():
    cfg = esrk.make_config(2, 3, (0, 4), (0, 0), (1, 1))
    h = C.c_void_p()
    assert esrk.load().esrk_create(C.byref(cfg), C.byref(h)) == 1
    assert esrk.load().esrk_create(None, C.byref(h)) == 1
    assert esrk.load().esrk_rhs_euler(None, None, None, None, None) == 1
    assert esrk.load().esrk_step(None, None, None, 0.0, None, None, None) == 1
    assert esrk.load().esrk_run_graph(None, None, None, 1, None, None) == 1
    assert esrk.load().esrk_set_boundaries(None, 1, None, 1, None) == 1


def test_create_rejects_meshes_beyond_32_bit_indexing():
    # (dim+2) * ne * (deg+1)^dim = 5 * 700^3 * 8 > 2^31 - 1
    cfg = esrk.make_config(3, 1, (700, 700, 700), (0, 0, 0), (1, 1, 1))
    h = C.c_void_p()
    assert esrk.load().esrk_create(C.byref(cfg), C.byref(h)) == 1
    assert not h.value


def test_batch_create_validation():
    L = esrk.load()
    h = C.c_void_p()
    c2 = esrk.make_config(2, 3, (4, 4), (0, 0), (1, 1))
    c3 = esrk.make_config(3, 3, (4, 4, 4), (0, 0, 0), (1, 1, 1))
    arr = (esrk.Config * 1)(c3)
    assert L.esrk_batch_create(arr, 1, C.byref(h)) == 7  # 3-D: not compiled
    other = esrk.make_config(2, 4, (4, 4), (0, 0), (1, 1))
    arr = (esrk.Config * 2)(c2, other)
    assert L.esrk_batch_create(arr, 2, C.byref(h)) == 1  # mixed degree
    big = esrk.make_config(2, 3, (20000, 20000), (0, 0), (1, 1))
    arr = (esrk.Config * 2)(c2, big)
    assert L.esrk_batch_create(arr, 2, C.byref(h)) == 1  # beyond 32-bit indexing
    assert L.esrk_batch_create(arr, 0, C.byref(h)) == 1
    emb = esrk.make_config(2, 3, (4, 4), (0, 0), (1, 1), tableau=esrk.BSRK43)
    arr = (esrk.Config * 1)(emb)
    assert L.esrk_batch_create(arr, 1, C.byref(h)) == 7  # embedded pairs: single meshes only
    assert not h.value


def test_network_entry_point_validation():
    L = esrk.load()
    assert L.esrk_mlp_grad_work_size(0) == 0
    assert L.esrk_mlp_grad_work_size(1) == esrk.MLP_TRAINED + 1
    assert L.esrk_mlp_grad_work_size(65) == 2 * (esrk.MLP_TRAINED + 1)
    assert L.esrk_mlp_forward(None, None, 4, None, None) == 1
    assert L.esrk_mlp_grad(None, None, None, 4, None, None, None, None) == 1
    assert L.esrk_mlp_adam(None, None, None, None, 1, 1e-3, None) == 1
    assert L.esrk_mlp_prepare(None, None, None, 4, 1, None, None, None) == 1
    assert L.esrk_set_step_model(None, None, None) == 1
    assert L.esrk_local_relaxation_solve_ml(None, None, None, None, 1.0, None, None, None,
                                            None, None, None, None) == 1


def test_global_relaxation_entry_point_validation():
    L = esrk.load()
    assert L.esrk_set_relaxation_mode(None, esrk.RELAX_GLOBAL) == 1
    assert L.esrk_global_relaxation_solve(None, None, None, None, None, None, None) == 1


def test_error_control_entry_point_validation():
    L = esrk.load()
    assert L.esrk_set_adaptive(None, 1e-4, 1e-4) == 1
    assert L.esrk_error_estimate(None, None, None, None) == 1
    assert L.esrk_stage_phi0(None, None, None) == 1
    assert L.esrk_set_root_method(None, esrk.ROOT_BRENT) == 1
    assert L.esrk_set_dirichlet(None, None, None) == 1
    assert L.esrk_local_relaxation_solve_phi0(None, None, None, None, None, None, None, None,
                                              None) == 1


def test_missing_library_fails_loudly():
    """Without the built HIP library every entry point raises (no CPU path)."""
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2003_08831_amd import esrk\n"
        "esrk.LIB_PATH = '/nonexistent/libesrk.so'\n"
        "try:\n"
        "    esrk.Context(esrk.make_config(2, 3, (4, 4), (0, 0), (1, 1)))\n"
        "except RuntimeError as e:\n"
        "    print('raised:', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(3)\n" % os.path.dirname(esrk.HERE)
    )
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "HIP library missing" in r.stdout
