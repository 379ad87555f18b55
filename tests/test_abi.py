"""The C-ABI library loads and exports every symbol include/ldsv.h declares
(CPU-only: no kernel is launched)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ldsv.h")
LIB = os.path.join(ROOT, "paper_2507_01975_amd", "lib", "libldsv.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"LDSV_API\s+(?:int|const char\*)\s+(ldsv_\w+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("ldsv_create", "ldsv_init_state", "ldsv_fv_step", "ldsv_learned_fv_step",
              "ldsv_project", "ldsv_rollout", "ldsv_fv_step_bwd", "ldsv_learned_fv_step_bwd",
              "ldsv_project_bwd", "ldsv_cnn_forward", "ldsv_cnn_backward"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build libldsv.so first (python -m paper_2507_01975_amd.build)"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (ldsv_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_binding_loads_and_covers_the_header():
    from paper_2507_01975_amd import ldsv
    assert ldsv._lib.ldsv_version() >= 100
    assert sorted(ldsv.exported_symbols()) == declared()


def test_create_rejects_bad_shapes_without_a_device():
    # argument validation happens before any HIP call
    import ctypes
    from paper_2507_01975_amd import ldsv
    h = ctypes.c_void_p()
    g = ldsv.Grid(12, 16, 1.0, 1.0, 1, ldsv.F32, ldsv.MAC)
    assert ldsv._lib.ldsv_create(ctypes.byref(h), ctypes.byref(g)) == ldsv.ESHAPE
    assert "powers of two" in ldsv.last_error()
    g = ldsv.Grid(16, 16, 1.0, 1.0, 0, ldsv.F32, ldsv.MAC)
    assert ldsv._lib.ldsv_create(ctypes.byref(h), ctypes.byref(g)) == ldsv.EINVAL
    g = ldsv.Grid(16, 16, 1.0, 1.0, 1, 7, ldsv.MAC)
    assert ldsv._lib.ldsv_create(ctypes.byref(h), ctypes.byref(g)) == ldsv.EDTYPE
    assert ldsv._lib.ldsv_create(None, ctypes.byref(g)) == ldsv.EINVAL
    assert ldsv._lib.ldsv_fv_step(None, None, None, None, None, None, None, 1, None) == ldsv.EINVAL
    assert ldsv._lib.ldsv_adam_step(None, None, None, None, 0, 1, 1e-4, 0.9, 0.999, 1e-8,
                                    None) == ldsv.EINVAL


def test_learned_derivative_entry_points_reject_bad_arguments_without_a_device():
    # every entry point validates its handle and pointers before any HIP call
    from paper_2507_01975_amd import ldsv
    L = ldsv._lib
    N = None
    assert L.ldsv_fv_step_d(N, N, N, N, N, N, N, N, 1, N) == ldsv.EINVAL
    assert L.ldsv_fv_step_d_bwd(*([N] * 13)) == ldsv.EINVAL
    assert L.ldsv_learned_d_fv_step(N, N, N, N, N, N, N, N, 1, N, N, N) == ldsv.EINVAL
    assert L.ldsv_learned_d_fv_step_bwd(N, N, N, N, N, N, 1, N, N, N, N, N, N, N) == ldsv.EINVAL
    assert "derivative network" in ldsv.last_error()
    assert L.ldsv_rollout_d(N, N, N, N, N, N, 1, 1, 1, N, N, N, N) == ldsv.EINVAL
    assert "null network" in ldsv.last_error()
    assert L.ldsv_rollout_d_bwd(N, N, N, N, N, N, 1, 1, 1, N, N, 1.0, N, N, N, N, N, N, N,
                                N) == ldsv.EINVAL
