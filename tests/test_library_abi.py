"""The C-ABI library loads on the CPU and exports every symbol declared in
include/rbffd.h; host-only logic (node generation, argument validation) is
checked without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import rbf_inputs as ri

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbffd.h")
LIB = os.path.join(ROOT, "paper_2206_06495_amd", "librbffd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbf_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librbffd.so is not built (run python paper_2206_06495_amd/build.py)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("rbf_build_nodes", "rbf_knn", "rbf_assemble_weights", "rbf_ell_apply",
              "rbf_ell_transpose", "rbf_ell_transpose_weights", "rbf_ell_apply_transpose",
              "rbf_solver_create", "rbf_step", "rbf_solve_pressure", "rbf_solver_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_abi_version(lib):
    lib.rbf_abi_version.restype = ctypes.c_int32
    assert lib.rbf_abi_version() == 5


@pytest.mark.parametrize("kind,K,seed", [(0, 7, 0), (0, 40, 3), (1, 50, 1), (2, 2, 0), (2, 9, 4),
                                         (2, 101, 2)])
def test_host_node_builder_matches_input_generator(lib, kind, K, seed):
    """rbf_build_nodes (C, host) and rbf_inputs (NumPy) implement the same
    SplitMix64 recipe independently; coordinates must be bit-identical."""
    f = lib.rbf_build_nodes
    f.restype = ctypes.c_int32
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                  ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    nv, npn = ctypes.c_int64(), ctypes.c_int64()
    assert f(kind, K, 0.3, seed, nv, None, None, npn, None, None, None) == 0
    xv = np.empty((2, nv.value))
    vt = np.empty(nv.value, np.int8)
    xp = np.empty((2, npn.value))
    pt = np.empty(npn.value, np.int8)
    pn = np.empty((2, npn.value))
    c = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    assert f(kind, K, 0.3, seed, nv, c(xv), c(vt), npn, c(xp), c(pt), c(pn)) == 0
    ref = ri.build_nodes(kind, K, 0.3, seed)
    for a, b in ((xv, ref.xv), (vt, ref.v_tag), (xp, ref.xp), (pt, ref.p_tag), (pn, ref.p_normal)):
        assert np.array_equal(a, b)
    # Invalid arguments are rejected on the host.
    assert f(0, 1, 0.3, 0, nv, None, None, npn, None, None, None) == -1
    assert f(7, 10, 0.3, 0, nv, None, None, npn, None, None, None) == -1
    assert f(0, 10, 0.9, 0, nv, None, None, npn, None, None, None) == -1
    assert f(0, 10, 0.3, 0, nv, c(xv), None, npn, None, None, None) == -1


def test_argument_validation_before_any_device_work(lib):
    """Calls with invalid sizes return RBF_E_ARG without touching the device."""
    lib.rbf_knn.restype = ctypes.c_int32
    lib.rbf_knn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.rbf_knn(None, 10, None, 5, 0, None, None) == -1
    assert lib.rbf_knn(None, 10, None, 5, 6, None, None) == -1
    assert lib.rbf_knn(None, 10, None, 100, 65, None, None) == -1
    lib.rbf_ell_apply.restype = ctypes.c_int32
    lib.rbf_ell_apply.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
    assert lib.rbf_ell_apply(10, 28, None, None, None, None, 2, None) == -1
    assert lib.rbf_ell_apply(0, 28, None, None, None, None, 0, None) == 0
    lib.rbf_last_error.restype = ctypes.c_char_p
    lib.rbf_ell_apply(10, 0, None, None, None, None, 0, None)
    assert b"k must be" in lib.rbf_last_error()
    # Transposed products: size, dtype and pointer checks; no columns is a no-op.
    lib.rbf_ell_transpose.restype = ctypes.c_int32
    lib.rbf_ell_transpose.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    bad = ctypes.c_int64(7)
    assert lib.rbf_ell_transpose(10, 0, None, 5, None, None, None, ctypes.byref(bad), None) == -1
    assert lib.rbf_ell_transpose(1 << 27, 28, None, 5, None, None, None, ctypes.byref(bad), None) == -1
    assert lib.rbf_ell_transpose(10, 28, None, -1, None, None, None, ctypes.byref(bad), None) == -1
    assert lib.rbf_ell_transpose(10, 28, None, 5, None, None, None, None, None) == -1
    assert lib.rbf_ell_transpose(10, 28, None, 5, None, None, None, ctypes.byref(bad), None) == -1
    assert bad.value == -1 and b"colptr" in lib.rbf_last_error()
    lib.rbf_ell_transpose_weights.restype = ctypes.c_int32
    lib.rbf_ell_transpose_weights.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_int32, ctypes.c_void_p]
    assert lib.rbf_ell_transpose_weights(10, 0, None, None, None, None, 0, None) == -1
    assert lib.rbf_ell_transpose_weights(10, 28, None, None, None, None, 2, None) == -1
    assert lib.rbf_ell_transpose_weights(10, 28, None, None, None, None, 0, None) == -1
    assert lib.rbf_ell_transpose_weights(0, 28, None, None, None, None, 0, None) == 0
    lib.rbf_ell_apply_transpose.restype = ctypes.c_int32
    lib.rbf_ell_apply_transpose.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int32, ctypes.c_void_p]
    assert lib.rbf_ell_apply_transpose(5, None, None, None, None, None, 2, None) == -1
    assert lib.rbf_ell_apply_transpose(5, None, None, None, None, None, 0, None) == -1
    assert lib.rbf_ell_apply_transpose(-1, None, None, None, None, None, 0, None) == -1
    assert lib.rbf_ell_apply_transpose(0, None, None, None, None, None, 0, None) == 0
    lib.rbf_solver_diagnostics.restype = ctypes.c_int32
    lib.rbf_solver_diagnostics.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.rbf_solver_diagnostics(None, None, None) == -1
    # Batch stepping: argument checks, and an empty batch is a no-op.
    lib.rbf_step_batch.restype = ctypes.c_int32
    lib.rbf_step_batch.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    assert lib.rbf_step_batch(None, -1, 1, None, None, None, 0) == -1
    assert lib.rbf_step_batch(None, 2, 1, None, None, None, 0) == -1
    assert lib.rbf_step_batch(None, 0, 1, None, None, None, 4) == 0
    nulls = (ctypes.c_void_p * 2)(None, None)
    assert lib.rbf_step_batch(nulls, 2, 1, ctypes.c_void_p(1), None, None, 0) == -1
    assert b"solver 0 is NULL" in lib.rbf_last_error()
    lib.rbf_solver_query.restype = ctypes.c_int32
    lib.rbf_solver_query.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.rbf_solver_query(None, None) == -1
