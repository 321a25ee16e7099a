"""The C-ABI library loads and exports every symbol include/mapmaker.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2501_16122_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mapmaker.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["mm_pointing_build", "mm_apply_P", "mm_apply_PT", "mm_apply_Ninv", "mm_apply_A",
                 "mm_apply_M", "mm_rhs", "mm_solve", "mm_noise_toeplitz", "mm_noise_white"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(binding.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    assert sorted(binding.SIGNATURES) == declared_functions()


@pytest.mark.skipif(not os.path.exists(binding.LIB_PATH), reason="library not built")
def test_host_only_calls():
    lib = binding.load()
    assert lib.mm_abi_version() == 5
    sz = ctypes.c_size_t()
    assert lib.mm_pointing_workspace_size(1 << 20, 4, 4096, binding.MM_F64, ctypes.byref(sz)) == 0
    assert sz.value > 4 * (1 << 20)
    assert lib.mm_pointing_workspace_size(10, 0, 4096, binding.MM_F64, ctypes.byref(sz)) == binding.MM_EINVAL
    assert b"bad" in lib.mm_last_error()
    assert lib.mm_pointing_workspace_size(10, 1, 4096, 7, ctypes.byref(sz)) == binding.MM_EINVAL
    assert b"dtype" in lib.mm_last_error()
    opts = binding.SolveOpts()
    assert lib.mm_solve_opts_default(ctypes.byref(opts)) == 0
    assert opts.tol == 1e-10 and opts.max_iter == 2000
    import numpy as np
    offs = np.array([0, 100, 250], dtype=np.int64)
    assert lib.mm_noise_toeplitz_workspace_size(64, 1, offs.ctypes.data_as(binding._pi64), 2,
                                                ctypes.byref(sz)) == 0
    assert sz.value > 0
    assert lib.mm_noise_toeplitz_workspace_size(5000, 1, offs.ctypes.data_as(binding._pi64), 2,
                                                ctypes.byref(sz)) == binding.MM_EINVAL
    # batched steps validate their arguments before touching a device
    assert lib.mm_batch_step(None, 0, 8) == binding.MM_EINVAL
    arr = (ctypes.c_void_p * 2)(None, None)
    assert lib.mm_batch_step(arr, 2, 8) == binding.MM_EINVAL
    assert b"null solver" in lib.mm_last_error()
