"""The C-ABI library loads and exports every function include/dmrg.h declares
(no compute calls: these run without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmrg.h")
LIB = os.path.join(ROOT, "paper_2311_02854_amd", "lib", "libdmrg.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(dmrg_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["dmrg_build_ops", "dmrg_sigma", "dmrg_davidson", "dmrg_create", "dmrg_destroy",
              "dmrg_last_error", "dmrg_ops_layout", "dmrg_ops_destroy", "dmrg_sigma_batched", "dmrg_diag"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_loads_and_rejects_bad_arguments():
    from paper_2311_02854_amd import binding
    lib = binding.load()
    assert lib.dmrg_sigma(None, None, None, None, 0) == -1
    assert lib.dmrg_build_ops(None, None, None, None, None) == -1
    assert lib.dmrg_sigma_batched(None, 0, None, None, None, 0, 0) == -1
    assert lib.dmrg_last_error(None) == b"null context"
