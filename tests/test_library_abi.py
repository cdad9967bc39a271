"""The C-ABI library loads on the CPU and exports every function that
include/hsrq.h declares (no compute call: that needs a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2101_05063_amd", "libhsrq.so")
HDR = os.path.join(ROOT, "include", "hsrq.h")


def declared():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"^int\s+(hsrq_\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for f in ["hsrq_create", "hsrq_destroy", "hsrq_set_stream", "hsrq_workspace_size", "hsrq_dhsrq3",
              "hsrq_workspace_size_batched", "hsrq_dhsrq3_batched"]:
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_all_declared_symbols():
    lib = ctypes.CDLL(LIB)
    for f in declared():
        assert hasattr(lib, f), f


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_names_match_header():
    import paper_2101_05063_amd as P
    assert sorted(P.EXPORTED) == sorted(n for n in declared() if n in P.EXPORTED)
    for f in declared():
        assert f in P.EXPORTED, f


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_argument_errors_without_gpu():
    """Argument checks happen before any HIP call (LAPACK-style -k codes)."""
    import paper_2101_05063_amd as P
    lib = P.load_library()
    # null handle -> -1
    assert lib.hsrq_dhsrq3(None, 4, None, 4, 1, None, None, None, 4, None, None, None, None, None, 0, None) == -1
    sz = ctypes.c_size_t()
    assert lib.hsrq_workspace_size(None, 4, 1, None, None, ctypes.byref(sz)) == -1
