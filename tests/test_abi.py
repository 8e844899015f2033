"""The C-ABI library loads and exports every function include/dmwf.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmwf.h")
LIB = os.path.join(ROOT, "paper_1702_08852_amd", "libdmwf.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dmwf_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("dmwf_plan_create", "dmwf_plan_destroy", "dmwf_workspace_bytes", "dmwf_alm2map",
                 "dmwf_adjoint", "dmwf_dm_iterate", "dmwf_solve", "dmwf_wf_residual",
                 "dmwf_status_string", "dmwf_last_error"):
        assert need in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdmwf.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdmwf.so not built")
def test_host_side_validation_without_gpu():
    """Invalid plan descriptions are rejected before any device call."""
    from paper_1702_08852_amd import dmwf as b
    lib = b.load()
    lib.dmwf_status_string.restype = ctypes.c_char_p
    assert lib.dmwf_status_string(0) == b"ok"
    h = ctypes.c_void_p()
    for nside, lmax, nmaps, prec, want in [(3, 4, 1, 0, 1), (0, 0, 1, 0, 1), (16384, 4, 1, 0, 1),
                                           (4, 12, 1, 0, 1), (4, -1, 1, 0, 1), (4, 8, 0, 0, 1),
                                           (4, 8, 65536, 0, 1),
                                           (4, 8, 1, 3, 1)]:
        desc = b._PlanDesc(nside, lmax, nmaps, prec)
        assert lib.dmwf_plan_create(ctypes.byref(desc), ctypes.byref(h)) == want
        assert not h.value
    assert lib.dmwf_plan_create(None, ctypes.byref(h)) == 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdmwf.so not built")
def test_null_plans_are_argument_errors():
    """Every entry point taking a plan rejects NULL before touching a device."""
    from paper_1702_08852_amd import dmwf as b
    lib = b.load()
    assert lib.dmwf_set_tiles(None, 2, 1, 8, 1) == b.ERR_INVALID_ARG
    assert lib.dmwf_autotune(None, None, 0, None, None, None) == b.ERR_INVALID_ARG
    nb = ctypes.c_size_t()
    assert lib.dmwf_workspace_bytes(None, ctypes.byref(nb)) == b.ERR_INVALID_ARG
    assert lib.dmwf_alm2map(None, None, None, None, 0, None) == b.ERR_INVALID_ARG
    assert lib.dmwf_adjoint(None, None, None, 0, None, 0, None) == b.ERR_INVALID_ARG
    assert lib.dmwf_profile_enable(None, 1) == b.ERR_INVALID_ARG
    lib.dmwf_plan_destroy(None)  # accepted
