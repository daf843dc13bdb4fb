"""CPU-side checks of the C ABI: the library loads, exports every entry point
declared in include/vrs.h, and rejects bad arguments on the host before any
device work (none of these calls touches a GPU)."""

import ctypes as C
import os
import re

import pytest

from paper_2403_15807_amd import vrs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vrs.h")).read()
    decl = r"^(?:vrs_status|int32_t|const char \*)\s*(vrs_[a-z_]+)\s*\("
    return sorted(set(re.findall(decl, src, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(vrs.LIB_PATH):
        from paper_2403_15807_amd import _build
        _build.build()
    return vrs.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(vrs.EXPORTS)


def test_header_struct_layout_matches_binding():
    assert C.sizeof(vrs.vrs_range) == 24
    assert C.sizeof(vrs.vrs_pred) == 8 + 24 * vrs.MAX_TERMS
    assert C.sizeof(vrs.vrs_opts) == 48  # 4 int32, 2 pointers, 2 int32, 1 pointer
    assert vrs.vrs_opts.passes.offset == 32
    assert vrs.vrs_opts.err_ratio.offset == 40


def test_host_side_argument_errors(L):
    h = C.c_void_p()
    assert L.vrs_build_table(None, 10, 4, None, 0, 0, 0, None, C.byref(h)) == vrs.VRS_E_ARG
    assert b"vec" in L.vrs_last_error()
    assert L.vrs_build_table(C.c_void_p(256), 10, 4, None, 0, 0, 0, None, None) == vrs.VRS_E_ARG
    assert L.vrs_build_table(C.c_void_p(256), 0, 4, None, 0, 0, 0, None, C.byref(h)) == vrs.VRS_E_ARG
    assert L.vrs_build_table(C.c_void_p(256), 10, 0, None, 0, 0, 0, None, C.byref(h)) == vrs.VRS_E_ARG
    assert L.vrs_build_table(C.c_void_p(256), 10, 4097, None, 0, 0, 0, None, C.byref(h)) == vrs.VRS_E_ARG
    assert L.vrs_build_table(C.c_void_p(256), 10, 4, None, 2, 0, 0, None, C.byref(h)) == vrs.VRS_E_ARG
    assert L.vrs_build_table(C.c_void_p(256), 10, 4, None, 0, 7, 0, None, C.byref(h)) == vrs.VRS_E_ARG
    assert L.vrs_destroy_table(None) == vrs.VRS_E_ARG
    assert L.vrs_scan_topk(None, None, 1, None, 1, 0, None, None, None, 0, None, None) == vrs.VRS_E_ARG
    nb = C.c_size_t()
    assert L.vrs_scan_workspace_bytes(None, 1, 1, None, C.byref(nb)) == vrs.VRS_E_ARG
    assert L.vrs_chooser_load(b"/nonexistent/chooser.bin") == vrs.VRS_E_ARG
    assert L.vrs_range_workspace_bytes(None, 1, 1, C.byref(nb)) == vrs.VRS_E_ARG
    assert L.vrs_scan_range(None, None, 1, None, 1, None, 1, None, None, None, None, 0, None,
                            None) == vrs.VRS_E_ARG
    assert L.vrs_num_tiles() >= 4
