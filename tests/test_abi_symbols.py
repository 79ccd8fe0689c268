"""The C-ABI library loads on a host without a GPU and exports every function
that include/mrpt.h declares (no compute call is made)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrpt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mrpt_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("mrpt_build", "mrpt_query", "mrpt_query_ex", "mrpt_free", "mrpt_last_error",
              "mrpt_debug_leaves", "mrpt_debug_votes", "mrpt_export_tree", "mrpt_export_projection"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1509_06957_amd import mrpt
    lib = mrpt.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(mrpt.EXPORTED) == set(declared_functions())


def test_binding_structs_match_header_layout():
    from paper_1509_06957_amd import mrpt
    # int32 precision, int32 rerank_factor, float recheck_rel, int32 check_finite,
    # then two pointers (8-byte aligned)
    assert ctypes.sizeof(mrpt.mrpt_query_opts) == 16 + 8 + 8
    assert mrpt.mrpt_query_opts.s_count.offset == 16
    assert mrpt.mrpt_query_opts.stage_events.offset == 24


def test_error_path_without_gpu():
    from paper_1509_06957_amd import mrpt
    lib = mrpt.load()
    h = ctypes.c_void_p()
    st = lib.mrpt_build(None, 10, 4, 2, 1, ctypes.c_float(0.5), 1, ctypes.byref(h))
    assert st == mrpt.MRPT_EINVAL
    assert "data" in mrpt.mrpt_last_error()
    st = lib.mrpt_query(None, None, 1, 1, 1, None, None, None)
    assert st == mrpt.MRPT_EINVAL
