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
    # n; d, T, depth; a; seed; nnz; max_leaf, id_chunk; device_bytes;
    # built_on_device, max_row_nnz
    assert ctypes.sizeof(mrpt.mrpt_index_desc) == 8 + 12 + 4 + 8 + 8 + 8 + 8 + 8
    assert mrpt.mrpt_index_desc.built_on_device.offset == 56
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


def test_plan_structs_match_header_layout():
    from paper_1509_06957_amd import mrpt
    # mrpt_batch: index, Q pointers; int64 nq; int32 k, v; two pointers
    assert ctypes.sizeof(mrpt.mrpt_batch) == 8 + 8 + 8 + 4 + 4 + 8 + 8
    assert mrpt.mrpt_batch.k.offset == 24 and mrpt.mrpt_batch.out_idx.offset == 32
    assert ctypes.sizeof(mrpt.mrpt_plan_opts) == 32 and mrpt.mrpt_plan_opts.fused.offset == 24
    assert mrpt.mrpt_plan_opts.vote_waves.offset == 28


def test_plan_error_paths_without_gpu():
    from paper_1509_06957_amd import mrpt
    lib = mrpt.load()
    o = mrpt.mrpt_plan_opts()
    lib.mrpt_default_plan_opts(ctypes.byref(o))
    assert (o.precision, o.rerank_factor, o.branches, o.proj_rows, o.vote_kernel, o.fused, o.vote_waves) == \
        (mrpt.MRPT_FP32, 4, 4, 0, 0, 1, 0)
    h = ctypes.c_void_p()
    assert lib.mrpt_plan_create(None, 0, None, ctypes.byref(h)) == mrpt.MRPT_EINVAL
    assert "nbatch" in mrpt.mrpt_last_error()
    arr = (mrpt.mrpt_batch * 1)()
    assert lib.mrpt_plan_create(arr, 1, None, None) == mrpt.MRPT_EINVAL
    o.branches = 0
    assert lib.mrpt_plan_create(arr, 1, ctypes.byref(o), ctypes.byref(h)) == mrpt.MRPT_EINVAL
    assert "branches" in mrpt.mrpt_last_error()
    o.branches, o.proj_rows = 4, 8
    assert lib.mrpt_plan_create(arr, 1, ctypes.byref(o), ctypes.byref(h)) == mrpt.MRPT_EINVAL
    assert "proj_rows" in mrpt.mrpt_last_error()
    o.proj_rows, o.vote_kernel = 0, 3
    assert lib.mrpt_plan_create(arr, 1, ctypes.byref(o), ctypes.byref(h)) == mrpt.MRPT_EINVAL
    assert "vote_kernel" in mrpt.mrpt_last_error()
    o.vote_kernel, o.vote_waves = 0, 4
    assert lib.mrpt_plan_create(arr, 1, ctypes.byref(o), ctypes.byref(h)) == mrpt.MRPT_EINVAL
    assert "vote_waves" in mrpt.mrpt_last_error()
    assert lib.mrpt_plan_launch(None, None) == mrpt.MRPT_EINVAL
    assert lib.mrpt_plan_device_bytes(None) == 0
    lib.mrpt_plan_free(None)


def test_batched_workload_stream():
    """The batched workload's stream covers the stated number of queries in
    batches of 1..max_batch, with every index and k drawn from their sets."""
    from paper_1509_06957_amd import workloads as W
    bw = W.BATCHED
    specs = W.batched_indexes(bw)
    assert len(specs) == bw.n_indexes
    for sp in specs:
        assert bw.n_lo <= sp.n <= bw.n_hi and sp.d in bw.dims
        assert (1 << sp.depth) <= sp.n and 16 <= sp.n / (1 << sp.depth) <= 64
    st = W.batched_stream(bw)
    assert sum(m for _, _, m, _ in st) == bw.total_queries
    assert all(1 <= m <= bw.max_batch and 0 <= ix < bw.n_indexes and k in bw.ks for _, ix, m, k in st)
    assert [b for b, _, _, _ in st] == list(range(len(st)))
