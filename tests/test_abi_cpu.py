"""The C ABI library loads and exports every declared symbol; argument
validation that happens before any device call works without a GPU."""
import ctypes

import pytest

import paper_2606_07148_amd as pkg


@pytest.fixture(scope="module")
def lib():
    return pkg.load()


def test_exports_every_declared_symbol(lib):
    names = pkg.declared_symbols()
    assert "abcore_build_csr" in names and "abcore_compute" in names and "abcore_query" in names
    for name in names:
        assert hasattr(lib, name), name


def test_null_handle_and_bad_arguments_rejected(lib):
    EINVAL = 1
    assert lib.abcore_destroy(None) == 0
    assert lib.abcore_set_option(None, 1, 1) == EINVAL
    st = pkg.abcore_stats()
    assert lib.abcore_compute(None, 1, 1, 0, None, ctypes.byref(st), None) == EINVAL
    assert b"null" in lib.abcore_last_error()
    h = ctypes.c_void_p()
    md = ctypes.c_int64()
    # negative sizes, missing output pointer
    assert lib.abcore_build_csr(-1, 4, None, None, 0, None, ctypes.byref(h), ctypes.byref(md)) == EINVAL
    assert lib.abcore_build_csr(4, 4, None, None, 3, None, ctypes.byref(h), ctypes.byref(md)) == EINVAL
    assert lib.abcore_build_csr(4, 4, None, None, 0, None, None, None) == EINVAL
    ans = ctypes.c_int32()
    upd = pkg.abcore_edge_update(0, 0, 1)
    assert lib.abcore_query(None, upd, 1, 1, ctypes.byref(ans), None, None) == EINVAL
    assert lib.abcore_core_numbers(None, None, None, None) == EINVAL
    assert lib.abcore_components(None, None, None) == EINVAL
    assert lib.abcore_graph_info(None, None, None, None) == EINVAL
    t = ctypes.c_uint64()
    assert lib.abcore_serve_start(None, 0, 0, 0) == EINVAL
    assert lib.abcore_submit(None, upd, 1, 1, ctypes.byref(t)) == EINVAL
    assert lib.abcore_poll(None, 0, None, None, None) == EINVAL
    assert lib.abcore_serve_stop(None, None) == EINVAL


def test_budget_and_debug_entry_points_validate_arguments(lib):
    EINVAL = 1
    assert lib.abcore_set_memory_budget(-1) == EINVAL
    assert lib.abcore_set_memory_budget(1 << 30) == 0
    assert lib.abcore_set_memory_budget(0) == 0  # back to no budget
    assert lib.abcore_debug_enqueue_counts(None, None, 0, None) == EINVAL
    assert lib.abcore_set_option(None, pkg.ABCORE_OPT_SERVE_DEADLINE_US, 10) == EINVAL


def test_debug_library_exports_the_same_symbols():
    with pkg.debug_library() as dlib:
        for name in pkg.declared_symbols():
            assert hasattr(dlib, name), name
    assert pkg.load() is not dlib
