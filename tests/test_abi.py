"""The C-ABI library loads and exports every entry point declared in include/tc_lcc.h (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2202_13976_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    with open(os.path.join(ROOT, "include", "tc_lcc.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:tc_lcc_status|const char\*)\s+(tc_lcc_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported():
    names = declared()
    assert len(names) >= 15
    L = pkg.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) <= set(pkg.EXPORTS)


def test_status_strings_and_null_arguments():
    L = pkg.lib()
    assert L.tc_lcc_status_string(0) == b"ok"
    assert L.tc_lcc_status_string(3) == b"over budget"
    # null handles are rejected before any device work
    assert L.tc_lcc_run(None, None, None, None) == pkg.INVALID_ARGUMENT
    assert b"null" in L.tc_lcc_last_error()
    assert L.tc_lcc_graph_free(None) == pkg.INVALID_ARGUMENT
    assert L.tc_lcc_ctx_destroy(None) == pkg.INVALID_ARGUMENT
    assert L.tc_lcc_batch_poll(None, 0, 0, None) == pkg.INVALID_ARGUMENT


def test_no_cpu_fallback_without_gpu():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(pkg.TcLccError) as e:
        pkg.Context(0)
    assert e.value.status == pkg.INVALID_ARGUMENT


def test_every_entry_point_rejects_null_handles():
    """Each handle-taking entry point checks its handle before any device work, so these calls
    need no GPU; each leaves a message for the calling thread."""
    L = pkg.lib()
    u64 = ctypes.c_uint64()
    calls = {
        "ctx_memory": lambda: L.tc_lcc_ctx_memory(None, ctypes.byref(u64), ctypes.byref(u64)),
        "build_csr": lambda: L.tc_lcc_build_csr(None, 3, 0, None, None, 0, 0, None, None),
        "graph_info": lambda: L.tc_lcc_graph_info(None, None),
        "graph_export": lambda: L.tc_lcc_graph_export(None, None, None, None, None),
        "batch_submit": lambda: L.tc_lcc_batch_submit(None, 1, None, None, None, None),
        "batch_progress": lambda: L.tc_lcc_batch_progress(None, 0, 0, None),
        "autotune": lambda: L.tc_lcc_autotune(None, 0, None, 0, 0, None, None),
        "tuning_load": lambda: L.tc_lcc_tuning_load(None, None),
        "get_tuning": lambda: L.tc_lcc_get_tuning(None, None),
        "set_tuning": lambda: L.tc_lcc_set_tuning(None, None),
        "set_profiling": lambda: L.tc_lcc_set_profiling(None, 1),
        "graph_timings": lambda: L.tc_lcc_graph_timings(None, None),
        "server_create": lambda: L.tc_lcc_server_create(None, 0, 1, 1, None),
        "server_submit": lambda: L.tc_lcc_server_submit(None, None, None, None, None),
        "server_poll": lambda: L.tc_lcc_server_poll(None, 0, 0, None),
        "server_destroy": lambda: L.tc_lcc_server_destroy(None),
    }
    for name, call in calls.items():
        assert call() == pkg.INVALID_ARGUMENT, name
        assert L.tc_lcc_last_error(), name


def test_status_strings_are_distinct():
    L = pkg.lib()
    codes = [pkg.OK, pkg.INVALID_ARGUMENT, pkg.OUT_OF_MEMORY, pkg.OVER_BUDGET, pkg.NOT_READY, pkg.BUSY,
             pkg.DEVICE_ERROR, pkg.UNSUPPORTED]
    assert codes == list(range(8))
    texts = [L.tc_lcc_status_string(c) for c in codes]
    assert all(texts) and len(set(texts)) == len(texts)
    assert L.tc_lcc_status_string(99)
