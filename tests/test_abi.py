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
