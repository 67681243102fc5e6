"""Host logic of bench.py that needs no GPU: the count-kernel fingerprint that ties a stored
HBM-traffic figure to the code it was measured on (comment edits keep it, code edits do not),
and the algorithmic-byte formula."""
import importlib.util
import os
from types import SimpleNamespace

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_code_only_ignores_comments_and_blank_lines():
    b = load_bench()
    src = "int a = 1;  // one\n\n/* block\n comment */ int b = 2;\n"
    assert b._code_only(src) == "int a = 1;\n int b = 2;"
    assert b._code_only(src.replace("// one", "// a changed comment")) == b._code_only(src)
    assert b._code_only(src.replace("= 2", "= 3")) != b._code_only(src)


def test_count_bytes_formula():
    """B = 4 P + (8 + w) K + 4 S + (4 w + 4) A + 8 n, with w the offset width."""
    b = load_bench()
    info = SimpleNamespace(offset_bytes=8, wedges=1000, kept_in_edges=100, staged_entries=50,
                           active_vertices=20, n=30)
    assert b.count_bytes(info) == 4 * 1000 + 16 * 100 + 4 * 50 + 36 * 20 + 8 * 30
    info.offset_bytes = 4
    assert b.count_bytes(info) == 4 * 1000 + 12 * 100 + 4 * 50 + 20 * 20 + 8 * 30
