"""tc_lcc_run_edges_noalloc through the C-ABI: the entry point for callers that cannot allocate.

Its outputs must equal tc_lcc_run_edges' (and the oracle's) bit for bit on two calls in a row,
the second with a smaller graph than the first (the shared static buffer keeps the first call's
contents, so anything not cleared would show).  The call must not touch the context's pool
(in-use and cached bytes unchanged), and a graph whose temporaries exceed the static buffer is
refused before any device work.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2202_13976_amd")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def outputs(n, m):
    out = (torch.full((n,), -1, dtype=torch.int64, device="cuda"),
           torch.full((n,), -1.0, dtype=torch.float64, device="cuda"),
           torch.full((max(m, 1),), -1, dtype=torch.int32, device="cuda"),
           torch.full((max(m, 1),), -1, dtype=torch.int32, device="cuda"),
           torch.full((max(m, 1),), -1, dtype=torch.int32, device="cuda"))
    # the calls below run on another stream: the fills must be done first
    torch.cuda.current_stream().synchronize()
    return out


def call(entry, g, outs, stream):
    tri, lcc, es, ed, ec = outs
    fn = getattr(pkg.lib(), entry)
    return fn(g.handle, ptr(tri), ptr(lcc), ptr(es), ptr(ed), ptr(ec), ctypes.c_void_p(stream.cuda_stream))


def host(outs, m):
    tri, lcc, es, ed, ec = outs
    return (tri.cpu().numpy().astype(np.uint64), lcc.cpu().numpy(), es[:m].cpu().numpy(), ed[:m].cpu().numpy(),
            ec[:m].cpu().numpy().view(np.uint32).astype(np.uint64))


def test_noalloc_equals_run_edges_twice_then_smaller():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = pkg.Context(0)
    graphs = []
    try:
        stream = torch.cuda.Stream()
        cases = [synth.rmat_scale(16, 16, seed=61), synth.rmat_scale(12, 16, seed=62)]  # second one smaller
        for n, s, d in cases:
            graphs.append((n, s, d, ctx.build_csr(n, dev(s), dev(d))))
        for n, s, d, g in graphs:
            m = int(g.info().m)
            print(f"[gpu] no-alloc per-edge run: n={n} m={m}", flush=True)
            ref_outs = outputs(n, m)
            assert call("tc_lcc_run_edges", g, ref_outs, stream) == pkg.OK, pkg.lib().tc_lcc_last_error()
            torch.cuda.synchronize()
            mem0 = ctx.memory()
            got_outs = outputs(n, m)
            st = call("tc_lcc_run_edges_noalloc", g, got_outs, stream)
            assert st == pkg.OK, pkg.lib().tc_lcc_last_error()
            assert ctx.memory() == mem0, "the no-allocation call touched the context's pool"
            torch.cuda.synchronize()
            ref, got = host(ref_outs, m), host(got_outs, m)
            for a, b in zip(ref, got):
                assert a.tobytes() == b.tobytes()
            og = oracle.csr(n, s, d)
            eu, ev, c = oracle.edge_counts(og)
            np.testing.assert_array_equal(got[2], eu)
            np.testing.assert_array_equal(got[3], ev)
            np.testing.assert_array_equal(got[4], c)
            t_ref, l_ref = oracle.tc_lcc(n, s, d)
            np.testing.assert_array_equal(got[0], t_ref)
            assert got[1].tobytes() == l_ref.tobytes()
        # beyond the static buffer: refused before any device work, outputs untouched
        n, s, d = synth.rmat_scale(19, 16, seed=63)
        big = ctx.build_csr(n, dev(s), dev(d))
        graphs.append((n, s, d, big))
        m = int(big.info().m)
        assert 20 * m + 4 * n > 64 << 20, "the case must exceed the static buffer (TC_LCC_NOALLOC_BYTES)"
        outs = outputs(n, m)
        st = call("tc_lcc_run_edges_noalloc", big, outs, stream)
        assert st == pkg.INVALID_ARGUMENT
        assert b"static buffer" in pkg.lib().tc_lcc_last_error()
        torch.cuda.synchronize()
        assert bool((outs[0] == -1).all()) and bool((outs[4] == -1).all())
    finally:
        for *_, g in graphs:
            g.free()
        ctx.close()
