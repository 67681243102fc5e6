"""Concurrency and failure paths of the library, against the oracle.

- several host threads submit batches that mix batched graphs with graphs that take the
  single-graph launches (their slots must never be shared);
- a tuning change while a batch holds a graph: the next tc_lcc_run rebuilds the schedule only
  after that batch is done;
- forced device-allocation failures (tc_lcc_debug_fail_alloc) at every allocation of a build,
  a run and a batch submission: each failing call returns OUT_OF_MEMORY, returns its memory
  to the context, and the same call then succeeds with the oracle's results.
Every case prints its name before it touches the GPU.
"""
import itertools
import threading

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2202_13976_amd")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pkg.Context(0)
    yield c
    import gc
    gc.collect()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def clique_pairs(k):
    a = np.array(list(itertools.combinations(range(k), 2)), dtype=np.int32)
    return a[:, 0].copy(), a[:, 1].copy()


@pytest.fixture(scope="module")
def mixed(ctx):
    """Small R-MAT and uniform graphs (batched) plus K_2200 (beyond a batched wave's LDS slice:
    single-graph launches), with the oracle's results."""
    raw = [synth.rmat_scale(10, 16, seed=s) for s in (31, 32, 33)]
    raw.append((3000, *synth.er(3000, 3000 * 12, seed=34)))
    raw.append((2200, *clique_pairs(2200)))
    graphs = [ctx.build_csr(n, dev(s), dev(d), offset_bytes=4) for n, s, d in raw]
    refs = []
    for n, s, d in raw[:-1]:
        refs.append(oracle.tc_lcc(n, s, d))
    t_k = np.full(2200, 2199 * 2198 // 2, dtype=np.uint64)   # K_n closed form (pinned in the oracle tests)
    refs.append((t_k, np.ones(2200)))
    yield graphs, refs
    for g in graphs:
        g.free()


def same_as_ref(tri, lcc, ref):
    t_ref, l_ref = ref
    np.testing.assert_array_equal(tri.cpu().numpy().astype(np.uint64), t_ref)
    assert lcc.cpu().numpy().tobytes() == np.asarray(l_ref, dtype=np.float64).tobytes()


def outputs(graphs):
    out = ([torch.full((g.n,), -1, dtype=torch.int64, device="cuda") for g in graphs],
           [torch.full((g.n,), -1.0, dtype=torch.float64, device="cuda") for g in graphs])
    # batches run on the library's streams: the fills must be done before the submission
    torch.cuda.current_stream().synchronize()
    return out


def test_threads_submit_batches_with_solo_graphs(ctx, mixed):
    say("[gpu] 4 threads x 6 batches with a single-launch graph each")
    graphs, refs = mixed
    errors = []

    def worker(k):
        try:
            for r in range(6):
                sel = list(range(len(graphs)))
                sel = sel[k % len(sel):] + sel[:k % len(sel)]
                if r % 2:
                    sel = sel[::-1]
                tris, lccs = outputs([graphs[i] for i in sel])
                tk = ctx.batch_submit([graphs[i] for i in sel], tris, lccs)
                done, nd = ctx.batch_poll(tk, block=True)
                assert done and nd == len(sel)
                for i, tri, lcc in zip(sel, tris, lccs):
                    same_as_ref(tri, lcc, refs[i])
        except Exception as e:  # noqa: BLE001 - reported in the main thread
            errors.append(repr(e))

    ths = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    assert not errors, errors


def test_tuning_change_while_batch_in_flight(ctx, mixed):
    say("[gpu] set_tuning + tc_lcc_run while a batch holds the graph")
    graphs, refs = mixed
    t0 = ctx.tuning().as_dict()
    try:
        for probe in (pkg.PROBE_HASH, pkg.PROBE_SORTED, pkg.PROBE_AUTO):
            tris, lccs = outputs(graphs)
            tk = ctx.batch_submit(graphs, tris, lccs)
            ctx.set_tuning(probe=probe, wave_work_max=1024 if probe != pkg.PROBE_AUTO else 4096)
            side = torch.cuda.Stream()
            runs = [g.run(stream=side) for g in graphs]
            assert ctx.batch_poll(tk, block=True)[0]
            torch.cuda.synchronize()
            for (tri, lcc), ref in zip(runs, refs):
                same_as_ref(tri, lcc, ref)
            for tri, lcc, ref in zip(tris, lccs, refs):
                same_as_ref(tri, lcc, ref)
    finally:
        ctx.set_tuning(**t0)


def test_forced_allocation_failures_build_run_batch():
    """A fresh context: every allocation of a build, a schedule rebuild and a batch submission
    is made to fail once in turn."""
    say("[gpu] forced allocation failures")
    c = pkg.Context(0)
    try:
        n, s, d = synth.rmat_scale(11, 16, seed=41)
        ref = oracle.tc_lcc(n, s, d)
        src, dst = dev(s), dev(d)
        in_use0, _ = c.memory()
        # build: fail allocation k for k = 0, 1, ... until the build needs fewer allocations
        g = None
        for k in range(200):
            c.fail_alloc_after(k)
            try:
                g = c.build_csr(n, src, dst, offset_bytes=8)
            except pkg.TcLccError as e:
                assert e.status == pkg.OUT_OF_MEMORY, e
                assert c.memory()[0] == in_use0, "a failed build must return its memory"
                continue
            break
        c.fail_alloc_after(-1)
        assert g is not None and k > 3, "the build never got past the injected failures"
        tri, lcc = g.run()
        torch.cuda.synchronize()
        same_as_ref(tri, lcc, ref)
        # schedule rebuild after a tuning change: its temporaries fail in turn
        for k in range(50):
            c.set_tuning(probe=pkg.PROBE_HASH if k % 2 == 0 else pkg.PROBE_AUTO)
            c.fail_alloc_after(k)
            try:
                tri, lcc = g.run()
            except pkg.TcLccError as e:
                assert e.status == pkg.OUT_OF_MEMORY, e
                continue
            finally:
                c.fail_alloc_after(-1)
            torch.cuda.synchronize()
            same_as_ref(tri, lcc, ref)
            break
        # batch: a first submission grows the slot, then bigger ones fail at each allocation
        others = [synth.rmat_scale(9, 8, seed=50 + i) for i in range(6)]
        gs = [c.build_csr(nn, dev(ss), dev(dd), offset_bytes=4) for nn, ss, dd in others]
        refs = [oracle.tc_lcc(nn, ss, dd) for nn, ss, dd in others]
        tris, lccs = outputs(gs[:1])
        tk = c.batch_submit(gs[:1], tris, lccs)
        assert c.batch_poll(tk, block=True)[0]
        same_as_ref(tris[0], lccs[0], refs[0])
        sel = gs + [g] * 3
        sel_refs = refs + [ref] * 3
        for k in range(8):
            tris, lccs = outputs(sel)
            c.fail_alloc_after(k)
            try:
                tk = c.batch_submit(sel, tris, lccs)
            except pkg.TcLccError as e:
                assert e.status == pkg.OUT_OF_MEMORY, e
                continue
            finally:
                c.fail_alloc_after(-1)
            assert c.batch_poll(tk, block=True)[0]
            for tri, lcc, r in zip(tris, lccs, sel_refs):
                same_as_ref(tri, lcc, r)
        for x in gs:
            x.free()
        g.free()
    finally:
        c.fail_alloc_after(-1)
        c.close()
