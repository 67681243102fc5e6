"""The streamed, partitioned build (tc_lcc_build_streamed) against the oracle.

The pairs are pulled from a source in chunks, once per pass, and the id range is split into
partitions by a histogram of the lower ends; the graph keeps compact reverse lists (u and a
16-bit row position per in-edge).  Every case runs the count on the result and compares every
vertex's t and LCC bits with the oracle, with one partition, several, and one per histogram bin
(down to one per id on small graphs), and with chunks that leave a ragged tail.  Also: the GPU
generator of the large-scale R-MAT recipe pair for pair against the C one, the error paths, and
a compact graph inside a batch.  Every case prints its name before it touches the GPU.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2202_13976_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def same_as_oracle(label, t, l, t_ref, l_ref):
    bad = np.nonzero(t != t_ref)[0]
    assert bad.size == 0, f"{label}: {bad.size} counts differ, first at v={bad[:5]}: {t[bad[:5]]} vs {t_ref[bad[:5]]}"
    assert l.tobytes() == np.asarray(l_ref, dtype=np.float64).tobytes(), f"{label}: LCC bits differ"


# ------------------------------------------------------------------ the generator

def test_gpu_generator_matches_host():
    """synth.GpuRmatFeistel writes the pairs synth.rmat_feistel computes, in any chunking."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    scale, m = 16, 16 << 16
    say(f"[gpu] R-MAT Feistel generator S{scale}: {m} pairs in uneven chunks")
    s_ref, d_ref = synth.rmat_feistel(scale, 0, m, seed=4)
    gen = synth.GpuRmatFeistel(scale, seed=4)
    s = torch.full((m,), -1, dtype=torch.int32, device="cuda")
    d = torch.full((m,), -1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    cuts = [0, 1, 64, 300001, 300002, 777777, m]
    for a, b in zip(cuts[:-1], cuts[1:]):
        gen.gen(a, b - a, s.data_ptr() + 4 * a, d.data_ptr() + 4 * a, stream)
    torch.cuda.synchronize()
    assert np.array_equal(s.cpu().numpy(), s_ref)
    assert np.array_equal(d.cpu().numpy(), d_ref)


# ------------------------------------------------------------------ parity

def _clique_ring(k, copies):
    """`copies` cliques K_k joined in a ring by one edge each, listed twice and with loops."""
    out = []
    for c in range(copies):
        base = c * k
        for i in range(k):
            for j in range(i + 1, k):
                out.append((base + i, base + j))
        out.append((base, ((c + 1) % copies) * k + 1))
        out.append((base + 2, base + 2))
    a = np.array(out + out[::-1], dtype=np.int32)
    return copies * k, a[:, 0].copy(), a[:, 1].copy()


CASES = {
    "er_3000_deg16": lambda: (3000, *synth.er(3000, 3000 * 8, seed=21)),
    "rmat_s12_loops_repeats": lambda: synth.rmat_scale(12, 16, seed=22),
    "clique_ring_40x6": lambda: _clique_ring(40, 6),
    "isolated_tail": lambda: (50000, np.array([0, 1, 2, 5], np.int32), np.array([1, 2, 0, 6], np.int32)),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("parts,chunk", [(0, 0), (5, 1000), (1, 777)])
def test_streamed_equals_oracle(ctx, name, parts, chunk):
    """parts: 0 = one partition, 5 = about a fifth of the pairs each, 1 = one per histogram bin."""
    n, s, d = CASES[name]()
    m_in = len(s)
    cap = 0 if parts == 0 else (1 if parts == 1 else max(1, m_in // parts))
    say(f"[gpu] streamed {name}: n={n} pairs={m_in} partition_pairs={cap} chunk={chunk}")
    t_ref, l_ref = oracle.tc_lcc(n, s, d)
    src = synth.DevicePairs(dev(s), dev(d))
    g = ctx.build_streamed(n, m_in, src.gen, chunk_pairs=chunk, partition_pairs=cap)
    try:
        info = g.info()
        assert info.compact == 1 and info.offset_bytes == 8
        ref = oracle.csr(n, s, d)
        assert info.m == ref.m
        assert np.array_equal(g.export()[0], np.asarray(ref.deg, dtype=np.int64))
        tri, lcc = g.run()
        torch.cuda.synchronize()
        same_as_oracle(name, tri.cpu().numpy().astype(np.uint64), lcc.cpu().numpy(), t_ref, l_ref)
    finally:
        g.free()


def test_streamed_rmat_feistel_s16_from_gpu_generator(ctx):
    """The large-scale recipe at scale 16, generated on the GPU chunk by chunk in every pass,
    seven partitions: every vertex against the oracle on the host generator's pairs."""
    scale, m = 16, 16 << 16
    n = 1 << scale
    s, d = synth.rmat_feistel(scale, 0, m, seed=3)
    say(f"[gpu] streamed R-MAT Feistel S{scale}: GPU source, 7 partitions, chunks of 100003")
    t_ref, l_ref = oracle.tc_lcc(n, s, d)
    gen = synth.GpuRmatFeistel(scale, seed=3)
    g = ctx.build_streamed(n, m, gen.gen, chunk_pairs=100003, partition_pairs=m // 7)
    try:
        tri, lcc = g.run()
        torch.cuda.synchronize()
        same_as_oracle("S16 Feistel", tri.cpu().numpy().astype(np.uint64), lcc.cpu().numpy(), t_ref, l_ref)
    finally:
        g.free()


def _golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


def test_streamed_dense_core_list_and_global_paths(ctx):
    """Lists longer than a block's hash (sorted-list launch) and, with the hash-only probe,
    beyond every table (searched in HBM), read through the compact reverse lists: every vertex
    against the oracle's stored digests."""
    name = "dense_core_13x200_drop5_p11_seed61"
    n, s, d = synth.dense_core(13, 200, 0.05, 11, 61)
    ref = _golden(name)
    src = synth.DevicePairs(dev(s), dev(d))
    probe0 = ctx.tuning().probe
    try:
        for probe in (pkg.PROBE_AUTO, pkg.PROBE_HASH):
            say(f"[gpu] streamed {name} probe={probe}, 3 partitions")
            ctx.set_tuning(probe=probe)
            g = ctx.build_streamed(n, len(s), src.gen, chunk_pairs=1 << 20, partition_pairs=len(s) // 3)
            try:
                info = g.info()
                assert info.max_out_degree > 2048
                assert (info.global_vertices > 0) == (probe == pkg.PROBE_HASH)
                tri, lcc = g.run()
                torch.cuda.synchronize()
                t = tri.cpu().numpy().astype(np.uint64)
                l = lcc.cpu().numpy()
                assert hashlib.sha256(np.ascontiguousarray(t, dtype="<u8").tobytes()).hexdigest() == \
                    ref["sha256_t_u64le"], f"{name} probe={probe}: t differs from the oracle's digest"
                assert hashlib.sha256(np.ascontiguousarray(l, dtype="<f8").tobytes()).hexdigest() == \
                    ref["sha256_lcc_f64le"], f"{name} probe={probe}: LCC bits differ"
            finally:
                g.free()
    finally:
        ctx.set_tuning(probe=probe0)


@pytest.mark.parametrize("probe", [pkg.PROBE_AUTO, pkg.PROBE_HASH])
def test_streamed_multipartite_beyond_every_table(ctx, probe):
    """Complete 50-partite graph with parts of 100: oriented lists of up to 4800 entries, beyond
    the LDS table's hash and sorted list: rank bitmaps in the block table by default, searched in
    HBM with the hash-only probe; closed form t = C(4900, 2) - 49 C(100, 2) (pinned in the
    oracle tests) for every vertex."""
    k, size = 50, 100
    nn = k * size
    iu, ju = np.triu_indices(nn, 1)
    keep = (iu // size) != (ju // size)
    s, d = iu[keep].astype(np.int32), ju[keep].astype(np.int32)
    say(f"[gpu] streamed complete {k}-partite, parts of {size}, 4 partitions, probe {probe}")
    src = synth.DevicePairs(dev(s), dev(d))
    probe0 = ctx.tuning().probe
    ctx.set_tuning(probe=probe)
    g = None
    try:
        g = ctx.build_streamed(nn, len(s), src.gen, chunk_pairs=1 << 21, partition_pairs=len(s) // 4)
        info = g.info()
        assert info.max_out_degree > 4096 and (info.global_vertices > 0) == (probe == pkg.PROBE_HASH)
        tri, lcc = g.run()
        torch.cuda.synchronize()
        dg = (k - 1) * size
        t_each = dg * (dg - 1) // 2 - (k - 1) * (size * (size - 1) // 2)
        assert np.all(tri.cpu().numpy() == t_each)
        want = np.float64(2 * t_each) / np.float64(dg * (dg - 1))
        assert np.all(lcc.cpu().numpy() == want)
    finally:
        if g is not None:
            g.free()
        ctx.set_tuning(probe=probe0)


# ------------------------------------------------------------------ errors and other paths

def test_streamed_error_paths(ctx):
    say("[gpu] streamed: id out of range, failing source, changing source, run_edges refused")
    n, s, d = synth.rmat_scale(10, 8, seed=30)
    bad_s = s.copy()
    bad_s[len(s) // 2] = n
    src = synth.DevicePairs(dev(bad_s), dev(d))
    with pytest.raises(pkg.TcLccError) as e:
        ctx.build_streamed(n, len(s), src.gen, chunk_pairs=1000)
    assert e.value.status == pkg.INVALID_ARGUMENT

    def failing(first, count, sp, dp, stp):
        raise RuntimeError("source broke")

    with pytest.raises(RuntimeError, match="source broke"):
        ctx.build_streamed(n, len(s), failing)

    # a source whose later passes put every pair into the first partition
    good = synth.DevicePairs(dev(s), dev(d))
    lo = np.minimum(s, d)
    first_part = synth.DevicePairs(dev(np.full_like(s, 0)), dev(np.where(s == d, 1, np.maximum(lo, 1))))
    calls = {"n": 0}
    per_pass = -(-len(s) // 500)

    def changing(first, count, sp, dp, stp):
        calls["n"] += 1
        (good if calls["n"] <= per_pass else first_part).gen(first, count, sp, dp, stp)

    with pytest.raises(pkg.TcLccError) as e:
        ctx.build_streamed(n, len(s), changing, chunk_pairs=500, partition_pairs=len(s) // 4)
    assert e.value.status == pkg.INVALID_ARGUMENT

    # the context is still usable, and per-edge counts are refused on a compact graph
    g = ctx.build_streamed(n, len(s), good.gen)
    try:
        with pytest.raises(pkg.TcLccError) as e:
            g.run_edges()
        assert e.value.status == pkg.UNSUPPORTED
        tri, lcc = g.run()
        torch.cuda.synchronize()
        t_ref, l_ref = oracle.tc_lcc(n, s, d)
        same_as_oracle("after errors", tri.cpu().numpy().astype(np.uint64), lcc.cpu().numpy(), t_ref, l_ref)
    finally:
        g.free()
    # no pairs at all
    g = ctx.build_streamed(7, 0, good.gen)
    try:
        tri, lcc = g.run()
        torch.cuda.synchronize()
        assert np.all(tri.cpu().numpy() == 0) and np.all(lcc.cpu().numpy() == 0.0)
    finally:
        g.free()


def test_streamed_graph_in_a_batch(ctx):
    """A compact graph in a batch takes the single-graph launches; every graph of the batch
    against the oracle."""
    raw = [synth.rmat_scale(9, 16, seed=40 + i) for i in range(3)]
    say("[gpu] batch with one streamed graph and three ordinary ones")
    n0, s0, d0 = synth.rmat_scale(11, 16, seed=44)
    src = synth.DevicePairs(dev(s0), dev(d0))
    gs = [ctx.build_streamed(n0, len(s0), src.gen, partition_pairs=len(s0) // 3)]
    gs += [ctx.build_csr(n, dev(s), dev(d), offset_bytes=4) for n, s, d in raw]
    refs = [oracle.tc_lcc(n0, s0, d0)] + [oracle.tc_lcc(n, s, d) for n, s, d in raw]
    try:
        tris = [torch.full((g.n,), -1, dtype=torch.int64, device="cuda") for g in gs]
        lccs = [torch.full((g.n,), -1.0, dtype=torch.float64, device="cuda") for g in gs]
        torch.cuda.current_stream().synchronize()
        tk = ctx.batch_submit(gs, tris, lccs)
        assert ctx.batch_poll(tk, block=True)[0]
        for i, (tri, lcc, (t_ref, l_ref)) in enumerate(zip(tris, lccs, refs)):
            same_as_oracle(f"batch graph {i}", tri.cpu().numpy().astype(np.uint64), lcc.cpu().numpy(), t_ref, l_ref)
    finally:
        for g in gs:
            g.free()
