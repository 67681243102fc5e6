"""GPU parity: the HIP path against the CPU oracle, element by element, bit for bit.

Counts are integers and must match exactly; LCC is one IEEE division of the same
exact integers on both sides, so it must match bit for bit too (tolerance 0).
Every case prints its name before it touches the GPU.
"""
import hashlib
import itertools
import json
import math
import os
from fractions import Fraction

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


def gpu_run(ctx, n, s, d, offset_bytes=0, host=False):
    if host:
        g = ctx.build_csr(n, s, d, offset_bytes=offset_bytes)
    else:
        g = ctx.build_csr(n, torch.from_numpy(np.ascontiguousarray(s, dtype=np.int32)).cuda(),
                          torch.from_numpy(np.ascontiguousarray(d, dtype=np.int32)).cuda(),
                          offset_bytes=offset_bytes)
    tri, lcc = g.run()
    torch.cuda.synchronize()
    out = tri.cpu().numpy().astype(np.uint64), lcc.cpu().numpy()
    g.free()
    return out


def check(ctx, n, s, d, label, **kw):
    say(f"[gpu] {label}: n={n} pairs={len(s)} {kw}")
    t_ref, l_ref = oracle.tc_lcc(n, s, d)
    t, l = gpu_run(ctx, n, s, d, **kw)
    bad = np.nonzero(t != t_ref)[0]
    assert bad.size == 0, f"{label}: {bad.size} counts differ, first at v={bad[:5]}: {t[bad[:5]]} vs {t_ref[bad[:5]]}"
    assert l.tobytes() == l_ref.tobytes(), f"{label}: LCC bits differ"
    return t_ref


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


def digests(t, l):
    return (hashlib.sha256(np.ascontiguousarray(t, dtype="<u8").tobytes()).hexdigest(),
            hashlib.sha256(np.ascontiguousarray(l, dtype="<f8").tobytes()).hexdigest())


def check_golden(name, t, l, n, s, d):
    """Whole-vector comparison with the oracle's stored digests (written by
    tests/golden/make_golden.py from oracle/ alone); on a mismatch, the oracle recomputes
    sampled vertices one by one to name the first differences."""
    ref = golden(name)
    assert ref["n"] == n and ref["raw_pairs"] == len(s)
    assert t[:16].tolist() == ref["t_head"]
    assert [float(x).hex() for x in l[:16]] == ref["lcc_head"]
    assert int(t.sum()) // 3 == ref["triangles"]
    dt, dl = digests(t, l)
    if dt != ref["sha256_t_u64le"]:
        g = oracle.csr(n, s, d)
        rng = np.random.default_rng(1)
        pick = np.unique(np.concatenate([rng.choice(n, min(n, 400), replace=False), np.argsort(g.deg)[-16:]]))
        want = oracle.tc_vertices(g, pick)
        bad = pick[want != t[pick]]
        raise AssertionError(f"{name}: t differs from the oracle's digest; sampled mismatches at {bad[:8]}")
    assert dl == ref["sha256_lcc_f64le"], f"{name}: LCC bits differ from the oracle's digest"


def arr(pairs):
    if not pairs:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    a = np.array(pairs, dtype=np.int32)
    return a[:, 0].copy(), a[:, 1].copy()


# ------------------------------------------------------------------ the workloads

def test_er4096_int32(ctx):
    n, s, d = synth.er_4096(seed=1)
    check(ctx, n, s, d, "ER n=4096 deg16", offset_bytes=4)


@pytest.mark.parametrize("scale", [8, 10, 12, 14, 16])
@pytest.mark.parametrize("ob", [4, 8])
def test_rmat_small(ctx, scale, ob):
    n, s, d = synth.rmat_scale(scale, 16, seed=scale)
    check(ctx, n, s, d, f"RMAT S{scale}", offset_bytes=ob)


def test_rmat_s20_full(ctx):
    """R-MAT scale 20, edge factor 16, int64 offsets: every vertex against the oracle (its
    stored full-vector digests)."""
    n, s, d = synth.rmat_scale(20, 16, seed=1)
    say(f"[gpu] RMAT S20 EF16: n={n} pairs={len(s)}")
    t, l = gpu_run(ctx, n, s, d, offset_bytes=8)
    check_golden("rmat_s20_ef16_seed1", t, l, n, s, d)


def test_rmat_s23_full(ctx):
    """R-MAT scale 23 at full size, as the benchmark runs it: all 8,388,608 counts and LCC
    values against the oracle's stored digests."""
    n, s, d = synth.rmat_scale(23, 16, seed=1)
    say("[gpu] RMAT S23 EF16 full size")
    t, l = gpu_run(ctx, n, s, d, offset_bytes=8)
    check_golden("rmat_s23_ef16_seed1", t, l, n, s, d)


def test_dense_core_list_and_global_paths(ctx):
    """A dense core that is not a clique (13 parts of 200, 5 % of the cross pairs dropped) with
    an R-MAT periphery: |N+(v)| passes 2048 at the lowest-ranked core vertices and most
    candidates of a core list miss.  The default probe keeps those lists in the block table as
    a rank bitmap (their ranks lie close together, so the bitmap fits), the hash-only probe sends
    them to the global-memory path (the miss branch runs); the sorted and hybrid probes take
    them in LDS.  Every vertex against the oracle's digests."""
    name = "dense_core_13x200_drop5_p11_seed61"
    n, s, d = synth.dense_core(13, 200, 0.05, 11, 61)
    probe0 = ctx.tuning().probe
    try:
        for probe, ob in [(pkg.PROBE_AUTO, 8), (pkg.PROBE_HASH, 4), (pkg.PROBE_SORTED, 8), (pkg.PROBE_MERGE, 4)]:
            say(f"[gpu] {name} probe={probe} offsets={ob}")
            ctx.set_tuning(probe=probe)
            g = ctx.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(), offset_bytes=ob)
            try:
                info = g.info()
                assert info.max_out_degree > 2048
                assert (info.global_vertices > 0) == (probe == pkg.PROBE_HASH)
                tri, lcc = g.run()
                torch.cuda.synchronize()
            finally:
                g.free()
            check_golden(name, tri.cpu().numpy().astype(np.uint64), lcc.cpu().numpy(), n, s, d)
    finally:
        ctx.set_tuning(probe=probe0)


@pytest.mark.parametrize("probe", [pkg.PROBE_AUTO, pkg.PROBE_HASH])
def test_multipartite_beyond_every_table(ctx, probe):
    """Complete 50-partite graph with parts of 100: all degrees equal, so ranks follow ids, the
    first part has no in-edges, and the first vertex of every later part has |N+(v)| of up to
    n - 2 * 100 = 4800, beyond the LDS table even as a sorted list.  The default probe takes
    those lists as rank bitmaps in the block table (4800 ranks span 150 words); the hash-only
    probe searches them in HBM, where a candidate in the vertex's own part misses.  Closed form
    t = C(4900, 2) - 49 C(100, 2), LCC = 2t/(d(d-1)) (pinned in the oracle tests), and the
    oracle on sampled vertices."""
    k, size = 50, 100
    nn = k * size
    iu, ju = np.triu_indices(nn, 1)
    keep = (iu // size) != (ju // size)
    s, d = iu[keep].astype(np.int32), ju[keep].astype(np.int32)
    say(f"[gpu] complete {k}-partite, parts of {size}, probe {probe}")
    probe0 = ctx.tuning().probe
    ctx.set_tuning(probe=probe)
    try:
        g = ctx.build_csr(nn, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(), offset_bytes=8)
        try:
            assert (g.info().global_vertices > 0) == (probe == pkg.PROBE_HASH)
            tri, lcc = g.run()
            torch.cuda.synchronize()
        finally:
            g.free()
    finally:
        ctx.set_tuning(probe=probe0)
    t = tri.cpu().numpy().astype(np.uint64)
    deg = (k - 1) * size
    want = math.comb(deg, 2) - (k - 1) * math.comb(size, 2)
    assert np.all(t == want)
    assert np.all(lcc.cpu().numpy() == float(Fraction(2 * want, deg * (deg - 1))))
    og = oracle.csr(nn, s, d)
    pick = np.arange(0, nn, 97)
    np.testing.assert_array_equal(oracle.tc_vertices(og, pick), t[pick])


# ------------------------------------------------------------------ strategies (results never depend on them)

@pytest.mark.parametrize("probe", [pkg.PROBE_HASH, pkg.PROBE_SORTED, pkg.PROBE_BITMAP, pkg.PROBE_MERGE])
@pytest.mark.parametrize("group,wave_max", [(0, 4096), (0, 0), (0, 1 << 40), (1, 0), (2, 0)])
def test_strategies(ctx, probe, group, wave_max):
    ctx.set_tuning(probe=probe, group=group, wave_work_max=wave_max)
    try:
        for label, (n, s, d) in [("RMAT S13", synth.rmat_scale(13, 16, seed=5)),
                                 ("ER 3000", (3000, *synth.er(3000, 3000 * 20, seed=6)))]:
            check(ctx, n, s, d, f"{label} probe={probe} group={group} wave_max={wave_max}", offset_bytes=8)
    finally:
        ctx.set_tuning(probe=pkg.PROBE_AUTO, group=0, wave_work_max=4096)


@pytest.mark.parametrize("ratio", [1, 100, 100000])
def test_hybrid_rule_branches(ctx, ratio):
    """The hybrid probe (Eq. 3): ratio 1 makes nearly every in-edge a binary search (both
    directions: tails longer and shorter than N+(v)), 100000 nearly every one a merge path,
    100 is the rule as printed.  Skewed, dense and uniform graphs, one- and multi-wave
    vertices."""
    ctx.set_tuning(probe=pkg.PROBE_MERGE, merge_ratio_x100=ratio)
    try:
        hub_s, hub_d = clique(120)
        star = np.arange(120, 2120, dtype=np.int32)
        hs = np.concatenate([hub_s, np.repeat(np.arange(0, 40, dtype=np.int32), 50), star[:1000]])
        hd = np.concatenate([hub_d, star, np.roll(star, 7)[:1000]])
        for label, (n, s, d) in [("RMAT S14", synth.rmat_scale(14, 16, seed=21)),
                                 ("ER 2000 dense", (2000, *synth.er(2000, 2000 * 60, seed=22))),
                                 ("K120 + stars", (2120, hs, hd))]:
            for ob in (4, 8):
                check(ctx, n, s, d, f"{label} merge ratio={ratio}", offset_bytes=ob)
    finally:
        ctx.set_tuning(probe=pkg.PROBE_AUTO, merge_ratio_x100=0)


# ------------------------------------------------------------------ edge cases

def test_edge_cases(ctx):
    cases = {
        "single vertex": (1, [], ),
        "no edges": (7, []),
        "only loops": (4, [(0, 0), (1, 1), (3, 3)]),
        "one triangle, repeated both ways": (3, [(0, 1), (1, 0), (1, 2), (2, 1), (0, 2), (0, 2), (2, 2)]),
        "star": (60, [(0, i) for i in range(1, 60)]),
        "wheel": (31, [(0, i) for i in range(1, 31)] + [(i, i % 30 + 1) for i in range(1, 31)]),
        "K40": (40, list(itertools.combinations(range(40), 2))),
        "isolated tail": (100000, [(0, 1), (1, 2), (2, 0), (99999, 0), (99999, 1)]),
    }
    for label, (n, pairs) in cases.items():
        s, d = arr(pairs)
        check(ctx, n, s, d, label)


@pytest.mark.parametrize("pairs", [16383, 16384, 16385, 32769])
def test_radix_tile_edges(ctx, pairs):
    """Pair counts at and around the sort's 16384-key tile, so that the last tile is full,
    one key long, or one key short."""
    n = 3000
    s, d = synth.er(n, pairs, seed=pairs)
    check(ctx, n, s, d, f"ER pairs at a tile edge ({pairs})", offset_bytes=4)


def test_ids_at_power_of_two(ctx):
    """Vertex ids that need one more key bit than the rest of the graph: n = 2^16 + 1, with
    triangles through the ids 2^16 - 1 and 2^16."""
    n = (1 << 16) + 1
    top, nxt = n - 1, n - 2
    pairs = [(0, top), (top, nxt), (nxt, 0), (1, top), (1, nxt), (2, 3), (3, top), (2, top)]
    pairs += [(i, i + 1) for i in range(4, 200)] + [(i, i + 2) for i in range(4, 200, 3)]
    s, d = arr(pairs)
    check(ctx, n, s, d, "ids 2^16 - 1 and 2^16", offset_bytes=8)


def test_heavy_duplicates(ctx):
    """Every undirected pair given ten times, in both directions and shuffled, plus loops."""
    n, s, d = synth.rmat_scale(11, 8, seed=5)
    rng = np.random.default_rng(3)
    s10 = np.concatenate([s, d] * 5 + [np.arange(0, n, 7, dtype=np.int32)])
    d10 = np.concatenate([d, s] * 5 + [np.arange(0, n, 7, dtype=np.int32)])
    p = rng.permutation(len(s10))
    check(ctx, n, s10[p].astype(np.int32), d10[p].astype(np.int32), "pairs x10, both ways, loops")


def test_hub_over_random_graph(ctx):
    """One vertex joined to all others over an ER graph: the hub ranks last (no out-list, every
    vertex's in-edge), and every triangle through it is closed at its middle vertex."""
    n = 5000
    s, d = synth.er(n, 40000, seed=8)
    hub = np.full(n - 1, 1234, dtype=np.int32)
    others = np.array([v for v in range(n) if v != 1234], dtype=np.int32)
    for ob in (4, 8):
        check(ctx, n, np.concatenate([s, hub]), np.concatenate([d, others]), f"hub + ER (offsets {ob})",
              offset_bytes=ob)


@pytest.mark.parametrize("k", [100, 200])
def test_wide_ids_packed_and_payload_in_edges(ctx, k):
    """n just above 2^24 (25-bit ids), so the in-edge sort key takes four digit passes and leaves
    32 bits under it for u and the row position.  A K_k at the top ids sets the largest
    out-list: k = 100 (positions in 7 bits) still packs u and the position into the word, k = 200
    (8 bits) does not, and the builder falls back to the edge index and a payload array.  Sparse
    uniform pairs over the whole id range and a few links into the clique come on top."""
    n = (1 << 24) + 3
    top = np.arange(n - k, n, dtype=np.int32)
    iu, ju = np.triu_indices(k, 1)
    s0, d0 = synth.er(n, 20000, seed=k)
    links_s = np.arange(0, 5000, 50, dtype=np.int32)
    links_d = top[(links_s // 50) % k]
    s = np.concatenate([top[iu], s0, links_s])
    d = np.concatenate([top[ju], d0, links_d])
    check(ctx, n, s.astype(np.int32), d.astype(np.int32), f"25-bit ids with K{k} at the top", offset_bytes=8)


def clique(n):
    a = np.array(list(itertools.combinations(range(n), 2)), dtype=np.int32)
    return a[:, 0].copy(), a[:, 1].copy()


def test_large_clique_global_path(ctx):
    """K_2800: |N+(v)| reaches 2799, beyond the largest hash table (2048 keys at load 1/2):
    by default such vertices keep the block table as a rank bitmap (their ranks are
    consecutive); with the hash-only probe they take the global-memory path.  Reference: the closed form for K_n (t = C(n-1, 2),
    LCC = 1), which the oracle's own pins establish; running the oracle on 3.9 M edges would be
    slow."""
    n = 2800
    s, d = clique(n)
    probe0 = ctx.tuning().probe
    try:
        for probe, ob, global_path in [(pkg.PROBE_AUTO, 8, False), (pkg.PROBE_HASH, 8, True),
                                       (pkg.PROBE_SORTED, 4, False), (pkg.PROBE_MERGE, 4, False)]:
            say(f"[gpu] K{n} probe={probe} offsets={ob}")
            ctx.set_tuning(probe=probe)
            g = ctx.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(), offset_bytes=ob)
            assert (g.info().global_vertices > 0) == global_path
            tri, lcc = g.run()
            torch.cuda.synchronize()
            assert bool((tri == (n - 1) * (n - 2) // 2).all()) and bool((lcc == 1.0).all())
            g.free()
    finally:
        ctx.set_tuning(probe=probe0)


def test_clique_beyond_every_table(ctx):
    """K_8200: |N+(v)| reaches 8199, beyond the LDS table even as a sorted list (4096 keys), and
    the longest lists' rank bitmaps (their words, first indices, counters and spare words) exceed
    the block's 32 KiB too, so the default probe sends those ranks to the global-memory path
    (rank 0 has no in-edge, so no work); the shorter lists beyond the hash take the bitmap.
    Reference: the closed form for K_n."""
    n = 8200
    say(f"[gpu] K{n} (global path under the default probe)")
    s, d = (x.astype(np.int32) for x in np.triu_indices(n, 1))
    g = ctx.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(), offset_bytes=8)
    # rank r holds N+ = {r + 1 .. n - 1}: dv = n - 1 - r entries over a span of dv ranks
    dv = n - 1 - np.arange(1, n - 1)
    bitmap = 8 * (((dv + 31) >> 5) + 1) + 4 * dv + 4 * 64
    want_global = int(np.count_nonzero((dv > 4096) & (bitmap > 4096 * 8)))
    assert want_global > 0 and g.info().global_vertices == want_global
    tri, lcc = g.run()
    torch.cuda.synchronize()
    assert bool((tri == (n - 1) * (n - 2) // 2).all()) and bool((lcc == 1.0).all())
    g.free()


def test_host_inputs_and_repeats(ctx):
    n, s, d = synth.rmat_scale(12, 16, seed=77)
    t_ref = check(ctx, n, s, d, "host inputs", host=True)
    g = ctx.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    outs = []
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for i in range(4):
        tri, lcc = g.run(stream=streams[i % 2])
        outs.append((tri, lcc))
    torch.cuda.synchronize()
    for tri, _ in outs:
        assert np.array_equal(tri.cpu().numpy().astype(np.uint64), t_ref)
    g.free()


def test_invalid_inputs(ctx):
    s = torch.tensor([0, 1, 5], dtype=torch.int32, device="cuda")
    d = torch.tensor([1, 2, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(pkg.TcLccError) as e:
        ctx.build_csr(5, s, d)
    assert e.value.status == pkg.INVALID_ARGUMENT
    with pytest.raises(pkg.TcLccError) as e:
        ctx.build_csr(0, s, d)
    assert e.value.status == pkg.INVALID_ARGUMENT
    neg = torch.tensor([-1], dtype=torch.int32, device="cuda")
    with pytest.raises(pkg.TcLccError):
        ctx.build_csr(5, neg, neg)


@pytest.mark.parametrize("row_sort_max", [0, 1])
def test_builder_structure(ctx, row_sort_max):
    """The exported CSR: degrees, rank order by (degree, id), orientation and sorted lists,
    and the schedule's counts (kept in-edges, probes, active vertices, staged entries) that
    the roofline accounting uses.  row_sort_max 0 sorts rows in registers after the sort by
    source (rows of 2..64 and of 65..4096 entries take different kernels); 1 sends the
    oriented edges through the full radix sort instead."""
    n, s, d = synth.rmat_scale(14, 16, seed=3)
    g_ref = oracle.csr(n, s, d)
    say(f"[gpu] builder structure RMAT S14 row_sort_max={row_sort_max}")
    t0 = ctx.tuning().row_sort_max
    ctx.set_tuning(row_sort_max=row_sort_max)
    try:
        g = ctx.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(), offset_bytes=8)
    finally:
        ctx.set_tuning(row_sort_max=t0)
    deg, order, off, adj = g.export()
    info = g.info()
    g.free()
    np.testing.assert_array_equal(deg, g_ref.deg)
    assert info.m == g_ref.m and info.n == n
    want_order = np.lexsort((np.arange(n), g_ref.deg))
    np.testing.assert_array_equal(order, want_order)
    src = np.repeat(np.arange(n), np.diff(off))
    assert np.all(src < adj), "every oriented edge goes to a higher rank"
    same = src[1:] == src[:-1]
    assert np.all(adj[1:][same] > adj[:-1][same]), "lists strictly ascending"
    a, b = order[src], order[adj]
    got = np.sort(np.minimum(a, b).astype(np.int64) * n + np.maximum(a, b))
    rows = np.repeat(np.arange(n), g_ref.deg)
    keep = rows < g_ref.adj
    want = np.sort(rows[keep].astype(np.int64) * n + g_ref.adj[keep])
    np.testing.assert_array_equal(got, want)
    assert info.max_out_degree == int(np.diff(off).max())
    assert info.max_out_degree > 64, "the workload must have rows for the LDS row sort"
    # kept in-edges: oriented edges with a nonempty tail whose target has a nonempty N+
    dplus = np.diff(off)
    tail = off[src + 1] - np.arange(len(adj)) - 1
    kept = (tail > 0) & (dplus[adj] > 0)
    assert info.kept_in_edges == int(np.count_nonzero(kept))
    # probes (oriented wedges that can close): the sum of the kept in-edges' tail lengths
    assert info.wedges == int(tail[kept].sum())
    # active vertices: those with probes (a kept in-edge); staged entries: their |N+(v)|
    work = np.bincount(adj[kept], weights=tail[kept], minlength=n)
    active = work > 0
    assert info.active_vertices == int(np.count_nonzero(active))
    assert info.staged_entries == int(dplus[active].sum())
