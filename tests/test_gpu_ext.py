"""GPU parity of the two extensions of the count, through the C-ABI, against the oracle:

- per-edge triangle counts (tc_lcc_run_edges): the entries c_ij of C = A A o A (Sec. V-B),
  one per undirected edge in (lower id, higher id) order, bit-exact;
- directed graphs (tc_lcc_build_directed + tc_lcc_run): the numerator of Eq. 1 and its
  clustering coefficient, bit-exact (one IEEE division of exact integers on both sides).

Every case prints its name before it touches the GPU.
"""
import itertools
import math
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def run_edges(ctx, n, s, d, ob=0):
    g = ctx.build_csr(n, dev(s), dev(d), offset_bytes=ob)
    tri, lcc, es, ed, ec = g.run_edges()
    t1, l1 = g.run()
    torch.cuda.synchronize()
    out = (tri.cpu().numpy().astype(np.uint64), lcc.cpu().numpy(), es.cpu().numpy(), ed.cpu().numpy(),
           ec.cpu().numpy().view(np.uint32).astype(np.uint64))
    assert torch.equal(tri, t1) and lcc.cpu().numpy().tobytes() == l1.cpu().numpy().tobytes(), \
        "per-vertex results of run_edges differ from run"
    g.free()
    return out


def check_edges(ctx, n, s, d, label, ob=0):
    say(f"[gpu] edges {label}: n={n} pairs={len(s)} offsets={ob}")
    t, l, es, ed, ec = run_edges(ctx, n, s, d, ob)
    g = oracle.csr(n, s, d)
    eu, ev, c = oracle.edge_counts(g)
    np.testing.assert_array_equal(es, eu)
    np.testing.assert_array_equal(ed, ev)
    bad = np.nonzero(ec != c)[0]
    assert bad.size == 0, f"{label}: {bad.size} edge counts differ, first {[(eu[i], ev[i], ec[i], c[i]) for i in bad[:4]]}"
    t_ref = oracle.tc_forward(g)
    np.testing.assert_array_equal(t, t_ref)
    assert l.tobytes() == oracle.lcc(g, t_ref).tobytes()


# ------------------------------------------------------------------ per-edge counts

@pytest.mark.parametrize("ob", [4, 8])
def test_edges_workload_shapes(ctx, ob):
    n, s, d = synth.er_4096(seed=1)
    check_edges(ctx, n, s, d, "ER n=4096", ob)
    for scale in (10, 13, 15):
        n, s, d = synth.rmat_scale(scale, 16, seed=scale + 100)
        check_edges(ctx, n, s, d, f"RMAT S{scale}", ob)


@pytest.mark.parametrize("probe,group,wave_max", [(pkg.PROBE_HASH, 0, 4096), (pkg.PROBE_SORTED, 0, 4096),
                                                  (pkg.PROBE_MERGE, 0, 0), (pkg.PROBE_AUTO, 1, 0),
                                                  (pkg.PROBE_AUTO, 2, 0), (pkg.PROBE_AUTO, 0, 1 << 40)])
def test_edges_schedules(ctx, probe, group, wave_max):
    """The extended count follows the schedule of each setting (block, wave, sorted-list and
    global classes); results never depend on it."""
    ctx.set_tuning(probe=probe, group=group, wave_work_max=wave_max)
    try:
        n, s, d = synth.rmat_scale(13, 16, seed=5)
        check_edges(ctx, n, s, d, f"RMAT S13 probe={probe} group={group}", 8)
        check_edges(ctx, 3000, *synth.er(3000, 3000 * 20, seed=6), f"ER 3000 probe={probe} group={group}", 4)
    finally:
        ctx.set_tuning(probe=pkg.PROBE_AUTO, group=0, wave_work_max=4096)


def test_edges_edge_cases(ctx):
    cases = {
        "no edges": (7, []),
        "only loops": (4, [(0, 0), (1, 1), (3, 3)]),
        "one triangle, repeated both ways": (3, [(0, 1), (1, 0), (1, 2), (2, 1), (0, 2), (0, 2), (2, 2)]),
        "star": (60, [(0, i) for i in range(1, 60)]),
        "wheel": (31, [(0, i) for i in range(1, 31)] + [(i, i % 30 + 1) for i in range(1, 31)]),
        "K40": (40, list(itertools.combinations(range(40), 2))),
    }
    for label, (n, pairs) in cases.items():
        a = np.array(pairs, dtype=np.int32).reshape(-1, 2)
        check_edges(ctx, n, a[:, 0].copy(), a[:, 1].copy(), label)


@pytest.mark.parametrize("k,size,probe", [(13, 200, pkg.PROBE_AUTO), (13, 200, pkg.PROBE_HASH),
                                          (50, 100, pkg.PROBE_AUTO)])
def test_edges_dense_multipartite(ctx, k, size, probe):
    """Complete k-partite graphs: every edge {a, b} lies on n - 2 size triangles (the vertices
    outside both parts), every vertex on C(d, 2) - (k-1) C(size, 2).  Ranks follow ids (equal
    degrees), so the longest active lists hold n - 2 size entries: 2200 for 13 x 200 and 4800 for
    50 x 100, beyond the hash; the default probe keeps them in the block table as rank bitmaps
    (their ranks lie close together), the hash-only probe searches them in HBM."""
    nn = k * size
    iu, ju = np.triu_indices(nn, 1)
    keep = (iu // size) != (ju // size)
    s, d = iu[keep].astype(np.int32), ju[keep].astype(np.int32)
    say(f"[gpu] edges complete {k}-partite parts of {size} probe={probe}")
    ctx.set_tuning(probe=probe)
    g = None
    try:
        g = ctx.build_csr(nn, dev(s), dev(d), offset_bytes=8)
        assert (g.info().global_vertices > 0) == (probe == pkg.PROBE_HASH)
        tri, lcc, es, ed, ec = g.run_edges()
        torch.cuda.synchronize()
    finally:
        if g is not None:
            g.free()
        ctx.set_tuning(probe=pkg.PROBE_AUTO)
    np.testing.assert_array_equal(es.cpu().numpy(), s)
    np.testing.assert_array_equal(ed.cpu().numpy(), d)
    assert bool((ec == nn - 2 * size).all())
    deg = (k - 1) * size
    assert bool((tri == math.comb(deg, 2) - (k - 1) * math.comb(size, 2)).all())


def test_edges_rmat_s18_sampled_invariants(ctx):
    """R-MAT S18 (4.1 M pairs): the full edge list against the oracle's, plus the identities
    sum_e c(e) = sum_v t(v) and sum of c over the edges at v = 2 t(v)."""
    n, s, d = synth.rmat_scale(18, 16, seed=7)
    say("[gpu] edges RMAT S18")
    t, l, es, ed, ec = run_edges(ctx, n, s, d, 8)
    g = oracle.csr(n, s, d)
    eu, ev, c = oracle.edge_counts(g)
    np.testing.assert_array_equal(es, eu)
    np.testing.assert_array_equal(ed, ev)
    np.testing.assert_array_equal(ec, c)
    assert int(ec.sum()) == int(t.sum())
    per_v = np.bincount(es, weights=ec, minlength=n) + np.bincount(ed, weights=ec, minlength=n)
    np.testing.assert_array_equal(per_v.astype(np.uint64), 2 * t)


# ------------------------------------------------------------------ directed (Eq. 1)

def directed_gpu(ctx, n, s, d, ob=0):
    g = ctx.build_directed(n, dev(s), dev(d), offset_bytes=ob)
    assert g.info().directed == 1
    tri, lcc = g.run()
    torch.cuda.synchronize()
    out = tri.cpu().numpy().astype(np.uint64), lcc.cpu().numpy()
    g.free()
    return out


def check_directed(ctx, n, s, d, label, ob=0):
    say(f"[gpu] directed {label}: n={n} pairs={len(s)} offsets={ob}")
    num, lcc = directed_gpu(ctx, n, s, d, ob)
    num_ref, lcc_ref = oracle.tc_lcc_directed(n, s, d)
    bad = np.nonzero(num != num_ref)[0]
    assert bad.size == 0, f"{label}: {bad.size} numerators differ, first at {bad[:5]}: {num[bad[:5]]} vs {num_ref[bad[:5]]}"
    assert lcc.tobytes() == lcc_ref.tobytes(), f"{label}: Eq. 1 bits differ"


@pytest.mark.parametrize("ob", [4, 8])
def test_directed_workload_shapes(ctx, ob):
    """R-MAT pairs taken as directed edges (their direction as drawn), uniform pairs, and a mix
    where a third of the edges also appear reversed."""
    for scale in (10, 14, 16):
        n, s, d = synth.rmat_scale(scale, 16, seed=scale + 200)
        check_directed(ctx, n, s, d, f"RMAT S{scale}", ob)
    n, s, d = synth.er_4096(seed=3)
    check_directed(ctx, n, s, d, "ER 4096", ob)
    n, s, d = synth.rmat_scale(13, 16, seed=77)
    k = len(s) // 3
    check_directed(ctx, n, np.concatenate([s, d[:k]]), np.concatenate([d, s[:k]]), "RMAT S13 partly reciprocal", ob)


@pytest.mark.parametrize("probe,group", [(pkg.PROBE_HASH, 0), (pkg.PROBE_SORTED, 0), (pkg.PROBE_AUTO, 1),
                                         (pkg.PROBE_AUTO, 2)])
def test_directed_schedules(ctx, probe, group):
    ctx.set_tuning(probe=probe, group=group)
    try:
        n, s, d = synth.rmat_scale(13, 16, seed=8)
        check_directed(ctx, n, s, d, f"RMAT S13 probe={probe} group={group}", 8)
    finally:
        ctx.set_tuning(probe=pkg.PROBE_AUTO, group=0)


def test_directed_symmetric_equals_undirected(ctx):
    """Both directions of every edge: the numerator of Eq. 1 is 2 t(v) and its LCC has Eq. 2's bits."""
    n, s, d = synth.rmat_scale(14, 16, seed=9)
    say("[gpu] directed symmetric input vs undirected")
    num, lcc_d = directed_gpu(ctx, n, np.concatenate([s, d]), np.concatenate([d, s]))
    g = ctx.build_csr(n, dev(s), dev(d))
    tri, lcc = g.run()
    torch.cuda.synchronize()
    g.free()
    np.testing.assert_array_equal(num, 2 * tri.cpu().numpy().astype(np.uint64))
    assert lcc_d.tobytes() == lcc.cpu().numpy().tobytes()


@pytest.mark.parametrize("n,probe", [(300, pkg.PROBE_AUTO), (2600, pkg.PROBE_AUTO), (2600, pkg.PROBE_HASH),
                                     (4400, pkg.PROBE_AUTO)])
def test_directed_tournament_closed_form(ctx, n, probe):
    """Transitive tournament (a -> b iff a < b, pairs given in shuffled order): out(i) = {i+1 ..
    n-1}, numerator C(n-1-i, 2), LCC 1/2.  Its skeleton is K_n, so n = 2600 sends the longest
    lists through the sorted-list table (default probe) or the HBM search (hash-only), and
    n = 4400 through the HBM search."""
    s, d = (x.astype(np.int32) for x in np.triu_indices(n, 1))
    p = np.random.default_rng(n).permutation(len(s))
    say(f"[gpu] directed transitive tournament n={n} probe={probe}")
    ctx.set_tuning(probe=probe)
    try:
        num, lcc = directed_gpu(ctx, n, s[p], d[p], 8)
    finally:
        ctx.set_tuning(probe=pkg.PROBE_AUTO)
    dout = n - 1 - np.arange(n)
    assert num.tolist() == [math.comb(int(k), 2) for k in dout]
    assert np.all(lcc[dout >= 2] == float(Fraction(1, 2))) and np.all(lcc[dout < 2] == 0.0)


def test_directed_edge_cases(ctx):
    cases = {
        "no edges": (5, []),
        "only loops": (3, [(0, 0), (2, 2)]),
        "directed 3-cycle": (3, [(0, 1), (1, 2), (2, 0)]),
        "transitive triangle, repeated": (3, [(0, 1), (0, 1), (1, 2), (0, 2), (0, 2)]),
        "complete digraph K5": (5, [(a, b) for a in range(5) for b in range(5) if a != b]),
        "out-star": (40, [(0, i) for i in range(1, 40)]),
        "in-star": (40, [(i, 0) for i in range(1, 40)]),
    }
    for label, (n, pairs) in cases.items():
        a = np.array(pairs, dtype=np.int32).reshape(-1, 2)
        check_directed(ctx, n, a[:, 0].copy(), a[:, 1].copy(), label)


def test_directed_in_a_batch(ctx):
    """A directed graph in a batch takes the single-graph launches and gives Eq. 1; the
    undirected graphs beside it are unchanged."""
    say("[gpu] directed graph in a batch")
    n1, s1, d1 = synth.rmat_scale(11, 16, seed=31)
    n2, s2, d2 = synth.rmat_scale(11, 16, seed=32)
    g1 = ctx.build_directed(n1, dev(s1), dev(d1))
    g2 = ctx.build_csr(n2, dev(s2), dev(d2))
    tris = [torch.empty(n1, dtype=torch.int64, device="cuda"), torch.empty(n2, dtype=torch.int64, device="cuda")]
    lccs = [torch.empty(n1, dtype=torch.float64, device="cuda"), torch.empty(n2, dtype=torch.float64, device="cuda")]
    tk = ctx.batch_submit([g1, g2], tris, lccs)
    assert ctx.batch_poll(tk, block=True)[0]
    num_ref, lcc_ref = oracle.tc_lcc_directed(n1, s1, d1)
    np.testing.assert_array_equal(tris[0].cpu().numpy().astype(np.uint64), num_ref)
    assert lccs[0].cpu().numpy().tobytes() == lcc_ref.tobytes()
    t_ref, l_ref = oracle.tc_lcc(n2, s2, d2)
    np.testing.assert_array_equal(tris[1].cpu().numpy().astype(np.uint64), t_ref)
    assert lccs[1].cpu().numpy().tobytes() == l_ref.tobytes()
    g1.free()
    g2.free()
    with pytest.raises(pkg.TcLccError) as e:
        g = ctx.build_directed(n1, dev(s1), dev(d1))
        try:
            g.run_edges()
        finally:
            g.free()
    assert e.value.status == pkg.UNSUPPORTED
