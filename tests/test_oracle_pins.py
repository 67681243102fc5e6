"""Pins for the CPU oracle: each check comes from outside the oracle's own code.

Brute force written here in plain Python, closed forms, dense and sparse linear
algebra (t = rowsum((A A) o A) / 2, the algebraic form of Sec. V-B), networkx,
and exact rationals for the LCC bits (Eq. 2).  A dropped term, a wrong index or
a transposed operand anywhere in the oracle fails at least one of them.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
import synth


# --------------------------------------------------------------------------- helpers

def py_reference(n, pairs):
    """Triangles and LCC of the simple graph behind `pairs`, by triple enumeration."""
    adj = [set() for _ in range(n)]
    for u, v in pairs:
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    t = [0] * n
    for i, j, k in itertools.combinations(range(n), 3):
        if j in adj[i] and k in adj[i] and k in adj[j]:
            t[i] += 1
            t[j] += 1
            t[k] += 1
    deg = [len(a) for a in adj]
    lcc = [float(Fraction(2 * t[v], deg[v] * (deg[v] - 1))) if deg[v] >= 2 else 0.0
           for v in range(n)]
    return np.array(t, dtype=np.uint64), np.array(lcc), np.array(deg)


def oracle_all(n, pairs):
    """(t from every oracle method, lcc, csr) for one input."""
    src = np.array([p[0] for p in pairs], dtype=np.int32)
    dst = np.array([p[1] for p in pairs], dtype=np.int32)
    g = oracle.csr(n, src, dst)
    ts = {
        "forward": oracle.tc_forward(g),
        "edge_ssi": oracle.tc_edge_centric(g, oracle.SSI),
        "edge_bs": oracle.tc_edge_centric(g, oracle.BS),
        "edge_hybrid": oracle.tc_edge_centric(g, oracle.HYBRID),
        "brute": oracle.tc_brute(g),
    }
    return ts, oracle.lcc(g, ts["forward"]), g


def assert_matches_reference(n, pairs):
    t_ref, lcc_ref, deg_ref = py_reference(n, pairs)
    ts, lcc, g = oracle_all(n, pairs)
    np.testing.assert_array_equal(g.deg, deg_ref)
    for name, t in ts.items():
        np.testing.assert_array_equal(t, t_ref, err_msg=name)
    assert lcc.tobytes() == lcc_ref.tobytes()


def edges_of(n, mask):
    pairs = list(itertools.combinations(range(n), 2))
    return [pairs[b] for b in range(len(pairs)) if mask >> b & 1]


# --------------------------------------------------------------------------- brute force

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exhaustive_small(n):
    for mask in range(1 << (n * (n - 1) // 2)):
        assert_matches_reference(n, edges_of(n, mask))


def test_exhaustive_n6():
    """All 2^15 labelled graphs on 6 vertices: every oracle method vs triple enumeration."""
    n = 6
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << 15):
        es = [pairs[b] for b in range(15) if mask >> b & 1]
        t_ref, lcc_ref, _ = py_reference(n, es)
        ts, lcc, _ = oracle_all(n, es)
        for name, t in ts.items():
            assert np.array_equal(t, t_ref), (mask, name)
        assert lcc.tobytes() == lcc_ref.tobytes(), mask


@settings(max_examples=150, deadline=None)
@given(st.integers(min_value=1, max_value=40).flatmap(
    lambda n: st.tuples(st.just(n), st.lists(
        st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=300))))
def test_random_multigraphs_with_loops(case):
    """Repeated pairs, self-loops and one-direction pairs all reduce to the simple graph."""
    n, pairs = case
    assert_matches_reference(n, pairs)


# --------------------------------------------------------------------------- closed forms

def run(n, pairs):
    ts, lcc, g = oracle_all(n, pairs)
    for name, t in ts.items():
        assert np.array_equal(t, ts["forward"]), name
    return ts["forward"], lcc, g


@pytest.mark.parametrize("n", [3, 4, 5, 8, 17, 40])
def test_complete_graph(n):
    t, lcc, _ = run(n, list(itertools.combinations(range(n), 2)))
    assert np.all(t == math.comb(n - 1, 2))
    assert int(t.sum()) == 3 * math.comb(n, 3)
    assert np.all(lcc == 1.0)


def test_triangle_free_families():
    fams = []
    fams.append((50, [(0, i) for i in range(1, 50)]))                       # star
    fams.append((64, [(i, (i - 1) // 2) for i in range(1, 64)]))             # binary tree
    fams.append((40, [(i, (i + 1) % 40) for i in range(40)]))                # even cycle
    fams.append((41, [(i, (i + 1) % 41) for i in range(41)]))                # odd cycle > 3
    grid = [(r * 7 + c, r * 7 + c + 1) for r in range(6) for c in range(6)]
    grid += [(r * 7 + c, (r + 1) * 7 + c) for r in range(5) for c in range(7)]
    fams.append((42, grid))                                                 # 6x7 grid
    fams.append((13, [(a, 5 + b) for a in range(5) for b in range(8)]))    # K_{5,8}
    cube = [(x, x ^ (1 << k)) for x in range(64) for k in range(6) if x < x ^ (1 << k)]
    fams.append((64, cube))                                                 # 6-cube
    for n, pairs in fams:
        t, lcc, _ = run(n, pairs)
        assert int(t.sum()) == 0
        assert np.all(lcc == 0.0)


def test_single_triangle():
    t, lcc, _ = run(3, [(0, 1), (1, 2), (2, 0)])
    assert t.tolist() == [1, 1, 1]
    assert lcc.tolist() == [1.0, 1.0, 1.0]


@pytest.mark.parametrize("rim", [4, 5, 6, 11, 30])
def test_wheel(rim):
    """Hub 0 joined to a cycle of `rim` vertices: n - 1 triangles, hub LCC 2/(n-2), rim 2/3."""
    n = rim + 1
    pairs = [(0, i) for i in range(1, n)] + [(i, i % rim + 1) for i in range(1, n)]
    t, lcc, _ = run(n, pairs)
    assert int(t.sum()) == 3 * (n - 1)
    assert int(t[0]) == n - 1
    assert np.all(t[1:] == 2)
    assert lcc[0] == float(Fraction(2, n - 2))
    assert np.all(lcc[1:] == float(Fraction(2, 3)))


@pytest.mark.parametrize("k", [1, 2, 5, 20])
def test_windmill(k):
    """k triangles sharing vertex 0: centre LCC 1/(2k-1), all others 1."""
    n = 2 * k + 1
    pairs = []
    for i in range(k):
        a, b = 2 * i + 1, 2 * i + 2
        pairs += [(0, a), (0, b), (a, b)]
    t, lcc, _ = run(n, pairs)
    assert int(t.sum()) == 3 * k
    assert int(t[0]) == k
    assert lcc[0] == float(Fraction(1, 2 * k - 1))
    assert np.all(lcc[1:] == 1.0)


@pytest.mark.parametrize("k,size", [(3, 1), (3, 4), (5, 3), (7, 6)])
def test_complete_multipartite(k, size):
    """k parts of `size` vertices, every pair in different parts joined: each vertex has
    d = (k-1) size and t = C(d, 2) - (k-1) C(size, 2) (neighbour pairs inside one other part
    are not joined); LCC = 2 t / (d (d - 1)).  Dense, yet most neighbour pairs of the same
    part miss, unlike K_n."""
    n = k * size
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n) if a // size != b // size]
    t, lcc, g = run(n, pairs)
    d = (k - 1) * size
    want = math.comb(d, 2) - (k - 1) * math.comb(size, 2)
    assert np.all(g.deg == d)
    assert np.all(t == want)
    assert np.all(lcc == (float(Fraction(2 * want, d * (d - 1))) if d >= 2 else 0.0))


def test_empty_and_isolated():
    t, lcc, g = run(5, [])
    assert t.tolist() == [0] * 5 and lcc.tolist() == [0.0] * 5 and g.m == 0
    t, lcc, g = run(1, [(0, 0), (0, 0)])
    assert t.tolist() == [0] and g.m == 0


# --------------------------------------------------------------------------- linear algebra and networkx

def dense_t(g):
    A = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), g.deg)
    A[rows, g.adj] = 1.0
    return ((A @ A) * A).sum(axis=1) / 2.0


def test_dense_algebraic_er4096():
    """The 4096-vertex uniform graph: every count equals rowsum((A A) o A) / 2 (exact in fp64)."""
    n, s, d = synth.er_4096(seed=1)
    g = oracle.csr(n, s, d)
    t = oracle.tc_forward(g)
    ref = dense_t(g)
    np.testing.assert_array_equal(t.astype(np.float64), ref)
    np.testing.assert_array_equal(oracle.tc_edge_centric(g, oracle.HYBRID), t)


def test_sparse_algebraic_rmat14():
    import scipy.sparse as sp
    n, s, d = synth.rmat_scale(14, 16, seed=3)
    g = oracle.csr(n, s, d)
    A = sp.csr_matrix((np.ones(len(g.adj)), g.adj, g.off), shape=(n, n))
    ref = np.asarray((A @ A).multiply(A).sum(axis=1)).ravel() / 2
    t = oracle.tc_forward(g)
    np.testing.assert_array_equal(t.astype(np.float64), ref)
    for method in (oracle.SSI, oracle.BS, oracle.HYBRID):
        np.testing.assert_array_equal(oracle.tc_edge_centric(g, method), t)


def test_csr_matches_scipy():
    import scipy.sparse as sp
    n, s, d = synth.rmat_scale(12, 8, seed=5)
    g = oracle.csr(n, s, d)
    keep = s != d
    r = np.concatenate([s[keep], d[keep]])
    c = np.concatenate([d[keep], s[keep]])
    M = sp.coo_matrix((np.ones(len(r)), (r, c)), shape=(n, n)).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    np.testing.assert_array_equal(g.off, M.indptr)
    np.testing.assert_array_equal(g.adj, M.indices)


@pytest.mark.parametrize("which", ["er", "rmat"])
def test_networkx(which):
    import networkx as nx
    if which == "er":
        n, s, d = 3000, *synth.er(3000, 3000 * 10, seed=2)
    else:
        n, s, d = synth.rmat_scale(12, 16, seed=4)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from((int(a), int(b)) for a, b in zip(s, d) if a != b)
    # networkx's convention for degree < 2 is LCC 0, the reading used here
    assert nx.clustering(nx.path_graph(2))[0] == 0
    t, lcc = oracle.tc_lcc(n, s, d)
    tri = nx.triangles(G)
    clu = nx.clustering(G)
    np.testing.assert_array_equal(t, np.array([tri[v] for v in range(n)], dtype=np.uint64))
    np.testing.assert_allclose(lcc, np.array([clu[v] for v in range(n)]), rtol=1e-15, atol=0)


# --------------------------------------------------------------------------- invariants

def test_invariants_rmat():
    n, s, d = synth.rmat_scale(15, 16, seed=6)
    g = oracle.csr(n, s, d)
    t = oracle.tc_forward(g)
    lcc = oracle.lcc(g, t)
    assert int(t.sum()) % 3 == 0
    deg = g.deg.astype(np.uint64)
    assert np.all(t <= deg * (deg - 1) // 2)
    assert np.all((lcc >= 0.0) & (lcc <= 1.0))
    # LCC bits: exact rational, correctly rounded
    rng = np.random.default_rng(0)
    for v in rng.choice(n, 300, replace=False):
        dv = int(g.deg[v])
        want = float(Fraction(2 * int(t[v]), dv * (dv - 1))) if dv >= 2 else 0.0
        assert lcc[v] == want


def test_relabel_equivariance():
    n, s, d = synth.rmat_scale(11, 16, seed=8)
    t, lcc = oracle.tc_lcc(n, s, d)
    p = synth.permutation(n, 99)
    t2, lcc2 = oracle.tc_lcc(n, p[s], p[d])
    np.testing.assert_array_equal(t2[p], t)
    np.testing.assert_array_equal(lcc2[p], lcc)


def test_duplicates_loops_direction_ignored():
    n, s, d = synth.rmat_scale(10, 8, seed=10)
    t, lcc = oracle.tc_lcc(n, s, d)
    loops = np.arange(0, n, 7, dtype=np.int32)
    s2 = np.concatenate([d, s, s[:1000], loops])
    d2 = np.concatenate([s, d, d[:1000], loops])
    t2, lcc2 = oracle.tc_lcc(n, s2, d2)
    np.testing.assert_array_equal(t, t2)
    assert lcc.tobytes() == lcc2.tobytes()


def test_vertex_at_a_time_and_ranges():
    n, s, d = synth.rmat_scale(13, 16, seed=12)
    g = oracle.csr(n, s, d)
    t = oracle.tc_forward(g)
    vs = np.arange(0, n, 37)
    np.testing.assert_array_equal(oracle.tc_vertices(g, vs), t[vs])
    hub = int(np.argmax(g.deg))
    assert oracle.tc_vertices(g, [hub])[0] == t[hub]
    acc = np.zeros(n, dtype=np.uint64)
    edges = 0
    for a, b in [(0, 1000), (1000, 5000), (5000, n)]:
        part, e = oracle.tc_forward_range(g, a, b)
        acc += part
        edges += e
    np.testing.assert_array_equal(acc, t)
    assert edges == g.m


@settings(max_examples=150, deadline=None)
@given(st.integers(min_value=1, max_value=30).flatmap(
    lambda n: st.tuples(st.just(n), st.lists(
        st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=250))))
def test_vertex_from_raw_pairs_brute_force(case):
    """t(v) and d(v) straight from raw pairs (repeats, loops, one-direction pairs) equal the
    independent Python triple enumeration of the simple graph, for every vertex."""
    n, pairs = case
    t_ref, _, deg_ref = py_reference(n, pairs)
    s = np.array([a for a, _ in pairs], dtype=np.int32)
    d = np.array([b for _, b in pairs], dtype=np.int32)
    for v in range(n):
        assert oracle.tc_vertex_pairs(n, s, d, v) == (int(t_ref[v]), int(deg_ref[v])), v


def test_vertex_from_raw_pairs_rmat():
    """The same on an R-MAT graph against the pinned forward count and CSR degrees, on every
    41st vertex and the hub (the mark array must come back clean between calls)."""
    n, s, d = synth.rmat_scale(12, 16, seed=21)
    g = oracle.csr(n, s, d)
    t = oracle.tc_forward(g)
    vs = list(range(0, n, 41)) + [int(np.argmax(g.deg))]
    for v in vs:
        assert oracle.tc_vertex_pairs(n, s, d, v) == (int(t[v]), int(g.deg[v])), v


# --------------------------------------------------------------------------- intersection routines

sorted_lists = st.lists(st.integers(-50, 400), max_size=120).map(lambda x: sorted(set(x)))


@settings(max_examples=300, deadline=None)
@given(sorted_lists, sorted_lists)
def test_intersections_agree_with_sets(A, B):
    want = len(set(A) & set(B))
    assert oracle.ssi(A, B) == want
    assert oracle.bs(A, B) == want
    assert oracle.bs(B, A) == want
    assert oracle.hybrid(A, B) == want


def test_eq3_rule():
    # |B|/|A| <= log2|B| - 1 selects SSI; ties select SSI; order of arguments does not matter
    assert oracle.eq3_prefers_ssi(4, 8)          # 2 <= 2 (tie)
    assert not oracle.eq3_prefers_ssi(3, 8)      # 2.67 > 2
    assert oracle.eq3_prefers_ssi(16, 16)
    assert not oracle.eq3_prefers_ssi(1, 2)      # 2 > 0
    assert not oracle.eq3_prefers_ssi(1, 1)      # 1 > -1
    assert oracle.eq3_prefers_ssi(200, 1000)     # 5 <= 8.97
    assert not oracle.eq3_prefers_ssi(100, 1000) # 10 > 8.97
    assert not oracle.eq3_prefers_ssi(10, 1000)  # 100 > 8.97
    assert oracle.eq3_prefers_ssi(8, 4) == oracle.eq3_prefers_ssi(4, 8)


# --------------------------------------------------------------------------- per-edge counts (Sec. V-B)

def py_edge_counts(n, pairs):
    """Common neighbours of every edge {i < j}, by Python sets, in (i, j) order."""
    adj = [set() for _ in range(n)]
    for u, v in pairs:
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    out = []
    for i in range(n):
        for j in sorted(adj[i]):
            if j > i:
                out.append((i, j, len(adj[i] & adj[j])))
    return out


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 30).flatmap(lambda n: st.tuples(
    st.just(n), st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=150))))
def test_edge_counts_brute_force(case):
    n, pairs = case
    src = np.array([p[0] for p in pairs], dtype=np.int32)
    dst = np.array([p[1] for p in pairs], dtype=np.int32)
    g = oracle.csr(n, src, dst)
    eu, ev, c = oracle.edge_counts(g)
    want = py_edge_counts(n, pairs)
    assert list(zip(eu.tolist(), ev.tolist(), c.tolist())) == want


def test_edge_counts_scipy_and_invariants():
    """C = (A A) o A with scipy on R-MAT S13: the upper-triangle entries in CSR order; sum of
    c over the edges = 3 T; sum over the edges at i = 2 t(i)."""
    import scipy.sparse as sp
    n, s, d = synth.rmat_scale(13, 16, seed=17)
    g = oracle.csr(n, s, d)
    eu, ev, c = oracle.edge_counts(g)
    rows = np.repeat(np.arange(n), g.deg)
    A = sp.csr_matrix((np.ones(len(g.adj), dtype=np.int64), (rows, g.adj)), shape=(n, n))
    C = sp.triu((A @ A).multiply(A), k=1).tocsr()
    C.sort_indices()
    Ccoo = C.tocoo()
    # scipy drops the explicit zeros of edges without triangles: compare on the edge list
    dense_vals = dict(zip(zip(Ccoo.row.tolist(), Ccoo.col.tolist()), Ccoo.data.tolist()))
    want = np.array([dense_vals.get((a, b), 0) for a, b in zip(eu.tolist(), ev.tolist())], dtype=np.uint64)
    np.testing.assert_array_equal(c, want)
    t = oracle.tc_forward(g)
    assert int(c.sum()) == int(t.sum())  # sum over edges = 3 T = sum over vertices
    per_vertex = np.bincount(eu, weights=c, minlength=n) + np.bincount(ev, weights=c, minlength=n)
    np.testing.assert_array_equal(per_vertex.astype(np.uint64), 2 * t)


@pytest.mark.parametrize("n", [3, 4, 9, 30])
def test_edge_counts_complete_graph(n):
    s, d = (x.astype(np.int32) for x in np.triu_indices(n, 1))
    eu, ev, c = oracle.edge_counts(oracle.csr(n, s, d))
    assert len(c) == n * (n - 1) // 2 and np.all(c == n - 2)


# --------------------------------------------------------------------------- directed graphs (Eq. 1)

def py_directed(n, pairs):
    """Eq. 1 by enumeration: ordered pairs (j, k), j != k, with i -> j, i -> k and j -> k."""
    out = [set() for _ in range(n)]
    for u, v in pairs:
        if u != v:
            out[u].add(v)
    num = [0] * n
    for i in range(n):
        for j in out[i]:
            for k in out[i]:
                if j != k and k in out[j]:
                    num[i] += 1
    dout = [len(o) for o in out]
    lcc = [float(Fraction(num[i], dout[i] * (dout[i] - 1))) if dout[i] >= 2 else 0.0 for i in range(n)]
    return np.array(num, dtype=np.uint64), np.array(lcc), np.array(dout)


@settings(max_examples=80, deadline=None)
@given(st.integers(1, 25).flatmap(lambda n: st.tuples(
    st.just(n), st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=160))))
def test_directed_brute_force(case):
    n, pairs = case
    src = np.array([p[0] for p in pairs], dtype=np.int32)
    dst = np.array([p[1] for p in pairs], dtype=np.int32)
    num_ref, lcc_ref, dout_ref = py_directed(n, pairs)
    g = oracle.csr_directed(n, src, dst)
    np.testing.assert_array_equal(g.deg, dout_ref)
    num, lcc = oracle.tc_lcc_directed(n, src, dst)
    np.testing.assert_array_equal(num, num_ref)
    assert lcc.tobytes() == lcc_ref.tobytes()


def test_directed_dense_algebraic():
    """Numerator of Eq. 1 = rowsum((A A) o A) for the directed adjacency A (no halving):
    (A A)_ik counts the paths i -> j -> k, o A keeps those with i -> k."""
    rng = np.random.default_rng(5)
    n = 400
    A = (rng.random((n, n)) < 0.05).astype(np.float64)
    np.fill_diagonal(A, 0.0)
    src, dst = (x.astype(np.int32) for x in np.nonzero(A))
    num, _ = oracle.tc_lcc_directed(n, src, dst)
    np.testing.assert_array_equal(num, ((A @ A) * A).sum(axis=1).astype(np.uint64))


@pytest.mark.parametrize("n", [3, 5, 12])
def test_directed_closed_forms(n):
    # complete digraph (both directions): num = d (d - 1), C = 1
    pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
    src = np.array([p[0] for p in pairs], dtype=np.int32)
    dst = np.array([p[1] for p in pairs], dtype=np.int32)
    num, lcc = oracle.tc_lcc_directed(n, src, dst)
    assert np.all(num == (n - 1) * (n - 2)) and np.all(lcc == 1.0)
    # transitive tournament (a -> b iff a < b): out(i) = {i+1 .. n-1}, num = C(n-1-i, 2), C = 1/2
    s, d = (x.astype(np.int32) for x in np.triu_indices(n, 1))
    num, lcc = oracle.tc_lcc_directed(n, s, d)
    dout = n - 1 - np.arange(n)
    assert num.tolist() == [math.comb(int(k), 2) for k in dout]
    assert np.all(lcc[dout >= 2] == 0.5) and np.all(lcc[dout < 2] == 0.0)
    # directed cycle: one out-neighbour each, no numerator
    cyc = np.arange(n, dtype=np.int32)
    num, lcc = oracle.tc_lcc_directed(n, cyc, np.roll(cyc, -1))
    assert np.all(num == 0) and np.all(lcc == 0.0)


def test_directed_symmetric_input_is_undirected():
    """Both directions of every edge: num = 2 t(v) and Eq. 1 gives Eq. 2's bits."""
    n, s, d = synth.rmat_scale(11, 16, seed=9)
    t, lcc_u = oracle.tc_lcc(n, s, d)
    num, lcc_d = oracle.tc_lcc_directed(n, np.concatenate([s, d]), np.concatenate([d, s]))
    np.testing.assert_array_equal(num, 2 * t)
    assert lcc_d.tobytes() == lcc_u.tobytes()
