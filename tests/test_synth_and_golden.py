"""Input generators (known answers, shapes of the paper's workloads) and stored oracle fixtures."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_splitmix64_known_answers():
    # published first outputs of SplitMix64 (Steele, Lea, Flood 2014; Vigna's reference splitmix64.c)
    assert synth.splitmix64_at(0, 0) == 0xE220A8397B1DCDAF
    assert synth.splitmix64_at(1234567, 0) == 6457827717110365317


def test_permutation_is_bijection_and_seeded():
    p = synth.permutation(100003, 5)
    assert np.array_equal(np.sort(p), np.arange(100003))
    assert np.array_equal(p, synth.permutation(100003, 5))
    assert not np.array_equal(p, synth.permutation(100003, 6))


def test_rmat_quadrant_probabilities():
    # with one level, the pair is the quadrant itself: frequencies a, b, c, d (before the permutation,
    # which on two vertices is either identity or swap, so only the diagonal/off-diagonal split is visible)
    s, d = synth.rmat(2, 400000, seed=3)
    diag = np.mean(s == d)
    assert abs(diag - (0.57 + 0.05)) < 0.005


def test_rmat_shape_table2_s21():
    """Table II: R-MAT S21 EF16 has 2.1 M vertices, 33.6 M edges and a 251.1 MiB CSR after
    degree-1 removal (int64 offsets, int32 ids).  The generator's graph lands within 3 %."""
    n, s, d = synth.rmat_scale(21, 16, seed=1)
    assert len(s) == 16 * 2 ** 21
    g = oracle.csr(n, s, d)
    keep = g.deg >= 2
    # removing degree<2 vertices drops their edges too; count entries among kept vertices
    rows = np.repeat(np.arange(n), g.deg)
    kept_entries = np.count_nonzero(keep[rows] & keep[g.adj])
    mib = (8 * (int(keep.sum()) + 1) + 4 * kept_entries) / 2 ** 20
    assert abs(mib - 251.1) / 251.1 < 0.03, mib


def test_non_power_of_two_rmat_in_range():
    s, d = synth.rmat(1000, 16000, seed=4)
    assert s.min() >= 0 and d.min() >= 0 and s.max() < 1000 and d.max() < 1000


def test_rmat_feistel_is_the_rmat_graph_relabelled():
    """The large-scale recipe draws the same R-MAT attempts as synth.rmat at a power of two and
    only relabels them, by a bijection: ids map one to one between the two, pair for pair."""
    scale = 12
    n, s0, d0 = synth.rmat_scale(scale, 16, seed=5)
    s1, d1 = synth.rmat_feistel(scale, 0, 16 * n, seed=5)
    a = np.concatenate([s0, d0]).astype(np.int64)
    b = np.concatenate([s1, d1]).astype(np.int64)
    assert b.min() >= 0 and b.max() < n
    fwd = np.full(n, -1, dtype=np.int64)
    fwd[a] = b
    assert np.array_equal(fwd[a], b), "one rmat id maps to two relabelled ids"
    used = fwd[fwd >= 0]
    assert len(np.unique(used)) == len(used), "two rmat ids map to one relabelled id"
    # any range of pairs on its own equals the same slice of the whole sequence
    s2, d2 = synth.rmat_feistel(scale, 1000, 5003, seed=5)
    assert np.array_equal(s2, s1[1000:6003]) and np.array_equal(d2, d1[1000:6003])
    assert not np.array_equal(synth.rmat_feistel(scale, 0, 64, seed=6)[0], s1[:64])
    with pytest.raises(ValueError):
        synth.rmat_feistel(13, 0, 10, seed=5)


def test_rmat_feistel_triangles_equal_rmat_triangles():
    """Relabelling changes no triangle count: the per-vertex counts agree through the id map."""
    scale = 10
    n, s0, d0 = synth.rmat_scale(scale, 16, seed=8)
    s1, d1 = synth.rmat_feistel(scale, 0, 16 * n, seed=8)
    t0, _ = oracle.tc_lcc(n, s0, d0)
    t1, _ = oracle.tc_lcc(n, s1, d1)
    fwd = np.arange(n)
    fwd[np.concatenate([s0, d0])] = np.concatenate([s1, d1])
    touched = np.zeros(n, dtype=bool)
    touched[np.concatenate([s0, d0])] = True
    assert np.array_equal(t1[fwd[touched]], t0[touched])
    assert t0.sum() == t1.sum()


def test_batch_specs_shape():
    specs = synth.batch_specs()
    assert len(specs) == 4096
    ns = np.array([x[1] for x in specs])
    assert ns.min() >= 64 and ns.max() <= 16384
    assert {x[0] for x in specs[0::2]} == {"er"} and {x[0] for x in specs[1::2]} == {"rmat"}
    for kind, n, m_gen, _ in specs[:200]:
        if kind == "er":
            assert 8 * n / 2 - 1 <= m_gen <= 32 * n / 2 + 1
        else:
            assert m_gen % n == 0 and 8 <= m_gen // n <= 16


@pytest.mark.parametrize("name", ["er4096_seed1", "rmat_s12_ef16_seed1", "rmat_s16_ef16_seed1"])
def test_golden_oracle_summaries(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        want = json.load(f)
    fn = {"er4096_seed1": lambda: synth.er_4096(seed=1),
          "rmat_s12_ef16_seed1": lambda: synth.rmat_scale(12, 16, seed=1),
          "rmat_s16_ef16_seed1": lambda: synth.rmat_scale(16, 16, seed=1)}[name]
    n, s, d = fn()
    g = oracle.csr(n, s, d)
    t = oracle.tc_forward(g)
    lcc = oracle.lcc(g, t)
    assert g.m == want["m_undirected"]
    assert int(t.sum()) // 3 == want["triangles"]
    assert hashlib.sha256(t.astype("<u8").tobytes()).hexdigest() == want["sha256_t_u64le"]
    assert hashlib.sha256(lcc.astype("<f8").tobytes()).hexdigest() == want["sha256_lcc_f64le"]
