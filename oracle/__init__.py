"""CPU oracle for per-vertex triangle counts and LCC (Python side of oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library, and it shares no code
with it.  Every routine follows its definition in Strausz et al. (Sec. II-C,
Eq. 1, Eq. 2, Alg. 1-3, and the per-edge counts of Sec. V-B); see oracle.c for the
readings of the paper it takes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

SSI, BS, HYBRID = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile oracle.c (plain C, no fast-math: the LCC division must be IEEE)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, u64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32
        vp = ctypes.c_void_p
        lib.oracle_csr.argtypes = [i64, i64, vp, vp, vp, vp]
        lib.oracle_csr.restype = i64
        for name in ("oracle_ssi", "oracle_bs", "oracle_hybrid"):
            getattr(lib, name).argtypes = [vp, i64, vp, i64]
            getattr(lib, name).restype = u64
        lib.oracle_eq3_prefers_ssi.argtypes = [i64, i64]
        lib.oracle_eq3_prefers_ssi.restype = ctypes.c_int
        lib.oracle_tc_edge_centric.argtypes = [i64, vp, vp, ctypes.c_int, vp]
        lib.oracle_tc_edge_centric.restype = None
        lib.oracle_tc_forward.argtypes = [i64, vp, vp, vp]
        lib.oracle_tc_forward.restype = None
        lib.oracle_tc_forward_range.argtypes = [i64, vp, vp, i64, i64, vp]
        lib.oracle_tc_forward_range.restype = i64
        lib.oracle_tc_brute.argtypes = [i64, vp, vp, vp]
        lib.oracle_tc_brute.restype = None
        lib.oracle_tc_vertex.argtypes = [vp, vp, i32, vp]
        lib.oracle_tc_vertex.restype = u64
        lib.oracle_tc_vertex_pairs.argtypes = [i64, vp, vp, i32, vp, vp]
        lib.oracle_tc_vertex_pairs.restype = u64
        lib.oracle_lcc_one.argtypes = [u64, i64]
        lib.oracle_lcc_one.restype = ctypes.c_double
        lib.oracle_lcc.argtypes = [i64, vp, vp, vp]
        lib.oracle_lcc.restype = None
        lib.oracle_edge_counts.argtypes = [i64, vp, vp, vp, vp, vp]
        lib.oracle_edge_counts.restype = i64
        lib.oracle_csr_directed.argtypes = [i64, i64, vp, vp, vp, vp]
        lib.oracle_csr_directed.restype = i64
        lib.oracle_tc_directed.argtypes = [i64, vp, vp, vp]
        lib.oracle_tc_directed.restype = None
        lib.oracle_lcc_directed_one.argtypes = [u64, i64]
        lib.oracle_lcc_directed_one.restype = ctypes.c_double
        lib.oracle_lcc_directed.argtypes = [i64, vp, vp, vp]
        lib.oracle_lcc_directed.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data


class CSR:
    """Sorted, deduplicated, loop-free undirected CSR (int64 offsets, int32 ids)."""

    def __init__(self, n: int, off: np.ndarray, adj: np.ndarray):
        self.n, self.off, self.adj = n, off, adj

    @property
    def deg(self) -> np.ndarray:
        return np.diff(self.off)

    @property
    def m(self) -> int:
        return int(self.off[-1]) // 2


def csr(n: int, src, dst) -> CSR:
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    assert src.shape == dst.shape
    off = np.empty(n + 1, dtype=np.int64)
    adj = np.empty(max(2 * len(src), 1), dtype=np.int32)
    nnz = _load().oracle_csr(n, len(src), _p(src), _p(dst), _p(off), _p(adj))
    if nnz < 0:
        raise ValueError("endpoint outside [0, n)")
    return CSR(n, off, adj[:nnz].copy())


def _arr32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def ssi(A, B) -> int:
    A, B = _arr32(A), _arr32(B)
    return int(_load().oracle_ssi(_p(A), len(A), _p(B), len(B)))


def bs(A, B) -> int:
    A, B = _arr32(A), _arr32(B)
    return int(_load().oracle_bs(_p(A), len(A), _p(B), len(B)))


def hybrid(A, B) -> int:
    A, B = _arr32(A), _arr32(B)
    return int(_load().oracle_hybrid(_p(A), len(A), _p(B), len(B)))


def eq3_prefers_ssi(na: int, nb: int) -> bool:
    return bool(_load().oracle_eq3_prefers_ssi(na, nb))


def tc_edge_centric(g: CSR, method: int = HYBRID) -> np.ndarray:
    t = np.empty(g.n, dtype=np.uint64)
    _load().oracle_tc_edge_centric(g.n, _p(g.off), _p(g.adj), method, _p(t))
    return t


def tc_forward(g: CSR) -> np.ndarray:
    t = np.empty(g.n, dtype=np.uint64)
    _load().oracle_tc_forward(g.n, _p(g.off), _p(g.adj), _p(t))
    return t


def tc_forward_range(g: CSR, u_begin: int, u_end: int):
    t = np.empty(g.n, dtype=np.uint64)
    edges = _load().oracle_tc_forward_range(g.n, _p(g.off), _p(g.adj), u_begin, u_end, _p(t))
    return t, int(edges)


def tc_brute(g: CSR) -> np.ndarray:
    t = np.empty(g.n, dtype=np.uint64)
    _load().oracle_tc_brute(g.n, _p(g.off), _p(g.adj), _p(t))
    return t


def tc_vertices(g: CSR, vertices) -> np.ndarray:
    """t(v) for the listed vertices, one at a time (for graphs too big for tc_forward)."""
    mark = np.zeros(g.n, dtype=np.uint8)
    lib = _load()
    return np.array([lib.oracle_tc_vertex(_p(g.off), _p(g.adj), int(v), _p(mark)) for v in vertices],
                    dtype=np.uint64)


def tc_vertex_pairs(n: int, src, dst, v: int):
    """(t(v), d(v)) straight from the raw pairs, without a CSR (for sampled checks on graphs
    whose CSR is too large to build on the host)."""
    s, d = _arr32(src), _arr32(dst)
    mark = np.zeros(n, dtype=np.uint8)
    deg = np.zeros(1, dtype=np.int64)
    t = _load().oracle_tc_vertex_pairs(len(s), _p(s), _p(d), int(v), _p(mark), _p(deg))
    return int(t), int(deg[0])


def lcc_one(t: int, d: int) -> float:
    return float(_load().oracle_lcc_one(t, d))


def lcc(g: CSR, t: np.ndarray) -> np.ndarray:
    t = np.ascontiguousarray(t, dtype=np.uint64)
    out = np.empty(g.n, dtype=np.float64)
    _load().oracle_lcc(g.n, _p(g.off), _p(t), _p(out))
    return out


def edge_counts(g: CSR):
    """Per-edge triangle counts (Sec. V-B, C = A A o A): (eu, ev, c) over the edges {eu < ev}
    in upper-triangle CSR order, c = |adj(eu) ∩ adj(ev)|."""
    m = g.m
    eu = np.empty(max(m, 1), dtype=np.int32)
    ev = np.empty(max(m, 1), dtype=np.int32)
    c = np.empty(max(m, 1), dtype=np.uint64)
    k = _load().oracle_edge_counts(g.n, _p(g.off), _p(g.adj), _p(eu), _p(ev), _p(c))
    assert k == m
    return eu[:m], ev[:m], c[:m]


def csr_directed(n: int, src, dst) -> CSR:
    """Out-list CSR of the directed graph behind the pairs (loops and repeats removed)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    off = np.empty(n + 1, dtype=np.int64)
    adj = np.empty(max(len(src), 1), dtype=np.int32)
    nnz = _load().oracle_csr_directed(n, len(src), _p(src), _p(dst), _p(off), _p(adj))
    if nnz < 0:
        raise ValueError("endpoint outside [0, n)")
    return CSR(n, off, adj[:nnz].copy())


def tc_directed(g: CSR) -> np.ndarray:
    """Numerator of Eq. 1 per vertex: edges e_jk with v_j, v_k out-neighbours of v_i."""
    num = np.empty(g.n, dtype=np.uint64)
    _load().oracle_tc_directed(g.n, _p(g.off), _p(g.adj), _p(num))
    return num


def lcc_directed_one(num: int, dout: int) -> float:
    return float(_load().oracle_lcc_directed_one(num, dout))


def lcc_directed(g: CSR, num: np.ndarray) -> np.ndarray:
    num = np.ascontiguousarray(num, dtype=np.uint64)
    out = np.empty(g.n, dtype=np.float64)
    _load().oracle_lcc_directed(g.n, _p(g.off), _p(num), _p(out))
    return out


def tc_lcc_directed(n: int, src, dst):
    """Per-vertex (numerator of Eq. 1, directed LCC of Eq. 1) of the raw directed pairs."""
    g = csr_directed(n, src, dst)
    num = tc_directed(g)
    return num, lcc_directed(g, num)


def tc_lcc(n: int, src, dst, method: str = "forward"):
    """Per-vertex (t, lcc) of the raw pairs; method 'forward', 'edge', or 'brute'."""
    g = csr(n, src, dst)
    if method == "forward":
        t = tc_forward(g)
    elif method == "edge":
        t = tc_edge_centric(g)
    elif method == "brute":
        t = tc_brute(g)
    else:
        raise ValueError(method)
    return t, lcc(g, t)
