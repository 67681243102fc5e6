"""Seeded synthetic inputs shaped like the paper's workloads (input generation only).

The graphs follow the experimental setup of Strausz et al. (Sec. IV-A and
Table II): R-MAT with a=0.57, b=c=0.19, d=0.05 and EF * 2^scale generated
pairs, plus uniform (Erdos-Renyi) pairs.  Raw pairs may repeat, be self-loops
or appear in one direction only; that cleanup belongs to the consumer.

Nothing here computes triangles, degrees or clustering coefficients: both the
oracle and the GPU path take their inputs from this module and nothing else.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_GPU_SRC = os.path.join(_HERE, "synth_gpu.hip")
_GPU_LIB = os.path.join(_HERE, "libsynth_gpu.so")
_lib = None
_gpu_lib = None

RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (OpenMP for the parallel draws), and its GPU twin
    for the large-scale recipe with hipcc (gfx950)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    if force or not os.path.exists(_GPU_LIB) or os.path.getmtime(_GPU_LIB) < os.path.getmtime(_GPU_SRC):
        tmp = _GPU_LIB + ".tmp"
        subprocess.check_call(["/opt/rocm/bin/hipcc", "-O3", "-fPIC", "-shared", "--offload-arch=gfx950",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-o", tmp, _GPU_SRC], stderr=subprocess.DEVNULL)
        os.replace(tmp, _GPU_LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, u64, f64 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        p32 = ctypes.POINTER(ctypes.c_int32)
        lib.synth_rmat.argtypes = [i64, i64, f64, f64, f64, u64, p32, p32]
        lib.synth_rmat.restype = ctypes.c_int
        lib.synth_er.argtypes = [i64, i64, u64, p32, p32]
        lib.synth_er.restype = ctypes.c_int
        lib.synth_permutation.argtypes = [i64, u64, p32]
        lib.synth_permutation.restype = None
        lib.synth_splitmix64_at.argtypes = [u64, u64]
        lib.synth_splitmix64_at.restype = u64
        lib.synth_splitmix64_fill.argtypes = [u64, u64, i64, ctypes.c_void_p]
        lib.synth_splitmix64_fill.restype = None
        lib.synth_rmat_feistel.argtypes = [ctypes.c_int, f64, f64, f64, u64, u64, i64, p32, p32]
        lib.synth_rmat_feistel.restype = ctypes.c_int
        lib.synth_rmat_stream.argtypes = [u64]
        lib.synth_rmat_stream.restype = u64
        lib.synth_feistel_keys.argtypes = [u64, ctypes.c_void_p]
        lib.synth_feistel_keys.restype = None
        lib.synth_rmat_thresholds.argtypes = [f64, f64, f64, ctypes.c_void_p]
        lib.synth_rmat_thresholds.restype = None
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def splitmix64_at(state: int, k: int) -> int:
    """k-th output of SplitMix64 started from `state` (exposed for its known-answer test)."""
    return int(_load().synth_splitmix64_at(state & (2**64 - 1), k))


def splitmix64_fill(state: int, k0: int, count: int) -> np.ndarray:
    """Outputs k0 .. k0 + count - 1 of SplitMix64 started from `state`."""
    out = np.empty(count, dtype=np.uint64)
    _load().synth_splitmix64_fill(state & (2**64 - 1), k0, count, out.ctypes.data)
    return out


def permutation(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _load().synth_permutation(n, seed, _p32(out))
    return out


def rmat(n: int, m_gen: int, seed: int, abc=RMAT_ABC):
    """R-MAT pairs over [0, n); ceil(log2 n) levels, rejection when n is not a power of two."""
    src = np.empty(m_gen, dtype=np.int32)
    dst = np.empty(m_gen, dtype=np.int32)
    rc = _load().synth_rmat(n, m_gen, abc[0], abc[1], abc[2], seed, _p32(src), _p32(dst))
    if rc != 0:
        raise ValueError(f"synth_rmat failed ({rc}) for n={n} m_gen={m_gen}")
    return src, dst


def er(n: int, m_gen: int, seed: int):
    """m_gen uniform ordered pairs over [0, n)."""
    src = np.empty(m_gen, dtype=np.int32)
    dst = np.empty(m_gen, dtype=np.int32)
    rc = _load().synth_er(n, m_gen, seed, _p32(src), _p32(dst))
    if rc != 0:
        raise ValueError(f"synth_er failed ({rc})")
    return src, dst


# ---- the workload recipes -------------------------------------------------------

def er_4096(seed: int = 1):
    """Uniform random graph, n = 4096, average degree 16: n*16/2 = 32768 raw pairs."""
    n = 4096
    s, d = er(n, n * 16 // 2, seed)
    return n, s, d


def rmat_scale(scale: int, edge_factor: int = 16, seed: int = 1):
    """R-MAT at 2^scale vertices with EF * 2^scale raw pairs (Table II's |E| column)."""
    n = 1 << scale
    s, d = rmat(n, edge_factor * n, seed)
    return n, s, d


def batch_specs(count: int = 4096, seed: int = 7):
    """Specs of the many-small-graphs batch.

    n_i = round(exp(U[ln 64, ln 16384])).  Even i: uniform pairs with average degree
    U[8, 32] (n_i * deg / 2 raw pairs).  Odd i: R-MAT with edge factor U{8..16}
    (EF * n_i raw pairs).  Graph i uses generator seed 1000 + i.
    """
    st = sub_seed_py(seed)
    specs = []
    for i in range(count):
        u0 = _unit(splitmix64_at(st, 3 * i))
        u1 = _unit(splitmix64_at(st, 3 * i + 1))
        n = int(round(math.exp(math.log(64) + u0 * (math.log(16384) - math.log(64)))))
        if i % 2 == 0:
            deg = 8.0 + 24.0 * u1
            specs.append(("er", n, int(round(n * deg / 2)), 1000 + i))
        else:
            ef = 8 + int(u1 * 9)
            specs.append(("rmat", n, ef * n, 1000 + i))
    return specs


def serving_specs(count: int = 64, seed: int = 9, lo_scale: int = 10, hi_scale: int = 21,
                  edge_factor: int = 16):
    """Pool of R-MAT graphs with n log-uniform in [2^lo, 2^hi]; graph i uses seed 5000 + i."""
    st = sub_seed_py(seed)
    specs = []
    for i in range(count):
        u0 = _unit(splitmix64_at(st, i))
        n = int(round(2.0 ** (lo_scale + u0 * (hi_scale - lo_scale))))
        specs.append(("rmat", n, edge_factor * n, 5000 + i))
    return specs


def dense_core(parts: int, size: int, drop: float, periphery_scale: int, seed: int):
    """A dense graph that is not a clique, with a sparse periphery.

    Core: vertices [0, parts * size) in `parts` parts of `size`; every pair in different parts
    is joined except a fraction `drop` of them (pair i of the row-major upper triangle is
    dropped when output i of the seed's stream falls below drop * 2^64).  Periphery: R-MAT
    pairs (edge factor 8) over the next 2^periphery_scale ids, each periphery vertex p also
    joined to core vertices 7 p and 13 p + 1 (mod the core size).  Returns (n, src, dst).
    """
    nc = parts * size
    iu, ju = np.triu_indices(nc, 1)
    keep = (iu // size) != (ju // size)
    if drop > 0:
        r = splitmix64_fill(sub_seed_py(seed), 0, len(iu))
        keep &= r >= np.uint64(int(drop * 2.0**64))
    cs, cd = iu[keep].astype(np.int32), ju[keep].astype(np.int32)
    npp = 1 << periphery_scale if periphery_scale > 0 else 0
    parts_s, parts_d = [cs], [cd]
    if npp:
        ps, pd = rmat(npp, 8 * npp, seed + 1)
        p = np.arange(npp, dtype=np.int64)
        parts_s += [ps + nc, (p + nc).astype(np.int32), (p + nc).astype(np.int32)]
        parts_d += [pd + nc, ((7 * p) % nc).astype(np.int32), ((13 * p + 1) % nc).astype(np.int32)]
    return nc + npp, np.concatenate(parts_s).astype(np.int32), np.concatenate(parts_d).astype(np.int32)


def rmat_feistel(scale: int, first: int, count: int, seed: int = 1, abc=RMAT_ABC):
    """Pairs first .. first + count - 1 of the large-scale R-MAT recipe (synth_rmat_feistel):
    n = 2^scale (scale even), pair e = R-MAT attempt e, ends relabelled by a seeded Feistel
    bijection.  The workload of scale s and edge factor EF is pairs 0 .. EF * 2^s - 1."""
    src = np.empty(count, dtype=np.int32)
    dst = np.empty(count, dtype=np.int32)
    rc = _load().synth_rmat_feistel(scale, abc[0], abc[1], abc[2], seed, first, count, _p32(src), _p32(dst))
    if rc != 0:
        raise ValueError(f"synth_rmat_feistel failed ({rc}) for scale {scale}")
    return src, dst


def _gpu():
    global _gpu_lib
    if _gpu_lib is None:
        if not os.path.exists(_GPU_LIB):
            build(force=False)
        lib = ctypes.CDLL(_GPU_LIB)
        vp, u64, i64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64
        lib.synth_gpu_rmat_feistel.argtypes = [ctypes.c_int, u64, vp, vp, u64, i64, vp, vp, vp]
        lib.synth_gpu_rmat_feistel.restype = ctypes.c_int
        lib.synth_gpu_copy_i32.argtypes = [vp, vp, i64, vp]
        lib.synth_gpu_copy_i32.restype = ctypes.c_int
        _gpu_lib = lib
    return _gpu_lib


class GpuRmatFeistel:
    """The same recipe written by the GPU into device memory: gen(first, count, src_ptr,
    dst_ptr, stream_ptr) fills int32 device arrays (plain integer addresses)."""

    def __init__(self, scale: int, seed: int = 1, abc=RMAT_ABC):
        self.scale = scale
        self.state = int(_load().synth_rmat_stream(seed))
        self.thr = np.empty(3, dtype=np.uint64)
        _load().synth_rmat_thresholds(abc[0], abc[1], abc[2], self.thr.ctypes.data)
        self.keys = np.empty(4, dtype=np.uint64)
        _load().synth_feistel_keys(seed, self.keys.ctypes.data)

    def gen(self, first: int, count: int, src_ptr: int, dst_ptr: int, stream_ptr: int = 0):
        rc = _gpu().synth_gpu_rmat_feistel(self.scale, self.state, self.thr.ctypes.data, self.keys.ctypes.data,
                                           first, count, src_ptr, dst_ptr, stream_ptr)
        if rc != 0:
            raise RuntimeError(f"synth_gpu_rmat_feistel failed ({rc})")


class DevicePairs:
    """Stored pairs in device memory (two int32 torch CUDA tensors) served in chunks:
    gen(first, count, src_ptr, dst_ptr, stream_ptr) copies pairs [first, first + count)."""

    def __init__(self, src, dst):
        assert src.dtype == dst.dtype and src.element_size() == 4 and src.numel() == dst.numel()
        self.src, self.dst = src, dst

    def gen(self, first: int, count: int, src_ptr: int, dst_ptr: int, stream_ptr: int = 0):
        if first < 0 or first + count > self.src.numel():
            raise IndexError(f"pairs [{first}, {first + count}) outside [0, {self.src.numel()})")
        for a, b in ((self.src, src_ptr), (self.dst, dst_ptr)):
            rc = _gpu().synth_gpu_copy_i32(a.data_ptr() + 4 * first, b, count, stream_ptr)
            if rc != 0:
                raise RuntimeError(f"synth_gpu_copy_i32 failed ({rc})")


def make(spec):
    """Raw pairs for one spec tuple (kind, n, m_gen, seed) -> (n, src, dst)."""
    kind, n, m_gen, sd = spec
    if kind == "er":
        s, d = er(n, m_gen, sd)
    else:
        s, d = rmat(n, m_gen, sd)
    return n, s, d


def poisson_gaps(count: int, rate: float, seed: int = 11) -> np.ndarray:
    """Exponential inter-arrival gaps (seconds) for a Poisson process of `rate` per second."""
    st = sub_seed_py(seed)
    u = np.array([_unit(splitmix64_at(st, k)) for k in range(count)])
    return -np.log1p(-u) / rate


def choices(count: int, bound: int, seed: int) -> np.ndarray:
    st = sub_seed_py(seed)
    return np.array([(splitmix64_at(st, k) * bound) >> 64 for k in range(count)], dtype=np.int64)


def sub_seed_py(seed: int) -> int:
    """A stream state for the spec lists (SplitMix64 output 0 of `seed`)."""
    return splitmix64_at(seed, 0)


def _unit(r: int) -> float:
    return (r >> 11) * (1.0 / (1 << 53))
