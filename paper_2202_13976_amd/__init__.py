"""Python binding of the tc_lcc C-ABI (libtc_lcc.so): argument marshalling only.

Every step of the computation runs in the HIP library; this module passes
pointers, sizes and streams.  torch supplies device memory and streams.  If
the shared library is missing the import of the binding fails loudly: there is
no fallback path.

Entry points mirror include/tc_lcc.h:
    Context(device, budget)            tc_lcc_ctx_create / destroy
    Context.build_csr(n, src, dst)     tc_lcc_build_csr     -> Graph
    Graph.run(tri, lcc, stream)        tc_lcc_run
    Context.batch_submit / batch_poll  tc_lcc_batch_submit / poll
    Context.batch_progress             tc_lcc_batch_progress
    Context.autotune / load_tuning     tc_lcc_autotune / tc_lcc_tuning_load
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtc_lcc.so")

OK, INVALID_ARGUMENT, OUT_OF_MEMORY, OVER_BUDGET, NOT_READY, BUSY, DEVICE_ERROR, UNSUPPORTED = range(8)
PROBE_AUTO, PROBE_HASH, PROBE_SORTED, PROBE_BITMAP, PROBE_MERGE = range(5)


class TcLccError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class GraphStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("offset_bytes", ctypes.c_int32),
                ("max_out_degree", ctypes.c_int32), ("max_degree", ctypes.c_int64),
                ("wedges", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64),
                ("kept_in_edges", ctypes.c_int64), ("active_vertices", ctypes.c_int64),
                ("staged_entries", ctypes.c_int64), ("block_vertices", ctypes.c_int64),
                ("count_grid", ctypes.c_int32), ("count_lds_bytes", ctypes.c_int32),
                ("count_blocks_per_cu", ctypes.c_int32), ("table_slots", ctypes.c_int32),
                ("push_words", ctypes.c_uint64), ("global_vertices", ctypes.c_int64),
                ("directed", ctypes.c_int32), ("compact", ctypes.c_int32)]


class Timings(ctypes.Structure):
    _fields_ = [(name, ctypes.c_float) for name in (
        "build_sort_unique_ms", "build_rank_ms", "build_orient_ms", "build_reverse_ms", "build_schedule_ms",
        "run_zero_ms", "run_count_ms", "run_epilogue_ms")]

    def as_dict(self):
        return {name: float(getattr(self, name)) for name, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("probe", ctypes.c_int32), ("group", ctypes.c_int32), ("wave_work_max", ctypes.c_int64),
                ("wave_outdeg_max", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("merge_ratio_x100", ctypes.c_int32), ("batch_grab", ctypes.c_int32),
                ("batch_heavy_bits", ctypes.c_int32), ("row_sort_max", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class RequestInfo(ctypes.Structure):
    _fields_ = [("arrival_ns", ctypes.c_int64), ("admit_ns", ctypes.c_int64), ("done_ns", ctypes.c_int64),
                ("batch_size", ctypes.c_int32), ("status", ctypes.c_int32)]


_lib = None
EXPORTS = [
    "tc_lcc_ctx_create", "tc_lcc_ctx_destroy", "tc_lcc_ctx_memory", "tc_lcc_debug_fail_alloc", "tc_lcc_build_csr",
    "tc_lcc_build_directed", "tc_lcc_build_streamed", "tc_lcc_run_edges", "tc_lcc_run_edges_noalloc", "tc_lcc_graph_info",
    "tc_lcc_graph_export", "tc_lcc_graph_free", "tc_lcc_run", "tc_lcc_batch_submit", "tc_lcc_batch_poll",
    "tc_lcc_batch_progress", "tc_lcc_autotune", "tc_lcc_tuning_load",
    "tc_lcc_get_tuning", "tc_lcc_set_tuning", "tc_lcc_set_profiling", "tc_lcc_graph_timings",
    "tc_lcc_server_create", "tc_lcc_server_submit", "tc_lcc_server_poll", "tc_lcc_server_destroy",
    "tc_lcc_hbm_copy", "tc_lcc_status_string", "tc_lcc_last_error",
]


# tc_lcc_pair_source: (user, first, count, src, dst, hip_stream) -> 0 on success
PAIR_SOURCE = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p)


def lib():
    """Load libtc_lcc.so (built in-tree by build.py); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
    st = ctypes.c_int
    L.tc_lcc_ctx_create.argtypes = [i32, u64, ctypes.POINTER(vp)]
    L.tc_lcc_ctx_destroy.argtypes = [vp]
    L.tc_lcc_ctx_memory.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]
    L.tc_lcc_debug_fail_alloc.argtypes = [vp, i64]
    L.tc_lcc_build_csr.argtypes = [vp, i64, i64, vp, vp, i32, i32, vp, ctypes.POINTER(vp)]
    L.tc_lcc_build_directed.argtypes = [vp, i64, i64, vp, vp, i32, i32, vp, ctypes.POINTER(vp)]
    L.tc_lcc_build_streamed.argtypes = [vp, i64, u64, PAIR_SOURCE, vp, u64, u64, vp, ctypes.POINTER(vp)]
    L.tc_lcc_run_edges.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.tc_lcc_run_edges_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.tc_lcc_graph_info.argtypes = [vp, ctypes.POINTER(GraphStats)]
    L.tc_lcc_graph_export.argtypes = [vp, vp, vp, vp, vp]
    L.tc_lcc_graph_free.argtypes = [vp]
    L.tc_lcc_run.argtypes = [vp, vp, vp, vp]
    L.tc_lcc_batch_submit.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(u64)]
    L.tc_lcc_batch_poll.argtypes = [vp, u64, i32, ctypes.POINTER(i32)]
    L.tc_lcc_batch_progress.argtypes = [vp, u64, i32, ctypes.POINTER(ctypes.c_uint8)]
    L.tc_lcc_autotune.argtypes = [vp, i32, vp, i32, i32, ctypes.c_char_p, ctypes.POINTER(Tuning)]
    L.tc_lcc_tuning_load.argtypes = [vp, ctypes.c_char_p]
    L.tc_lcc_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.tc_lcc_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.tc_lcc_set_profiling.argtypes = [vp, i32]
    L.tc_lcc_graph_timings.argtypes = [vp, ctypes.POINTER(Timings)]
    L.tc_lcc_server_create.argtypes = [vp, u64, i32, i32, ctypes.POINTER(vp)]
    L.tc_lcc_server_submit.argtypes = [vp, vp, vp, vp, ctypes.POINTER(u64)]
    L.tc_lcc_server_poll.argtypes = [vp, u64, i32, ctypes.POINTER(RequestInfo)]
    L.tc_lcc_server_destroy.argtypes = [vp]
    L.tc_lcc_hbm_copy.argtypes = [vp, vp, u64, vp]
    for name in EXPORTS[:-2]:
        getattr(L, name).restype = st
    L.tc_lcc_status_string.argtypes = [st]
    L.tc_lcc_status_string.restype = ctypes.c_char_p
    L.tc_lcc_last_error.argtypes = []
    L.tc_lcc_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int, where: str):
    if status != OK:
        detail = lib().tc_lcc_last_error().decode(errors="replace")
        raise TcLccError(status, where, detail)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Graph:
    """Immutable device-resident graph (tc_lcc_graph)."""

    def __init__(self, ctx: "Context", handle: ctypes.c_void_p):
        self.ctx = ctx
        self.handle = handle

    def info(self) -> GraphStats:
        s = GraphStats()
        _check(lib().tc_lcc_graph_info(self.handle, ctypes.byref(s)), "tc_lcc_graph_info")
        return s

    @property
    def n(self) -> int:
        return int(self.info().n)

    def run(self, tri=None, lcc=None, stream=None, want_lcc: bool = True):
        """Launch the count + LCC on `stream`; returns (tri, lcc) device tensors (async)."""
        import torch
        n = self.n
        dev = torch.device("cuda", self.ctx.device)
        if tri is None:
            tri = torch.empty(n, dtype=torch.int64, device=dev)
        if lcc is None and want_lcc:
            lcc = torch.empty(n, dtype=torch.float64, device=dev)
        assert tri.is_cuda and tri.numel() >= n and tri.element_size() == 8 and tri.is_contiguous()
        if lcc is not None:
            assert lcc.is_cuda and lcc.numel() >= n and lcc.dtype == torch.float64 and lcc.is_contiguous()
        _check(lib().tc_lcc_run(self.handle, _dptr(tri), _dptr(lcc), _stream_ptr(stream)), "tc_lcc_run")
        return tri, lcc

    def run_edges(self, tri=None, lcc=None, stream=None, want_lcc: bool = True):
        """Per-vertex results plus per-edge triangle counts (tc_lcc_run_edges, synchronous):
        returns (tri, lcc, edge_src, edge_dst, edge_tri) device tensors, edges {src < dst} in
        ascending (src, dst) order, edge_tri as int32 holding the uint32 counts."""
        import torch
        s = self.info()
        n, m = int(s.n), int(s.m)
        dev = torch.device("cuda", self.ctx.device)
        if tri is None:
            tri = torch.empty(n, dtype=torch.int64, device=dev)
        if lcc is None and want_lcc:
            lcc = torch.empty(n, dtype=torch.float64, device=dev)
        es = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
        ed = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
        ec = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
        _check(lib().tc_lcc_run_edges(self.handle, _dptr(tri), _dptr(lcc), _dptr(es), _dptr(ed), _dptr(ec),
                                      _stream_ptr(stream)), "tc_lcc_run_edges")
        return tri, lcc, es[:m], ed[:m], ec[:m]

    def export(self):
        """(degree[n], order[n], out_off[n+1], out_adj[m]) on the host, for checking the builder."""
        s = self.info()
        n, m = int(s.n), int(s.m)
        deg = np.empty(n, dtype=np.int64)
        order = np.empty(n, dtype=np.int32)
        off = np.empty(n + 1, dtype=np.int64)
        adj = np.empty(max(m, 1), dtype=np.int32)
        _check(lib().tc_lcc_graph_export(self.handle, deg.ctypes.data, order.ctypes.data, off.ctypes.data,
                                         adj.ctypes.data), "tc_lcc_graph_export")
        return deg, order, off, adj[:m]

    def timings(self) -> Timings:
        t = Timings()
        _check(lib().tc_lcc_graph_timings(self.handle, ctypes.byref(t)), "tc_lcc_graph_timings")
        return t

    def free(self):
        if self.handle:
            _check(lib().tc_lcc_graph_free(self.handle), "tc_lcc_graph_free")
            self.handle = None

    def __del__(self):
        try:
            if self.handle and lib() is not None:
                lib().tc_lcc_graph_free(self.handle)
        except Exception:
            pass


class BatchArgs:
    """The pointer arrays of one batch (graph handles, output pointers), built once: a batch that is
    submitted many times need not marshal thousands of pointers each time.  Keeps the graphs and
    outputs alive while it exists."""

    def __init__(self, graphs, tris, lccs=None):
        count = len(graphs)
        self.count = count
        # built by numpy from the handles and data pointers (a ctypes array built from a list of
        # Python ints costs about twice as much for thousands of graphs)
        self.gh = np.fromiter(((g.handle.value or 0) if g.handle else 0 for g in graphs), dtype=np.uint64,
                              count=count)
        self.th = np.fromiter((t.data_ptr() for t in tris), dtype=np.uint64, count=count)
        self.lh = np.fromiter(((l.data_ptr() if l is not None else 0) for l in (lccs or [None] * count)),
                              dtype=np.uint64, count=count)
        self._keep = (list(graphs), list(tris), list(lccs) if lccs else None)


class Context:
    """One GPU: memory pool with an optional HBM budget, tuning, batch queues (tc_lcc_ctx)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        self.device = device
        h = ctypes.c_void_p()
        _check(lib().tc_lcc_ctx_create(device, budget_bytes, ctypes.byref(h)), "tc_lcc_ctx_create")
        self.handle = h

    def build_csr(self, n: int, src, dst, offset_bytes: int = 0, stream=None, _entry: str = "tc_lcc_build_csr") -> Graph:
        """src/dst: int32 torch CUDA tensors (device path) or numpy arrays (host path)."""
        import torch
        if isinstance(src, torch.Tensor):
            assert src.dtype == torch.int32 and dst.dtype == torch.int32 and src.is_contiguous() and dst.is_contiguous()
            assert src.numel() == dst.numel()
            on_dev = 1 if src.is_cuda else 0
            ps, pd, m = ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), src.numel()
            keep = (src, dst)
        else:
            s = np.ascontiguousarray(src, dtype=np.int32)
            d = np.ascontiguousarray(dst, dtype=np.int32)
            assert s.shape == d.shape
            on_dev, ps, pd, m = 0, ctypes.c_void_p(s.ctypes.data), ctypes.c_void_p(d.ctypes.data), s.size
            keep = (s, d)
        h = ctypes.c_void_p()
        _check(getattr(lib(), _entry)(self.handle, n, m, ps, pd, on_dev, offset_bytes, _stream_ptr(stream),
                                      ctypes.byref(h)), _entry)
        del keep
        return Graph(self, h)

    def build_directed(self, n: int, src, dst, offset_bytes: int = 0, stream=None) -> Graph:
        """Directed input (tc_lcc_build_directed): src[e] -> dst[e]; Graph.run then gives the
        numerator and the clustering coefficient of Eq. 1.  Same argument forms as build_csr."""
        return self.build_csr(n, src, dst, offset_bytes=offset_bytes, stream=stream, _entry="tc_lcc_build_directed")

    def build_streamed(self, n: int, m_in: int, source, chunk_pairs: int = 0, partition_pairs: int = 0,
                       stream=None) -> Graph:
        """tc_lcc_build_streamed: pairs pulled from `source(first, count, src_ptr, dst_ptr, stream_ptr)`,
        which writes pairs [first, first + count) into the two device buffers (int addresses) with
        work on the given HIP stream, the same pairs on every call.  An exception in the source
        ends the build with INVALID_ARGUMENT and is raised again here."""
        errors = []

        def cb(_user, first, count, sp, dp, stp):
            try:
                source(int(first), int(count), int(sp or 0), int(dp or 0), int(stp or 0))
                return 0
            except Exception as e:  # noqa: BLE001 - re-raised below
                errors.append(e)
                return 1

        fn = PAIR_SOURCE(cb)
        h = ctypes.c_void_p()
        status = lib().tc_lcc_build_streamed(self.handle, n, m_in, fn, None, chunk_pairs, partition_pairs,
                                             _stream_ptr(stream), ctypes.byref(h))
        if errors:
            raise errors[0]
        _check(status, "tc_lcc_build_streamed")
        return Graph(self, h)

    def tuning(self) -> Tuning:
        t = Tuning()
        _check(lib().tc_lcc_get_tuning(self.handle, ctypes.byref(t)), "tc_lcc_get_tuning")
        return t

    def set_tuning(self, **kw):
        t = self.tuning()
        for k, v in kw.items():
            setattr(t, k, v)
        _check(lib().tc_lcc_set_tuning(self.handle, ctypes.byref(t)), "tc_lcc_set_tuning")
        return t

    def set_profiling(self, on: bool = True):
        _check(lib().tc_lcc_set_profiling(self.handle, 1 if on else 0), "tc_lcc_set_profiling")

    def memory(self):
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().tc_lcc_ctx_memory(self.handle, ctypes.byref(a), ctypes.byref(b)), "tc_lcc_ctx_memory")
        return int(a.value), int(b.value)

    def fail_alloc_after(self, after: int):
        """Failure injection (tc_lcc_debug_fail_alloc): the next `after` device allocations
        succeed, the one after fails; a negative value turns it off."""
        _check(lib().tc_lcc_debug_fail_alloc(self.handle, after), "tc_lcc_debug_fail_alloc")

    def batch_submit(self, graphs, tris=None, lccs=None) -> int:
        """tc_lcc_batch_submit: `graphs` with their outputs `tris` (and `lccs`), or a BatchArgs
        built once for repeated submissions of the same batch."""
        a = graphs if isinstance(graphs, BatchArgs) else BatchArgs(graphs, tris, lccs)
        tk = ctypes.c_uint64()
        _check(lib().tc_lcc_batch_submit(self.handle, a.count, a.gh.ctypes.data, a.th.ctypes.data, a.lh.ctypes.data,
                                         ctypes.byref(tk)), "tc_lcc_batch_submit")
        return int(tk.value)

    def batch_poll(self, ticket: int, block: bool = False):
        """(done?, graphs_done)."""
        done = ctypes.c_int()
        s = lib().tc_lcc_batch_poll(self.handle, ticket, 1 if block else 0, ctypes.byref(done))
        if s == NOT_READY:
            return False, int(done.value)
        _check(s, "tc_lcc_batch_poll")
        return True, int(done.value)

    def autotune(self, graphs, what: int = 3, reps: int = 3, path: str | None = None) -> Tuning:
        """Time candidate settings on `graphs` and install the fastest (tc_lcc_autotune):
        what & 1 single-graph bins/probe, what & 2 the batched launch's knobs."""
        count = len(graphs)
        gh = (ctypes.c_void_p * count)(*[g.handle for g in graphs])
        t = Tuning()
        _check(lib().tc_lcc_autotune(self.handle, count, gh, what, reps, path.encode() if path else None,
                                     ctypes.byref(t)), "tc_lcc_autotune")
        return t

    def load_tuning(self, path: str):
        """Install a setting saved by autotune (tc_lcc_tuning_load)."""
        _check(lib().tc_lcc_tuning_load(self.handle, path.encode()), "tc_lcc_tuning_load")

    def batch_progress(self, ticket: int, count: int):
        """Per-graph completion flags (list of bool, submission order) of an unreleased ticket."""
        flags = (ctypes.c_uint8 * max(count, 1))()
        _check(lib().tc_lcc_batch_progress(self.handle, ticket, count, flags), "tc_lcc_batch_progress")
        return [bool(flags[i]) for i in range(count)]

    def close(self):
        if self.handle:
            _check(lib().tc_lcc_ctx_destroy(self.handle), "tc_lcc_ctx_destroy")
            self.handle = None


class Server:
    """Continuous-batching request server (tc_lcc_server); max_inflight = max_batch = 1 is the
    plain one-request-per-launch path."""

    def __init__(self, ctx: Context, budget_bytes: int = 0, max_inflight: int = 2, max_batch: int = 4096):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(lib().tc_lcc_server_create(ctx.handle, budget_bytes, max_inflight, max_batch, ctypes.byref(h)),
               "tc_lcc_server_create")
        self.handle = h

    def submit(self, graph: Graph, tri, lcc=None) -> int:
        rid = ctypes.c_uint64()
        _check(lib().tc_lcc_server_submit(self.handle, graph.handle, _dptr(tri), _dptr(lcc), ctypes.byref(rid)),
               "tc_lcc_server_submit")
        return int(rid.value)

    def poll(self, request_id: int, block: bool = False):
        """RequestInfo when the request is complete, None while it is queued or running."""
        info = RequestInfo()
        s = lib().tc_lcc_server_poll(self.handle, request_id, 1 if block else 0, ctypes.byref(info))
        if s == NOT_READY:
            return None
        _check(s, "tc_lcc_server_poll")
        return info

    def close(self):
        if self.handle:
            _check(lib().tc_lcc_server_destroy(self.handle), "tc_lcc_server_destroy")
            self.handle = None


def hbm_copy(src, dst, stream=None):
    """tc_lcc_hbm_copy: dst[:] = src[:] (device tensors of equal byte size) by the streaming copy
    kernel, asynchronous on `stream`."""
    nb = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nb and src.is_cuda and dst.is_cuda
    _check(lib().tc_lcc_hbm_copy(_dptr(src), _dptr(dst), nb, _stream_ptr(stream)), "tc_lcc_hbm_copy")


def tc_lcc(n: int, src, dst, offset_bytes: int = 0, ctx: Context | None = None):
    """Convenience: build, run, return (tri int64 tensor, lcc float64 tensor) on the device."""
    own = ctx is None
    ctx = ctx or Context(0)
    g = ctx.build_csr(n, src, dst, offset_bytes=offset_bytes)
    tri, lcc = g.run()
    import torch
    torch.cuda.current_stream().synchronize()
    g.free()
    if own:
        ctx.close()
    return tri, lcc
