"""Benchmark: per-vertex triangle counts + LCC on one MI355X.

One step = the whole path over one graph whose raw pairs are already in HBM:
build (loop removal, sort, dedup, degrees, rank, orientation, reverse lists,
work bins) + count (intersection + scatter) + LCC epilogue, then free.
Prints one JSON line with the roofline of the count kernel and the oracle's CPU rate.

    python bench.py [--steps K] [--warmup W] [--workload rmat_s23_ef16]
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
RMAT_ABC_TXT = "a=0.57 b=0.19 c=0.19"
METRIC = "edges/sec (TEPS) for TC+LCC, batched vs per-graph, p50/p99 latency"

WORKLOADS = {
    "rmat_s23_ef16": dict(kind="rmat", scale=23, ef=16, seed=1, offset_bytes=8),
    "rmat_s20_ef16": dict(kind="rmat", scale=20, ef=16, seed=1, offset_bytes=8),
    "er_4096_deg16": dict(kind="er", n=4096, seed=1, offset_bytes=4),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_input(w):
    import synth
    if w["kind"] == "rmat":
        return synth.rmat_scale(w["scale"], w["ef"], seed=w["seed"])
    return synth.er_4096(seed=w["seed"])


def count_bytes(info) -> int:
    """Algorithmic bytes of one count launch (the dominant kernel), from the graph's own counts.

    4 B per candidate probe (one id of a tail of N+(u)), (8 + w) B per kept in-edge
    (u, tail start, tail length; compact reverse lists: u, the 2-byte position and u's two
    8-byte row offsets, 22 B), 4 B per staged entry of N+(v), (4w + 4) B per active vertex (its
    two offset pairs and its slot in the work list), 8 B per vertex for t.
    """
    w = int(info.offset_bytes)
    per_in = 22 if int(getattr(info, "compact", 0)) else 8 + w
    return (4 * int(info.wedges) + per_in * int(info.kept_in_edges) + 4 * int(info.staged_entries)
            + (4 * w + 4) * int(info.active_vertices) + 8 * int(info.n))


def full_list_bytes(info) -> int:
    """The whole-list streaming figure 4 W + (4 + 2w) m + (2w + 16) n, W = sum over oriented
    edges (u -> v) of |N+(v)|: bytes a push-style merge would read (reported for comparison)."""
    w = int(info.offset_bytes)
    return 4 * int(info.push_words) + (4 + 2 * w) * int(info.m) + (2 * w + 16) * int(info.n)


COUNT_SOURCES = ("count.hip", "count_device.hpp", "common.hpp", "internal.hpp")


def _code_only(text: str) -> str:
    """C++ source without comments and blank lines (an edit of a comment leaves the kernel as
    it was).  String literals in these sources hold no comment markers."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = [re.sub(r"//.*", "", line).rstrip() for line in text.splitlines()]
    return "\n".join(line for line in lines if line.strip())


def count_source_sha() -> str:
    """SHA-256 over the code (comments dropped) of the sources that define the count kernel, in
    a fixed order."""
    h = hashlib.sha256()
    for name in COUNT_SOURCES:
        with open(os.path.join(ROOT, "paper_2202_13976_amd", "csrc", name), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def stored_traffic():
    """HBM bytes per count launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", "count_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != count_source_sha():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(n, s, d, target_s: float, samples: int = 3):
    """The oracle's forward algorithm, single-threaded and pinned to one core, on a bounded
    sample of vertices: the median rate of `samples` runs of about target_s / samples each."""
    import numpy as np
    import oracle
    g = oracle.csr(n, s, d)
    old_aff = os.sched_getaffinity(0)
    core = min(old_aff)
    os.sched_setaffinity(0, {core})  # the calling thread, which runs the oracle
    try:
        t0 = time.perf_counter()
        oracle.tc_forward_range(g, 0, 0)  # setup only: orientation of the whole graph
        setup = time.perf_counter() - t0
        probe = max(1, n // 2000)
        t0 = time.perf_counter()
        oracle.tc_forward_range(g, 0, probe)
        t1 = time.perf_counter() - t0 - setup
        per = target_s / samples
        frac = min(1.0, max(probe / n, (probe / n) * per / max(t1, 1e-3)))
        hi = max(probe, int(n * frac))
        rates, secs = [], []
        for _ in range(samples):
            t0 = time.perf_counter()
            _, edges = oracle.tc_forward_range(g, 0, hi)
            el = time.perf_counter() - t0 - setup
            rates.append(edges / el)
            secs.append(el)
    finally:
        os.sched_setaffinity(0, old_aff)
    k = int(np.argsort(rates)[len(rates) // 2])
    return {"value": rates[k], "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"forward algorithm (lowest-ranked vertex owns each triangle) over the "
                      f"{hi} vertices with ids in [0, {hi}) of {n} (ids are a random permutation, "
                      f"so a uniform vertex sample); {edges} oriented edges per run; median of "
                      f"{samples} runs ({', '.join(f'{x:.1f}' for x in secs)} s) on one pinned core "
                      f"(cpu {core}); orientation setup ({setup:.1f} s) excluded",
            "runs_edges_per_s": rates, "seconds": float(sum(secs))}


GOLDEN = os.path.join(ROOT, "tests", "golden")


def golden_lines(name):
    """Per-graph lines stored by tests/golden/make_golden.py from the oracle (m, triangles,
    sha256(t || LCC)[:16])."""
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)["graphs"]


def result_line(m, tri, lcc) -> str:
    import numpy as np
    t = tri.cpu().numpy().astype(np.uint64)
    l = lcc.cpu().numpy()
    h = hashlib.sha256(t.astype("<u8").tobytes() + l.astype("<f8").tobytes()).hexdigest()[:16]
    return f"{m} {int(t.sum()) // 3} {h}"


def result_lines(torch, ms, tris, lccs):
    """result_line of many graphs with one device-to-host copy of each kind."""
    import numpy as np
    sizes = [t.numel() for t in tris]
    cut = np.cumsum(sizes)[:-1]
    ts = np.split(torch.cat([t.reshape(-1) for t in tris]).cpu().numpy().astype(np.uint64), cut)
    ls = np.split(torch.cat([x.reshape(-1) for x in lccs]).cpu().numpy(), cut)
    out = []
    for m, t, l in zip(ms, ts, ls):
        h = hashlib.sha256(t.astype("<u8").tobytes() + l.astype("<f8").tobytes()).hexdigest()[:16]
        out.append(f"{m} {int(t.sum()) // 3} {h}")
    return out


def hbm_copy_rate(torch, pkg, nbytes: int = 2 << 30, reps: int = 10):
    """Achievable HBM bandwidth: the library's streaming copy kernel (tc_lcc_hbm_copy) over
    nbytes, timed with HIP events on its stream; read + written bytes over the median time."""
    import numpy as np
    dev = torch.device("cuda", 0)
    a = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    for _ in range(2):
        pkg.hbm_copy(a, b, st)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        pkg.hbm_copy(a, b, st)
        e1.record(st)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ok = bool(torch.equal(a, b))
    del a, b
    med = float(np.median(ts))
    return {"kernel": "k_hbm_copy (16-byte nontemporal loads and stores)", "bytes_read": nbytes,
            "bytes_written": nbytes, "median_ms": med, "gbs": 2 * nbytes / (med * 1e-3) / 1e9, "copy_correct": ok}


def build_bytes(info, raw_pairs: int) -> int:
    """Least HBM bytes of one build: the raw pairs read once (8 B per pair) and the graph
    written once (its device bytes).  The sorts move far more; this is the floor."""
    return 8 * int(raw_pairs) + int(info.device_bytes)


def ext_bench(ctx, torch, pkg, n, src, dst, offset_bytes, triangles: int, reps: int = 5):
    """The two extensions of the count on the same workload, each timed on HIP events of its
    stream (the graph's phase timings): per-edge triangle counts (tc_lcc_run_edges) and the
    clustering coefficient of Eq. 1 with the raw pairs taken as directed edges (as drawn)."""
    import numpy as np
    out = {}
    ctx.set_profiling(True)
    g = ctx.build_csr(n, src, dst, offset_bytes=offset_bytes)
    info = g.info()
    g.run_edges()
    cnt, rest, wall = [], [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        tri, lcc, es, ed, ec = g.run_edges()
        wall.append(time.perf_counter() - t0)
        tm = g.timings()
        cnt.append(tm.run_count_ms)
        rest.append(tm.run_epilogue_ms)
    sum_c = int(ec.to(torch.int64).sum())
    sum_t = int(tri.sum())
    g.free()
    del es, ed, ec
    # bytes of the extended count: the plain count's, plus one read-modify-write of a 4-byte
    # counter per triangle (its tail entry), per kept in-edge (its tail's hits) and per staged
    # entry (the flush), and the clearing of the m counters
    w = int(info.offset_bytes)
    eb = count_bytes(info) + 8 * triangles + 8 * int(info.kept_in_edges) + 8 * int(info.staged_entries) + 4 * int(info.m)
    c_ms = float(np.median(cnt))
    out["edges"] = {"entry": "tc_lcc_run_edges", "m": int(info.m), "count_ms": c_ms,
                    "epilogue_and_edge_output_ms": float(np.median(rest)), "call_ms": float(np.median(wall)) * 1e3,
                    "teps": int(info.m) / (float(np.median(wall))), "alg_bytes_per_launch": eb,
                    "roofline_frac": eb / (c_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "sum_edge_counts_equals_sum_t": sum_c == sum_t}
    gd = ctx.build_directed(n, src, dst, offset_bytes=offset_bytes)
    bt = gd.timings().as_dict()
    infod = gd.info()
    num = torch.empty(n, dtype=torch.int64, device=src.device)
    cl = torch.empty(n, dtype=torch.float64, device=src.device)
    gd.run(num, cl)
    dc = []
    for _ in range(reps):
        gd.run(num, cl)
        dc.append(gd.timings().run_count_ms)
    torch.cuda.synchronize()
    gd.free()
    # directed: the plain count's bytes plus the direction byte of every hit's two list entries,
    # of every kept in-edge and of every staged entry
    db = count_bytes(infod) + 2 * triangles + int(infod.kept_in_edges) + int(infod.staged_entries)
    d_ms = float(np.median(dc))
    out["directed"] = {"entry": "tc_lcc_build_directed + tc_lcc_run (Eq. 1)", "directed_pairs": int(src.numel()),
                       "skeleton_m": int(infod.m), "build_ms": sum(v for k, v in bt.items() if k.startswith("build")),
                       "count_ms": d_ms, "teps": int(infod.m) / (d_ms * 1e-3), "alg_bytes_per_launch": db,
                       "roofline_frac": db / (d_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "sum_numerator": int(num.sum())}
    ctx.set_profiling(False)
    return out


def streamed_bench(ctx, torch, pkg, log_fn, scale: int, ef: int = 16, seed: int = 1,
                   partition_pairs: int = 3 << 30, chunk: int = 1 << 28, reps: int = 3):
    """R-MAT at 2^scale vertices and ef * 2^scale pairs (the large-scale recipe: Feistel
    relabelling, generated on the GPU in any range), built by tc_lcc_build_streamed from a source
    that regenerates each chunk on every pass, then counted.  The generation is input creation:
    one pass of it alone is timed to show its share of the build.  Checks: sum t = 0 mod 3,
    t(v) <= C(d(v), 2), and LCC equal to 2 t / (d (d - 1)) computed on the host in binary64."""
    import numpy as np
    import synth
    n, m_in = 1 << scale, ef << scale
    dev = torch.device("cuda", 0)
    st = torch.cuda.current_stream()
    gen = synth.GpuRmatFeistel(scale, seed=seed)
    per_pass = -(-m_in // chunk)
    buf = torch.empty(2 * min(chunk, m_in), dtype=torch.int32, device=dev)
    half = min(chunk, m_in)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for first in range(0, m_in, chunk):
        cnt = min(chunk, m_in - first)
        gen.gen(first, cnt, buf.data_ptr(), buf.data_ptr() + 4 * half, st.cuda_stream)
    e1.record(st)
    e1.synchronize()
    gen_ms = e0.elapsed_time(e1)
    del buf
    calls = [0]

    def source(first, count, sp, dp, stp):
        calls[0] += 1
        gen.gen(first, count, sp, dp, stp)

    ctx.set_profiling(True)
    torch.cuda.synchronize()
    log_fn(f"[bench] streamed build of R-MAT S{scale} EF{ef}: {m_in} pairs, partitions of {partition_pairs}")
    t0 = time.perf_counter()
    g = ctx.build_streamed(n, m_in, source, chunk_pairs=chunk, partition_pairs=partition_pairs)
    build_s = time.perf_counter() - t0
    passes = calls[0] / per_pass
    bt = g.timings().as_dict()
    info = g.info()
    tri = torch.empty(n, dtype=torch.int64, device=dev)
    lcc = torch.empty(n, dtype=torch.float64, device=dev)
    log_fn(f"[bench] count S{scale}: m={int(info.m)} wedges={int(info.wedges)}")
    g.run(tri, lcc)
    torch.cuda.synchronize()
    cnt, tot = [], []
    for _ in range(reps):
        g.run(tri, lcc)
        tm = g.timings()
        cnt.append(tm.run_count_ms)
        tot.append(tm.run_zero_ms + tm.run_count_ms + tm.run_epilogue_ms)
    torch.cuda.synchronize()
    deg = np.empty(n, dtype=np.int64)
    pkg.lib().tc_lcc_graph_export(g.handle, deg.ctypes.data, None, None, None)
    g.free()
    ctx.set_profiling(False)
    t = tri.cpu().numpy().view(np.uint64)
    l = lcc.cpu().numpy()
    del tri, lcc
    total = int(t.sum(dtype=np.uint64))
    du = deg.astype(np.uint64)
    pairs_at = du * (du - np.uint64(1)) // np.uint64(2)
    bound_ok = bool(np.all(t[deg >= 2] <= pairs_at[deg >= 2])) and bool(np.all(t[deg < 2] == 0))
    want = np.zeros(n, dtype=np.float64)
    big = deg >= 2
    want[big] = (2 * t[big]).astype(np.float64) / (du[big] * (du[big] - np.uint64(1))).astype(np.float64)
    lcc_ok = want.tobytes() == l.tobytes()
    c_ms = float(np.median(cnt))
    alg = count_bytes(info)
    return {"workload": f"rmat_s{scale}_ef{ef} (R-MAT {RMAT_ABC_TXT}, Feistel-relabelled ids, generated on "
                        f"the GPU per pass)", "n": n, "raw_pairs": m_in, "m_undirected": int(info.m),
            "entry": "tc_lcc_build_streamed + tc_lcc_run", "partition_pairs": partition_pairs,
            "chunk_pairs": chunk, "passes": passes, "build_s": build_s,
            "build_phases_ms": {k: v for k, v in bt.items() if k.startswith("build")},
            "generation_ms_per_pass": gen_ms, "generation_share_of_build": passes * gen_ms * 1e-3 / build_s,
            "count_ms": c_ms, "run_ms": float(np.median(tot)), "count_teps": int(info.m) / (c_ms * 1e-3),
            "roofline": {"bound": "hbm", "alg_bytes_per_launch": alg, "achieved": alg / (c_ms * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": alg / (c_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "graph": {"wedges": int(info.wedges), "kept_in_edges": int(info.kept_in_edges),
                      "max_out_degree": int(info.max_out_degree), "max_degree": int(info.max_degree),
                      "global_vertices": int(info.global_vertices), "block_vertices": int(info.block_vertices),
                      "device_bytes": int(info.device_bytes), "triangles": total // 3},
            "checks": {"sum_t_divisible_by_3": total % 3 == 0, "t_at_most_pairs_of_neighbours": bound_ok,
                       "lcc_equals_host_division": lcc_ok}}


def large_bench(torch, pkg, log_fn, scale: int, ef: int = 16, seed: int = 1, sample: int = 24, reps: int = 3):
    """R-MAT at 2^scale vertices and ef * 2^scale raw pairs (Table II's recipe, the host
    generator), built by tc_lcc_build_csr from the raw pairs in HBM (the one-pass build; offsets
    of 4 bytes while the pairs number fewer than 2^31) and counted.  Reports the build and count
    times and the count kernel's roofline, checks every vertex against invariants (sum t = 0 mod 3,
    t <= C(d, 2), LCC equal to 2 t / (d (d - 1)) divided on the host in binary64), and checks t and
    LCC of `sample` vertices (drawn uniformly among those with at least two pair ends, plus the one
    with the most) against the oracle's count straight from the raw pairs (on the host, a few
    seconds per vertex at scale 26)."""
    import numpy as np
    import oracle
    import synth
    n, m_in = 1 << scale, ef << scale
    log_fn(f"[bench] large leg: generating R-MAT S{scale} EF{ef} ({m_in} pairs) on the host")
    t0 = time.perf_counter()
    n, s, d = synth.rmat_scale(scale, ef, seed)
    gen_s = time.perf_counter() - t0
    dev = torch.device("cuda", 0)
    src = torch.from_numpy(s).to(dev)
    dst = torch.from_numpy(d).to(dev)
    ctx = pkg.Context(0)
    ctx.set_profiling(True)
    try:
        build_ms, count_ms, walls = [], [], []
        g = None
        for r in range(reps):
            log_fn(f"[bench] large leg: build {r + 1} of {reps}")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            g = ctx.build_csr(n, src, dst, offset_bytes=0)
            torch.cuda.synchronize()
            walls.append((time.perf_counter() - t1) * 1e3)
            tm = g.timings().as_dict()
            build_ms.append(sum(v for k, v in tm.items() if k.startswith("build")))
            if r + 1 < reps:
                g.free()
        del src, dst
        torch.cuda.empty_cache()
        info = g.info()
        tri = torch.empty(n, dtype=torch.int64, device=dev)
        lcc = torch.empty(n, dtype=torch.float64, device=dev)
        for r in range(reps + 1):
            log_fn(f"[bench] large leg: count {r + 1} of {reps + 1}")
            g.run(tri, lcc)
            torch.cuda.synchronize()
            if r:
                count_ms.append(g.timings().run_count_ms)
        deg = np.empty(n, dtype=np.int64)
        pkg.lib().tc_lcc_graph_export(g.handle, deg.ctypes.data, None, None, None)
        g.free()
        t = tri.cpu().numpy().view(np.uint64)
        lv = lcc.cpu().numpy()
        del tri, lcc
    finally:
        ctx.close()
        torch.cuda.empty_cache()
    total = int(t.sum(dtype=np.uint64))
    du = deg.astype(np.uint64)
    big = deg >= 2
    bound_ok = bool(np.all(t[big] <= du[big] * (du[big] - np.uint64(1)) // np.uint64(2))) and bool(np.all(t[~big] == 0))
    want = np.zeros(n, dtype=np.float64)
    want[big] = (2 * t[big]).astype(np.float64) / (du[big] * (du[big] - np.uint64(1))).astype(np.float64)
    lcc_ok = want.tobytes() == lv.tobytes()
    res = {"workload": f"rmat_s{scale}_ef{ef} (R-MAT {RMAT_ABC_TXT}, host generator, seed {seed})",
           "n": n, "raw_pairs": m_in, "m_undirected": int(info.m), "offset_bytes": int(info.offset_bytes),
           "entry": "tc_lcc_build_csr + tc_lcc_run", "generation_s": gen_s,
           "build_ms": float(np.median(build_ms)), "build_wall_ms": float(np.median(walls)),
           "count_ms": float(np.median(count_ms)),
           "teps_build_and_count": int(info.m) / ((np.median(build_ms) + np.median(count_ms)) * 1e-3),
           "graph": {"wedges": int(info.wedges), "kept_in_edges": int(info.kept_in_edges),
                     "max_out_degree": int(info.max_out_degree), "max_degree": int(info.max_degree),
                     "device_bytes": int(info.device_bytes), "triangles": total // 3},
           "checks": {"sum_t_divisible_by_3": total % 3 == 0, "t_at_most_pairs_of_neighbours": bound_ok,
                      "lcc_equals_host_division": lcc_ok}}
    alg = count_bytes(info)
    c = res["count_ms"] * 1e-3
    res["roofline"] = {"bound": "hbm", "alg_bytes_per_launch": alg, "achieved": alg / c / 1e9, "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": alg / c / 1e9 / HBM_PEAK_GBS}
    if sample > 0:
        # vertices with at least two pair ends (counted on the host), uniformly, and the vertex with
        # the most pair ends
        ends = np.bincount(s, minlength=n) + np.bincount(d, minlength=n)
        rng = np.random.default_rng(seed)
        vs = np.sort(rng.choice(np.flatnonzero(ends >= 2), size=sample - 1, replace=False))
        vs = np.append(vs, int(np.argmax(ends)))
        del ends
        t2 = time.perf_counter()
        tr, dr = [], []
        for i, v in enumerate(vs):
            a, b = oracle.tc_vertex_pairs(n, s, d, int(v))
            tr.append(a)
            dr.append(b)
            log_fn(f"[bench] large leg: oracle vertex {i + 1} of {sample}: v={int(v)} d={b} t={a}")
        tr = np.array(tr, dtype=np.uint64)
        lr = np.array([oracle.lcc_one(int(a), int(b)) for a, b in zip(tr, dr)])
        res["oracle_sample"] = {"vertices": int(sample), "seconds": time.perf_counter() - t2,
                                "degrees_equal": bool(np.array_equal(np.array(dr), deg[vs])),
                                "t_equal": bool(np.array_equal(tr, t[vs])),
                                "lcc_bits_equal": lr.tobytes() == lv[vs].tobytes(),
                                "sampled_triangles": int(tr.sum())}
    return res


def batch_bench(ctx, torch, pkg, log_fn, reps: int = 3, autotune: bool = True):
    """4096 uneven graphs: a loop of single-graph runs against one batched submission."""
    import numpy as np
    import synth
    specs = synth.batch_specs()
    dev = torch.device("cuda", 0)
    graphs, tris, lccs, ms = [], [], [], []
    m_total = 0
    wedges = 0
    alg_bytes = 0
    log_fn(f"[bench] building {len(specs)} batch graphs")
    for spec in specs:
        n, s, d = synth.make(spec)
        g = ctx.build_csr(n, torch.from_numpy(s).to(dev), torch.from_numpy(d).to(dev), offset_bytes=4)
        graphs.append(g)
        info = g.info()
        ms.append(int(info.m))
        m_total += int(info.m)
        wedges += int(info.wedges)
        alg_bytes += count_bytes(info)
        tris.append(torch.empty(n, dtype=torch.int64, device=dev))
        lccs.append(torch.empty(n, dtype=torch.float64, device=dev))
    loop_tris = [torch.empty_like(t) for t in tris]

    def per_graph():
        for g, t, l in zip(graphs, loop_tris, lccs):
            g.run(t, l)
        torch.cuda.synchronize()

    submit_s = []
    bargs = pkg.BatchArgs(graphs, tris, lccs)

    def batched():
        t0 = time.perf_counter()
        tk = ctx.batch_submit(bargs)
        submit_s.append(time.perf_counter() - t0)
        ctx.batch_poll(tk, block=True)

    per_graph()
    batched()
    t_loop, t_batch = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        per_graph()
        t_loop.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        batched()
        t_batch.append(time.perf_counter() - t0)
    same = all(torch.equal(a, b) for a, b in zip(tris, loop_tris))
    ref = golden_lines("batch4096_seed7")
    oracle_ok = None if ref is None else result_lines(torch, ms, tris, lccs) == ref
    tl, tb = float(np.median(t_loop)), float(np.median(t_batch))
    res = {"workload": "4096 graphs, n log-uniform in [64, 16384], half uniform (avg degree 8-32), "
                       "half R-MAT (EF 8-16), int32 offsets",
           "graphs": len(specs), "m_total": m_total, "wedges": wedges, "alg_bytes": alg_bytes,
           "per_graph_ms": tl * 1e3, "batched_ms": tb * 1e3, "speedup": tl / tb,
           "submit_host_ms": float(np.median(submit_s)) * 1e3,
           "per_graph_teps": m_total / tl, "batched_teps": m_total / tb, "results_identical": bool(same),
           "matches_oracle_digests": oracle_ok}
    if not autotune:
        for g in graphs:
            g.free()
        return res
    # the autotuner on the batched launch's knobs, then the same measurement again
    log_fn("[bench] autotuning the batched launch")
    default = ctx.tuning().as_dict()
    t0 = time.perf_counter()
    tuned = ctx.autotune(graphs, what=2, reps=3)
    tune_s = time.perf_counter() - t0
    for t in tris:
        t.fill_(-1)
    torch.cuda.synchronize()  # the batch runs on the library's streams, not ordered after torch's
    t_tuned = []
    for _ in range(reps):
        t0 = time.perf_counter()
        batched()
        t_tuned.append(time.perf_counter() - t0)
    same_tuned = all(torch.equal(a, b) for a, b in zip(tris, loop_tris))
    ctx.set_tuning(**default)
    for g in graphs:
        g.free()
    tt = float(np.median(t_tuned))
    res["autotuned"] = {"batch_grab": tuned.batch_grab, "batch_heavy_bits": tuned.batch_heavy_bits,
                        "batched_ms": tt * 1e3, "speedup": tl / tt, "tuning_seconds": tune_s,
                        "results_identical": bool(same_tuned)}
    return res


def run_timing(ctx, torch, n, src, dst, offset_bytes, tri, lcc, warm: int = 3, lo: int = 10, hi: int = 200):
    """tc_lcc_run alone on a resident graph, on HIP events of the launch stream: warm up, then
    repeat until the 95% interval of the median is within 5% of it (10 to 200 repeats)."""
    import numpy as np
    g = ctx.build_csr(n, src, dst, offset_bytes=offset_bytes)
    m = int(g.info().m)
    for _ in range(warm):
        g.run(tri, lcc)
    st = torch.cuda.current_stream()
    times = []
    while len(times) < hi:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        g.run(tri, lcc, stream=st)
        e1.record(st)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
        if len(times) >= lo:
            a = np.array(times)
            half = 1.96 * 1.2533 * a.std(ddof=1) / np.sqrt(len(a))  # normal approximation for the median
            if half <= 0.05 * np.median(a):
                break
    g.free()
    a = np.array(times)
    med = float(np.median(a))
    return {"median_ms": med, "p99_ms": float(np.percentile(a, 99)), "repeats": len(times),
            "teps": m / (med * 1e-3)}


def strategy_timing(ctx, torch, pkg, n, src, dst, offset_bytes, tri, reps: int = 4):
    """Count-kernel time of each probe strategy on one resident graph (median of `reps` runs
    after one warm-up; the schedule is rebuilt when the strategy changes), and whether its
    per-vertex counts equal those of the default strategy."""
    import numpy as np
    t0 = ctx.tuning().as_dict()
    g = ctx.build_csr(n, src, dst, offset_bytes=offset_bytes)
    out, ref = {}, None
    try:
        for name, kw in [("bitmap_or_hash", dict(probe=pkg.PROBE_AUTO)), ("hash", dict(probe=pkg.PROBE_HASH)),
                         ("sorted_binary_search", dict(probe=pkg.PROBE_SORTED)),
                         ("hybrid_eq3_merge_path_or_search", dict(probe=pkg.PROBE_MERGE))]:
            ctx.set_tuning(**kw)
            g.run(tri, None)
            ts = []
            for _ in range(reps):
                g.run(tri, None)
                ts.append(g.timings().run_count_ms)
            torch.cuda.synchronize()
            if ref is None:
                ref = tri.clone()
            out[name] = {"count_ms": float(np.median(ts)), "same_counts": bool(torch.equal(ref, tri))}
    finally:
        ctx.set_tuning(**t0)
        g.free()
    return out


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


SERVE_INFLIGHT = 4


def serve_bench(ctx, torch, log_fn, n_req: int = 2000, n_warm: int = 200, load: float = 0.7,
                sweep=(0.5, 0.9, 1.2), sweep_req: int = 1000, sweep_warm: int = 100):
    """Poisson request stream over a pool of resident R-MAT graphs: plain server (one request
    per launch) against the continuous-batching server, same arrivals, same GPU."""
    import numpy as np
    import paper_2202_13976_amd as pkg
    import synth
    dev = torch.device("cuda", 0)
    specs = synth.serving_specs(count=64, seed=9)
    graphs, outs, ms = [], [], []
    log_fn(f"[bench] building {len(specs)} resident serving graphs")
    for spec in specs:
        n, s, d = synth.make(spec)
        g = ctx.build_csr(n, torch.from_numpy(s).to(dev), torch.from_numpy(d).to(dev))
        graphs.append(g)
        ms.append(int(g.info().m))
        outs.append((torch.empty(n, dtype=torch.int64, device=dev), torch.empty(n, dtype=torch.float64, device=dev)))
    picks_all = synth.choices(n_warm + n_req, len(graphs), seed=13)

    def run(server, rate, n_req=n_req, n_warm=n_warm):
        picks = picks_all[:n_warm + n_req]
        gaps = synth.poisson_gaps(n_warm + n_req, rate, seed=11) if rate else np.zeros(n_warm + n_req)
        ids = []
        t0 = time.perf_counter()
        due = t0
        for k, gap in zip(picks, gaps):
            due += gap
            while time.perf_counter() < due:
                pass
            g = graphs[k]
            ids.append(server.submit(g, *outs[k]))
        infos = [server.poll(i, block=True) for i in ids]
        lat = np.array([(x.done_ns - x.arrival_ns) * 1e-6 for x in infos[n_warm:]])
        first = min(x.arrival_ns for x in infos[n_warm:])
        last = max(x.done_ns for x in infos[n_warm:])
        span = (last - first) * 1e-9
        edges = sum(ms[k] for k in picks[n_warm:])
        return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "teps": edges / span, "mean_batch": float(np.mean([x.batch_size for x in infos[n_warm:]]))}

    # saturation of the plain path: all requests submitted at once
    plain = pkg.Server(ctx, budget_bytes=0, max_inflight=1, max_batch=1)
    sat = run(plain, 0.0)
    plain.close()
    torch.cuda.synchronize()
    # every graph of the pool was requested at least once by now (2000 picks of 64): the plain
    # path's outputs are the reference for the batched runs, and are checked against the oracle
    seen = sorted(set(int(k) for k in picks_all))
    ref_outs = {k: (outs[k][0].clone(), outs[k][1].clone()) for k in seen}
    gold = golden_lines("serving64_seed9")
    plain_oracle_ok = None
    if gold is not None:
        plain_oracle_ok = result_lines(torch, [ms[k] for k in seen], [ref_outs[k][0] for k in seen],
                                       [ref_outs[k][1] for k in seen]) == [gold[k] for k in seen]
    t_edges = sum(ms[k] for k in picks_all[n_warm:])
    sat_rate = n_req * sat["teps"] / t_edges  # requests per second when the plain path is saturated
    rate = load * sat_rate
    log_fn(f"[bench] plain saturation {sat_rate:.0f} req/s; offered load {rate:.0f} req/s")
    res = {"workload": "64 resident R-MAT EF16 graphs, n log-uniform in [2^10, 2^21]; Poisson arrivals, "
                       "uniform graph choice", "requests": n_req, "warmup": n_warm,
           "plain_saturation_rps": sat_rate, "offered_rps": rate, "load": load}
    plain = pkg.Server(ctx, budget_bytes=0, max_inflight=1, max_batch=1)
    res["plain"] = run(plain, rate)
    batched = pkg.Server(ctx, budget_bytes=8 << 30, max_inflight=SERVE_INFLIGHT, max_batch=4096)
    res["batched"] = run(batched, rate)
    res["batched_saturated"] = run(batched, 0.0)
    res["batched_inflight"] = SERVE_INFLIGHT
    res["sweep"] = []
    for x in sweep:
        log_fn(f"[bench] serving sweep at {x} x plain saturation")
        r = x * sat_rate
        res["sweep"].append({"load": x, "offered_rps": r,
                             "plain": run(plain, r, sweep_req, sweep_warm),
                             "batched": run(batched, r, sweep_req, sweep_warm)})
    plain.close()
    batched.close()
    torch.cuda.synchronize()
    # the last runs were the batched server's: every request's outputs overwrite their graph's
    res["results_identical"] = all(torch.equal(outs[k][0], ref_outs[k][0]) and
                                   torch.equal(outs[k][1], ref_outs[k][1]) for k in seen)
    res["matches_oracle_digests"] = plain_oracle_ok
    res["graphs_checked"] = len(seen)
    for g in graphs:
        g.free()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat_s23_ef16", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the many-small-graphs comparison")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving comparison")
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuner in the batch leg")
    ap.add_argument("--no-strategies", action="store_true", help="skip the per-probe-strategy count times")
    ap.add_argument("--no-ext", action="store_true", help="skip the per-edge and directed legs")
    ap.add_argument("--streamed-scale", type=int, default=0,
                    help="also build R-MAT at this (even) scale with the streamed build and count it; "
                         "0 skips it.  Scales above 16 are refused: a run at scale 26 ended in a GPU "
                         "memory fault whose cause is not found yet")
    ap.add_argument("--streamed-only", action="store_true", help="run only the streamed leg")
    ap.add_argument("--large-scale", type=int, default=0,
                    help="run only a large leg: R-MAT at this scale from the host generator through the "
                         "one-pass build (pairs in HBM), with sampled oracle checks; 0 skips it")
    ap.add_argument("--large-sample", type=int, default=24, help="vertices the large leg checks against the oracle")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, copy 1 GiB with the library's streaming copy kernel 3 times "
                         "(reference for HBM counters)")
    args = ap.parse_args()
    if args.streamed_scale > 16 or (args.streamed_only and not args.streamed_scale):
        print("bench.py: the streamed leg is limited to scales up to 16 until the memory fault seen "
              "at scale 26 is explained", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the path runs on a "
              f"single GPU (the graph, its count and its LCC live in one GPU's HBM)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2202_13976_amd as pkg

    if args.large_scale:
        res = large_bench(torch, pkg, log, args.large_scale, sample=args.large_sample)
        print(json.dumps({"large": res}), flush=True)
        return

    if args.streamed_only:
        ctx = pkg.Context(0)
        res = streamed_bench(ctx, torch, pkg, log, args.streamed_scale)
        ctx.close()
        print(json.dumps({"streamed": res}), flush=True)
        return

    w = WORKLOADS[args.workload]
    log(f"[bench] generating {args.workload}")
    n, s, d = make_input(w)
    dev = torch.device("cuda", 0)
    src = torch.from_numpy(s).to(dev)
    dst = torch.from_numpy(d).to(dev)
    tri = torch.empty(n, dtype=torch.int64, device=dev)
    lcc = torch.empty(n, dtype=torch.float64, device=dev)
    ctx = pkg.Context(0)
    ctx.set_profiling(True)

    def step():
        g = ctx.build_csr(n, src, dst, offset_bytes=w["offset_bytes"])
        g.run(tri, lcc)
        tm = g.timings()
        info = g.info()
        g.free()
        return tm, info

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    rec = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rec.append(step())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    info = rec[-1][1]
    m = int(info.m)
    ms_step = el / args.steps * 1e3
    value = m * args.steps / el
    phases = {k: float(np.mean([r[0].as_dict()[k] for r in rec])) for k in rec[0][0].as_dict()}
    count_ms = phases["run_count_ms"]
    run_ms = phases["run_zero_ms"] + count_ms + phases["run_epilogue_ms"]
    alg = count_bytes(info)
    achieved = alg / (count_ms * 1e-3) / 1e9
    traffic = stored_traffic()
    ctx.set_profiling(False)
    log("[bench] tc_lcc_run on the resident graph")
    run_res = run_timing(ctx, torch, n, src, dst, w["offset_bytes"], tri, lcc)
    triangles = int(tri.sum()) // 3
    log("[bench] streaming copy (achievable HBM bandwidth)")
    copy = hbm_copy_rate(torch, pkg)
    build_ms = sum(v for k, v in phases.items() if k.startswith("build"))
    bb = build_bytes(info, len(s))

    out = {
        "metric": METRIC, "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64+f64", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "raw_pairs": int(len(s)), "m_undirected": m,
                   "offset_bytes": int(info.offset_bytes), "step": "build+count+lcc from raw pairs in HBM",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_count (intersection + scatter)", "alg_bytes_per_launch": alg,
                     "avg_launch_ms": count_ms,
                     "achievable_gbs": copy["gbs"], "frac_of_achievable": achieved / copy["gbs"],
                     "dram_frac": (traffic / (count_ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None,
                     "full_list_alg_frac": full_list_bytes(info) / (count_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "full_list_note": "the whole-list streaming figure 4W + (4+2w)m + (2w+16)n prices work "
                                       "(every head's full N+ per oriented edge) that the wedge-pull kernel "
                                       "does not do; above 1 here, so it is not a fraction of anything"},
        "build_roofline": {"bound": "hbm", "least_bytes": bb, "ms": build_ms,
                           "achieved": bb / (build_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": bb / (build_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                           "bytes_note": "8 B per raw pair read + the built graph's device bytes written"},
        "hbm_copy": copy,
        "run_only_teps": m / (run_ms * 1e-3),
        "phases_ms": phases,
        "run_resident": run_res,
        "graph": {"wedges": int(info.wedges), "kept_in_edges": int(info.kept_in_edges),
                  "active_vertices": int(info.active_vertices), "block_vertices": int(info.block_vertices),
                  "staged_entries": int(info.staged_entries), "max_out_degree": int(info.max_out_degree),
                  "max_degree": int(info.max_degree), "device_bytes": int(info.device_bytes),
                  "count_grid": int(info.count_grid), "count_lds_bytes": int(info.count_lds_bytes),
                  "count_blocks_per_cu": int(info.count_blocks_per_cu), "table_slots": int(info.table_slots),
                  "triangles": triangles},
    }
    if not args.no_ext:
        log("[bench] per-edge counts and directed Eq. 1 on the same workload")
        out["ext"] = ext_bench(ctx, torch, pkg, n, src, dst, w["offset_bytes"], triangles)
    if not args.no_strategies:
        log("[bench] probe strategies on the resident graph")
        ctx.set_profiling(True)
        out["probe_strategies"] = strategy_timing(ctx, torch, pkg, n, src, dst, w["offset_bytes"], tri)
    if args.streamed_scale:
        out["streamed"] = streamed_bench(ctx, torch, pkg, log, args.streamed_scale)
    if not args.no_batch:
        ctx.set_profiling(False)
        out["batch"] = batch_bench(ctx, torch, pkg, log, autotune=not args.no_autotune)
    if not args.no_serve:
        ctx.set_profiling(False)
        out["serve"] = serve_bench(ctx, torch, log)
    ctx.close()
    if args.calibrate_copy:
        # the library's streaming copy (tc_lcc_hbm_copy): reads 1 GiB and writes 1 GiB through the
        # shader cores (copy_ itself may use the DMA engines, which the counters do not see)
        a = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            pkg.hbm_copy(a, b)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = a.numel() * 4
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cb = cpu_baseline(n, s, d, args.cpu_seconds)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "runs_edges_per_s")}
        out["cpu_baseline"]["host"] = host_cpu()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
