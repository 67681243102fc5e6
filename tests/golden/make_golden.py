"""Write the stored oracle summaries under tests/golden/ (calls only oracle/ and synth/).

Run from the repository root:  python tests/golden/make_golden.py [case ...]
With no arguments every case is written.  Each fixture pins the generator and the oracle
together: if either changes, the stored digest no longer matches and the change has to be
justified.

Single graphs store the full-vector digests of t (uint64 little-endian) and LCC (binary64
little-endian) plus a few leading values; graph lists (the 4096-graph batch, the serving
pool) store one line per graph with its size, triangle total and the digest of its t and
LCC vectors, so that a mismatch names the graph.
"""
import hashlib
import json
import os
import sys
import multiprocessing

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

SINGLE = {
    "er4096_seed1": lambda: synth.er_4096(seed=1),
    "rmat_s12_ef16_seed1": lambda: synth.rmat_scale(12, 16, seed=1),
    "rmat_s16_ef16_seed1": lambda: synth.rmat_scale(16, 16, seed=1),
    "rmat_s20_ef16_seed1": lambda: synth.rmat_scale(20, 16, seed=1),
    "rmat_s23_ef16_seed1": lambda: synth.rmat_scale(23, 16, seed=1),
    # 13 parts of 200, 5 % of the cross pairs dropped, R-MAT S11 periphery: |N+(v)| just above
    # 2048 for the lowest-ranked core vertices, and most probes of a core list miss
    "dense_core_13x200_drop5_p11_seed61": lambda: synth.dense_core(13, 200, 0.05, 11, 61),
}

LISTS = {
    # the many-small-graphs batch: synth.batch_specs() (4096 graphs, list seed 7)
    "batch4096_seed7": lambda: synth.batch_specs(),
    # the serving pool: synth.serving_specs() (64 R-MAT EF16 graphs, n in [2^10, 2^21])
    "serving64_seed9": lambda: synth.serving_specs(count=64, seed=9),
}


def vector_digest(t, lcc) -> str:
    """sha256 over t (u64 LE) followed by LCC (f64 LE)."""
    return hashlib.sha256(t.astype("<u8").tobytes() + lcc.astype("<f8").tobytes()).hexdigest()


def summary(n, s, d):
    g = oracle.csr(n, s, d)
    t = oracle.tc_forward(g)
    lcc = oracle.lcc(g, t)
    return {
        "n": int(n),
        "raw_pairs": int(len(s)),
        "m_undirected": int(g.m),
        "max_degree": int(g.deg.max()),
        "triangles": int(t.sum()) // 3,
        "t_head": [int(x) for x in t[:16]],
        "lcc_head": [float(x).hex() for x in lcc[:16]],
        "sha256_t_u64le": hashlib.sha256(t.astype("<u8").tobytes()).hexdigest(),
        "sha256_lcc_f64le": hashlib.sha256(lcc.astype("<f8").tobytes()).hexdigest(),
        "sha256_csr": hashlib.sha256(g.off.astype("<i8").tobytes() + g.adj.astype("<i4").tobytes()).hexdigest(),
    }


def graph_line(spec):
    n, s, d = synth.make(tuple(spec))
    g = oracle.csr(n, s, d)
    t = oracle.tc_forward(g)
    lcc = oracle.lcc(g, t)
    return f"{int(g.m)} {int(t.sum()) // 3} {vector_digest(t, lcc)[:16]}"


def write(name, out):
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        if "graphs" in out:  # one graph per line
            head = {k: v for k, v in out.items() if k != "graphs"}
            f.write(json.dumps(head)[:-1] + ', "graphs": [\n')
            f.write(",\n".join(json.dumps(x) for x in out["graphs"]))
            f.write("\n]}\n")
        else:
            json.dump(out, f, indent=1)
            f.write("\n")


def main(names):
    for name in names:
        if name in SINGLE:
            out = summary(*SINGLE[name]())
            write(name, out)
            print(name, out["m_undirected"], out["triangles"], flush=True)
        elif name in LISTS:
            specs = LISTS[name]()
            # spawned workers: a forked child of a process whose OpenMP runtime already started
            # (the generator uses it) can hang in its first parallel region
            with multiprocessing.get_context("spawn").Pool(min(8, os.cpu_count() or 1)) as p:
                lines = p.map(graph_line, specs, chunksize=1)
            whole = hashlib.sha256("\n".join(lines).encode()).hexdigest()
            write(name, {"per_graph": "m_undirected triangles sha256(t u64 LE || LCC f64 LE)[:16], "
                                      "one string per graph in list order",
                         "sha256_of_lines": whole, "graphs": lines})
            print(name, len(lines), sum(int(x.split()[1]) for x in lines), flush=True)
        else:
            raise SystemExit(f"unknown case {name}")


if __name__ == "__main__":
    main(sys.argv[1:] or list(SINGLE) + list(LISTS))
