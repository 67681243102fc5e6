"""Write the stored oracle summaries under tests/golden/ (calls only oracle/ and synth/).

Run from the repository root:  python tests/golden/make_golden.py
Each fixture pins the generator and the oracle together: if either changes, the
stored digest no longer matches and the change has to be justified.
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

CASES = {
    "er4096_seed1": lambda: synth.er_4096(seed=1),
    "rmat_s12_ef16_seed1": lambda: synth.rmat_scale(12, 16, seed=1),
    "rmat_s16_ef16_seed1": lambda: synth.rmat_scale(16, 16, seed=1),
}


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


def main():
    for name, fn in CASES.items():
        out = summary(*fn())
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")
        print(name, out["m_undirected"], out["triangles"])


if __name__ == "__main__":
    main()
