"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/oracle_sanitized_main.c includes oracle.c and runs every routine on the graphs written
here (generated inputs, degenerate ones, repeats, loops, both directions); any out-of-bounds
access or undefined behaviour aborts the run.  Its per-graph summary lines must equal what the
normal build gives through ctypes, so the sanitized build computes the same results.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def cases():
    out = []
    for n, pairs in [(1, []), (5, []), (4, [(0, 0), (1, 1)]), (3, [(0, 1), (1, 2), (2, 0), (0, 1), (1, 0)]),
                     (40, [(a, b) for a in range(40) for b in range(a + 1, 40)])]:
        a = np.array(pairs, dtype=np.int32).reshape(-1, 2)
        out.append((n, a[:, 0].copy(), a[:, 1].copy()))
    out.append(synth.er_4096(seed=4))
    for scale in (8, 10, 11):
        out.append(synth.rmat_scale(scale, 16, seed=scale))
    n, s, d = synth.rmat_scale(9, 8, seed=3)
    out.append((n, np.concatenate([s, d, s]), np.concatenate([d, s, s])))  # repeats, both ways, loops
    out.append(synth.dense_core(5, 30, 0.1, 6, 2))
    return out


def summary(n, s, d):
    g = oracle.csr(n, s, d)
    t = oracle.tc_forward(g)
    lcc = oracle.lcc(g, t)
    bits = lcc.view(np.uint64)
    lx = 0
    for v in range(n):
        lx ^= (int(bits[v]) + v * 0x9E3779B97F4A7C15) & (2**64 - 1)
    _, _, c = oracle.edge_counts(g)
    gd = oracle.csr_directed(n, s, d)
    num = oracle.tc_directed(gd)
    return f"{n} {g.m} {int(t.sum())} {lx} {int(c.sum())} {len(gd.adj)} {int(num.sum())}"


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           os.path.join(HERE, "oracle_sanitized_main.c"), "-o", exe, "-lm"])
    blob = bytearray()
    want = []
    for n, s, d in cases():
        s = np.ascontiguousarray(s, dtype=np.int32)
        d = np.ascontiguousarray(d, dtype=np.int32)
        blob += struct.pack("<qq", n, len(s)) + s.astype("<i4").tobytes() + d.astype("<i4").tobytes()
        want.append(summary(n, s, d))
    # the environment is left as it is; ASan is told not to insist on coming first among the
    # loaded libraries, since the process may have others preloaded
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], input=bytes(blob), capture_output=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr.decode(errors="replace")[-4000:]
    assert r.stdout.decode().split("\n")[:-1] == want
