"""A graph with more than 2^30 edges on 4-byte offsets: the tails that start at entry 2^30 of
adj or later have byte offsets above 32 bits, which the count kernel's tail pointer must keep.

The graph is 533,131 disjoint cliques K_64 (34,120,384 vertices, 1,074,792,096 edges, generated
on the GPU), so every vertex closes C(63, 2) = 1953 triangles and has LCC 1 (Eq. 2): a closed
form, checked on every vertex.  It needs about 60 GB of device memory at its peak.
"""
import math

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2202_13976_amd")


def say(msg):
    print(msg, flush=True)


def test_cliques_past_2_30_edges_on_4_byte_offsets():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    k = 64
    per = k * (k - 1) // 2
    cliques = -(-((1 << 30) + (1 << 20)) // per)  # a little past 2^30 edges
    n, m = cliques * k, cliques * per
    say(f"[gpu] {cliques} cliques K_{k}: n={n} m={m}, 4-byte offsets")
    dev = torch.device("cuda", 0)
    ctx = pkg.Context(0)
    try:
        iu = torch.triu_indices(k, k, 1, device=dev).to(torch.int32)
        base = torch.arange(cliques, device=dev, dtype=torch.int32) * k
        src = (iu[0].view(1, -1) + base.view(-1, 1)).view(-1)
        dst = (iu[1].view(1, -1) + base.view(-1, 1)).view(-1)
        del iu, base
        assert src.numel() == m and int(dst.max()) == n - 1
        g = ctx.build_csr(n, src, dst, offset_bytes=4)
        del src, dst
        torch.cuda.empty_cache()
        info = g.info()
        assert info.m == m and info.offset_bytes == 4 and info.max_out_degree == k - 1
        tri, lcc = g.run()
        torch.cuda.synchronize()
        g.free()
        want = math.comb(k - 1, 2)
        assert bool(torch.all(tri == want)), "a vertex does not close C(63, 2) triangles"
        assert bool(torch.all(lcc == 1.0)), "a vertex's LCC is not 1"
        del tri, lcc
    finally:
        ctx.close()
        torch.cuda.empty_cache()
