"""Autotuner and tuning validation: the tuner's candidates never change results, its choice is
one of its candidates, it can be saved and loaded again, and bad settings are refused."""
import json
import os
import tempfile

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2202_13976_amd")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pkg.Context(0)
    yield c
    import gc
    gc.collect()
    c.close()


@pytest.fixture(scope="module")
def graphs(ctx):
    specs = synth.batch_specs(count=24, seed=17)
    raw = [synth.make(sp) for sp in specs] + [synth.rmat_scale(14, 16, seed=8)]
    gs = [ctx.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(), offset_bytes=4)
          for n, s, d in raw]
    yield raw, gs
    for g in gs:
        g.free()


def expect(raw):
    return [oracle.tc_lcc(n, s, d) for n, s, d in raw]


def test_autotune_picks_a_candidate_and_keeps_results(ctx, graphs):
    print("[gpu] autotune single + batch", flush=True)
    raw, gs = graphs
    refs = expect(raw)
    default = ctx.tuning().as_dict()
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "tuning.json")
        t = ctx.autotune(gs, what=3, reps=2, path=path)
        assert t.probe in (pkg.PROBE_AUTO, pkg.PROBE_HASH, pkg.PROBE_MERGE)
        assert t.wave_work_max in (1024, 2048, 4096, 8192, 16384)
        assert t.batch_grab in (1, 4, 8, 16)
        assert t.batch_heavy_bits in (12, 13, 14, 15, 16, 18)
        assert ctx.tuning().as_dict() == t.as_dict()
        rec = json.load(open(path))
        assert rec["tuning"]["wave_work_max"] == t.wave_work_max and rec["device"]
        # exact results under the installed setting, single and batched
        for g, (t_ref, l_ref) in zip(gs, refs):
            tri, lcc = g.run()
            np.testing.assert_array_equal(tri.cpu().numpy().astype(np.uint64), t_ref)
            assert lcc.cpu().numpy().tobytes() == l_ref.tobytes()
        tris = [torch.empty(g.n, dtype=torch.int64, device="cuda") for g in gs]
        lccs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for g in gs]
        assert ctx.batch_poll(ctx.batch_submit(gs, tris, lccs), block=True)[0]
        for tri, lcc, (t_ref, l_ref) in zip(tris, lccs, refs):
            np.testing.assert_array_equal(tri.cpu().numpy().astype(np.uint64), t_ref)
            assert lcc.cpu().numpy().tobytes() == l_ref.tobytes()
        # saved and loaded again
        ctx.set_tuning(**default)
        ctx.load_tuning(path)
        assert ctx.tuning().as_dict() == t.as_dict()
    ctx.set_tuning(**default)


def test_autotune_batch_only(ctx, graphs):
    print("[gpu] autotune batch knobs only", flush=True)
    _, gs = graphs
    default = ctx.tuning().as_dict()
    t = ctx.autotune(gs, what=2, reps=1)
    assert t.wave_work_max == default["wave_work_max"] and t.probe == default["probe"]
    ctx.set_tuning(**default)


def test_tuning_validation_and_load_errors(ctx, graphs):
    raw, gs = graphs
    default = ctx.tuning().as_dict()
    for bad, status in [(dict(probe=5), pkg.INVALID_ARGUMENT), (dict(merge_ratio_x100=-1), pkg.INVALID_ARGUMENT),
                        (dict(merge_ratio_x100=100001), pkg.INVALID_ARGUMENT),
                        (dict(row_sort_max=4097), pkg.INVALID_ARGUMENT), (dict(row_sort_max=-1), pkg.INVALID_ARGUMENT),
                        (dict(batch_grab=65), pkg.INVALID_ARGUMENT), (dict(batch_heavy_bits=41), pkg.INVALID_ARGUMENT),
                        (dict(block_threads=512), pkg.INVALID_ARGUMENT), (dict(wave_outdeg_max=-1), pkg.INVALID_ARGUMENT),
                        (dict(group=3), pkg.INVALID_ARGUMENT)]:
        with pytest.raises(pkg.TcLccError) as e:
            ctx.set_tuning(**bad)
        assert e.value.status == status, bad
    assert ctx.tuning().as_dict() == default
    with pytest.raises(pkg.TcLccError) as e:
        ctx.autotune(gs, what=4)
    assert e.value.status == pkg.INVALID_ARGUMENT
    with tempfile.TemporaryDirectory() as tmp:
        other = os.path.join(tmp, "other.json")
        with open(other, "w") as f:
            json.dump({"device": "some other device", "tuning": {"probe": 0, "group": 0, "wave_work_max": 4096,
                                                                  "wave_outdeg_max": 0, "block_threads": 256,
                                                                  "batch_grab": 8, "batch_heavy_bits": 15}}, f)
        with pytest.raises(pkg.TcLccError) as e:
            ctx.load_tuning(other)
        assert e.value.status == pkg.UNSUPPORTED
        broken = os.path.join(tmp, "broken.json")
        with open(broken, "w") as f:
            f.write("{}")
        with pytest.raises(pkg.TcLccError) as e:
            ctx.load_tuning(broken)
        assert e.value.status == pkg.INVALID_ARGUMENT
        with pytest.raises(pkg.TcLccError) as e:
            ctx.load_tuning(os.path.join(tmp, "missing.json"))
        assert e.value.status == pkg.INVALID_ARGUMENT


@pytest.mark.parametrize("outdeg", [1, 8, 40])
def test_wave_outdeg_limit_keeps_results(ctx, graphs, outdeg):
    raw, gs = graphs
    default = ctx.tuning().as_dict()
    ctx.set_tuning(wave_outdeg_max=outdeg)
    try:
        n, s, d = raw[-1]
        t_ref, l_ref = oracle.tc_lcc(n, s, d)
        tri, lcc = gs[-1].run()
        np.testing.assert_array_equal(tri.cpu().numpy().astype(np.uint64), t_ref)
        assert lcc.cpu().numpy().tobytes() == l_ref.tobytes()
    finally:
        ctx.set_tuning(**default)
