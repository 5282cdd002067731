"""Batched persistent launch: many scenes of uneven size in one launch.

Per-scene outputs of the persistent work-stealing kernel must equal the
single-scene launches bit for bit, every 64-probe tile must be claimed
exactly once, other launch shapes must give the same bits, graph replays
must match the eager result, and the autotuner must return a valid shape.
The kernels the batched workload runs (line model evaluated at rest and
stored as static emission, BF16 storage, 2D and 3D, path-graded levels) are
checked against the FP64 oracle on the same adapted cells, with the BF16
rounding of the stored level values emulated on the oracle's side.
"""
import numpy as np
import pytest

import oracle as orc
from oracle.nrc import bf16_round
from synth import cfg4_specs, make_cfg4_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_08498_amd as rt
    rt.lib()
    return rt


def small_specs():
    """Uneven 2D and 3D scenes with the cfg4 recipe, sized for a test."""
    specs = []
    for i, (N, dim, B, L, nd, nl) in enumerate([(64, 2, 16, 3, 16, 16), (128, 2, 16, 5, 32, 16), (64, 2, 16, 2, 64, 16),
                                                 (32, 3, 8, 3, 16, 16), (48, 3, 8, 4, 32, 16), (64, 3, 8, 2, 16, 16)]):
        specs.append(dict(index=i, seed=4100 + i, N=N, dim=dim, brick=B, n_levels=L, n_dir=nd, n_lam=nl))
    return specs


@pytest.fixture(scope="module")
def scenes(rt):
    import torch
    out = []
    for sp in small_specs():
        sc = make_cfg4_scene(sp)
        s = rt.Scene.from_dict(sc, emission="static")
        s.build(0, 8, iod_threshold=1e-2, storage="bf16")
        dirs = torch.from_numpy(sc["dirs"]).cuda()
        out.append((sc, s, dirs))
    return out


def eager(scenes, level_dist=None, grade="entry"):
    return [s.trace(d, mode="vlm", level_dist=level_dist, grade=grade).clone() for _, s, d in scenes]


def jobs_for(scenes, outs, level_dist=None, grade="entry"):
    return [dict(scene=s, dirs=d, out=o, mode="vlm", level_dist=level_dist, grade=grade)
            for (_, s, d), o in zip(scenes, outs)]


def test_batched_equals_single_scene_launches(rt, scenes):
    import torch
    ref = eager(scenes)
    outs = [torch.full_like(r, float("nan")) for r in ref]
    b0 = rt.Batch(jobs_for(scenes, outs))
    claims = torch.zeros(b0.tiles(), dtype=torch.int32, device="cuda")
    b = rt.Batch(jobs_for(scenes, outs), claims=claims)
    b.run()
    torch.cuda.synchronize()
    for r, o in zip(ref, outs):
        assert torch.equal(r, o)
    c = claims.cpu().numpy()
    assert c.size == sum(d.shape[0] * ((s.info["n_probes"] + 63) // 64) for _, s, d in scenes)
    assert np.all(c == 1)
    assert b.device_error() == (0, -1)


def test_batched_path_grading_equals_single_scene_launches(rt, scenes):
    """The cap taken along the path (cascade intervals' rule) in the persistent kernel: the same bits as the
    single-scene launches, and different from block-entry grading on these scenes."""
    import torch
    ref = eager(scenes, rt.CASCADE_LEVEL_DIST, "path")
    outs = [torch.full_like(r, float("nan")) for r in ref]
    b = rt.Batch(jobs_for(scenes, outs, rt.CASCADE_LEVEL_DIST, "path"))
    b.run()
    torch.cuda.synchronize()
    for r, o in zip(ref, outs):
        assert torch.equal(r, o)
    entry = eager(scenes, rt.CASCADE_LEVEL_DIST, "entry")
    assert any(not torch.equal(r, e) for r, e in zip(ref, entry))
    assert b.device_error() == (0, -1)


@pytest.mark.parametrize("shape", [dict(wg_waves=1, wgs_per_cu=1, tiles_per_pop=1, order=1),
                                   dict(wg_waves=8, wgs_per_cu=4, tiles_per_pop=4, order=0),
                                   dict(wg_waves=2, wgs_per_cu=16, tiles_per_pop=64, order=0),
                                   dict(wg_waves=4, wgs_per_cu=2, tiles_per_pop=1, order=0, tile_shape="cubes"),
                                   dict(wg_waves=8, wgs_per_cu=4, tiles_per_pop=4, order=1, tile_shape="cubes")])
def test_launch_shapes_give_identical_bits(rt, scenes, shape):
    import torch
    ref = eager(scenes, rt.CASCADE_LEVEL_DIST)
    outs = [torch.zeros_like(r) for r in ref]
    claims = torch.zeros(sum(d.shape[0] * ((s.info["n_probes"] + 63) // 64) for _, s, d in scenes),
                         dtype=torch.int32, device="cuda")
    b = rt.Batch(jobs_for(scenes, outs, rt.CASCADE_LEVEL_DIST), claims=claims, **shape)
    b.run()
    b.run()  # the queue resets on every run
    torch.cuda.synchronize()
    for r, o in zip(ref, outs):
        assert torch.equal(r, o)
    assert np.all(claims.cpu().numpy() == 2)


def test_graph_replays_match_eager(rt, scenes):
    """Build of two wavelength batches + batched trace captured once, replayed
    three times with eager work in between; every replay matches."""
    import torch
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        outs = {b: [torch.zeros((d.shape[0], 8, s.info["n_probes"]), device="cuda") for _, s, d in scenes]
                for b in (0, 1)}
        batches = {b: rt.Batch(jobs_for(scenes, outs[b]), stream=stream) for b in (0, 1)}
        # eager reference
        ref = {}
        for b in (0, 1):
            for _, s, _ in scenes:
                s.build(8 * b, 8 * b + 8, iod_threshold=1e-2, storage="bf16", stream=stream)
            batches[b].run(stream)
            ref[b] = [o.clone() for o in outs[b]]
        stream.synchronize()
        with rt.Graph(stream) as g:
            for b in (0, 1):
                for _, s, _ in scenes:
                    s.build(8 * b, 8 * b + 8, iod_threshold=1e-2, storage="bf16", stream=stream)
                batches[b].run(stream)
        for rep in range(3):
            for b in (0, 1):
                for o in outs[b]:
                    o.fill_(-1.0)
            stream.synchronize()
            g.replay()
            stream.synchronize()
            for b in (0, 1):
                for r, o in zip(ref[b], outs[b]):
                    assert torch.equal(r, o), (rep, b)
            # eager work between replays
            _ = torch.ones(1024, device="cuda").sum().item()
    torch.cuda.synchronize()


def test_autotune_returns_a_valid_shape(rt, scenes):
    import torch
    outs = [torch.zeros((d.shape[0], 8, s.info["n_probes"]), device="cuda") for _, s, d in scenes]
    best, ms = rt.batch_autotune(jobs_for(scenes, outs), reps=2)
    assert best["wg_waves"] in (2, 4, 8) and best["wgs_per_cu"] in (1, 2, 4) and best["tiles_per_pop"] in (1, 4)
    assert best["tile_shape"] in ("rows", "cubes")
    assert ms > 0


def test_cfg4_specs_shapes():
    specs = cfg4_specs()
    assert len(specs) == 48
    assert sum(s["dim"] == 2 for s in specs) == 24
    assert all(64 <= s["N"] <= 1024 for s in specs if s["dim"] == 2)
    assert all(64 <= s["N"] <= 192 for s in specs if s["dim"] == 3)


def oracle_static_bf16(sc, lam_idx, T, lv_gpu):
    """Oracle side of a line-model scene stored as static emission in BF16: MIP-0 values at rest (FP64), the
    level chain and per-wavelength levels (their batch minimum must equal the device's map: Gaussian lines,
    FP64 statistics in the same order), then the stored level values rounded as the device stores them
    (FP64 -> FP32 -> BF16, ties to even)."""
    s = orc.Scene(sc, lam_idx=lam_idx)
    E = np.zeros((len(lam_idx), s.nvox))
    C = np.zeros_like(E)
    for il in range(len(lam_idx)):
        E[il], C[il] = orc.lines_mip0(s, il, 0)
    lvs, st_e, st_c = orc.static_level_values(s, E, C, sc["block_active"], T)
    lv = orc.batch_levels(lvs)
    assert np.array_equal(lv, lv_gpu), "level maps differ: blocks %s" % np.nonzero(lv != lv_gpu)[0][:8]
    s.set_static_levels(bf16_round(st_e), bf16_round(st_c))
    return s, lv


@pytest.mark.parametrize("batch", [0, 1])
def test_batched_workload_kernels_match_oracle(rt, scenes, batch):
    """Every scene of the small uneven batch (2D and 3D, 2-5 levels), path-graded VLM, BF16 storage: the
    persistent launch gives the single-scene bits, and both match the FP64 oracle marching the same levels and
    the same BF16-rounded values to FP32 accumulation (relative error < 2e-5 on sampled rays)."""
    import torch
    T = 1e-2
    for _, s, _ in scenes:
        s.build(8 * batch, 8 * batch + 8, iod_threshold=T, storage="bf16")
    ref = eager(scenes, rt.CASCADE_LEVEL_DIST, "path")
    outs = [torch.full_like(r, float("nan")) for r in ref]
    b = rt.Batch(jobs_for(scenes, outs, rt.CASCADE_LEVEL_DIST, "path"))
    b.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(41 + batch)
    for (sc, s, d), r, o in zip(scenes, ref, outs):
        assert torch.equal(r, o)
        print("scene %s: %dD N=%d L=%d" % (sc["name"], sc["dim"], sc["n"][0], sc["n_levels"]), flush=True)
        os_, lv = oracle_static_bf16(sc, list(range(8 * batch, 8 * batch + 8)), T, s.levels())
        os_.set_level_dist(rt.CASCADE_LEVEL_DIST, "path")
        probes = s.probe_voxels()
        k = rng.choice(probes.size, min(512, probes.size), replace=False)
        dd = rng.integers(0, d.shape[0], k.size).astype(np.int32)
        want = orc.march(os_, orc.STATIC, lv, probes[k], dd)
        got = o.cpu().numpy()[dd, :, k]
        st = orc.rel_err_stats(got, want)
        assert st["n_ref_zero_mismatch"] == 0 and st["p100"] < 2e-5, (sc["name"], st)
    for _, s, _ in scenes:  # leave the module's scenes on batch 0 as the fixture built them
        s.build(0, 8, iod_threshold=T, storage="bf16")
