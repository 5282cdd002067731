"""Prefiltered merged cells (Sect. 5.1) on the GPU against the FP64 oracle.

The device builds, for every merged cell and signed axis, the homogeneous cell with the same row-averaged transfer
as the cell's MIP-0 voxels, and a ray blends the axes it propagates along with weights w_a^2.  Checked on the same
level map and the same cells as the oracle's PREFILTER march:
  * 2D static scene (cfg1 recipe, IoD threshold 1), VLM and cascade-graded VLM, FP32 storage: relative error
    < 2e-5;
  * 3D and 2D line-model scenes stored at rest (the batched workload's recipe), path-graded, FP32 and BF16
    storage (the oracle rounds its FP64 values as the device stores them);
  * at MIP 0 the prefiltered scene traces the static scene's bits.
"""
import numpy as np
import pytest

import oracle as orc
from oracle.nrc import bf16_round
from synth import make_cfg1, make_cfg4_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_08498_amd as rt
    rt.lib()
    return rt


def oracle_prefilter(sc, eta, chi, T, lv_gpu, storage):
    """Oracle scene holding the static level values and the prefiltered cells of [8][nvox] MIP-0 values, rounded as
    the device stores them; the oracle's level map must equal the device's."""
    s = orc.Scene(sc) if sc["model"] == "static" else orc.Scene(sc, lam_idx=list(range(8)))
    lvs, st_e, st_c = orc.static_level_values(s, eta, chi, sc["block_active"], T)
    lv = orc.batch_levels(lvs)
    assert np.array_equal(lv, lv_gpu), "level maps differ: blocks %s" % np.nonzero(lv != lv_gpu)[0][:8]
    pe, pc = orc.prefilter_values(s, eta, chi)
    rnd = bf16_round if storage == "bf16" else (lambda a: a.astype(np.float32).astype(np.float64))
    s.set_static_levels(rnd(st_e), rnd(st_c))
    s.set_prefilter(rnd(pe), rnd(pc))
    return s, lv


def sample_pairs(scene, n_dir, n, seed):
    rng = np.random.default_rng(seed)
    probes = scene.probe_voxels()
    k = rng.choice(probes.size, min(n, probes.size), replace=False)
    return probes, k, rng.integers(0, n_dir, k.size).astype(np.int32)


@pytest.mark.parametrize("graded", [False, True])
def test_static_2d_prefilter_matches_oracle(rt, graded):
    import torch
    sc = make_cfg1()
    T = 1.0  # the paper's deployment threshold (Sect. 4.1): most blocks merge
    scene = rt.Scene.from_dict(sc, emission="prefilter")
    scene.build(0, 8, iod_threshold=T)
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    ld = rt.CASCADE_LEVEL_DIST if graded else None
    I = scene.trace(dirs, mode="vlm", level_dist=ld, grade="path").cpu().numpy()
    s, lv = oracle_prefilter(sc, sc["eta"][:8].astype(np.float64), sc["chi"][:8].astype(np.float64), T,
                             scene.levels(), "f32")
    assert (lv > 0).sum() > 10, "the test needs merged blocks"
    s.set_level_dist(ld, "path")
    probes, k, d = sample_pairs(scene, 8, 2048, 1)
    want = orc.march(s, orc.PREFILTER, lv, probes[k], d)
    st = orc.rel_err_stats(I[d, :, k], want)
    assert st["n_ref_zero_mismatch"] == 0 and st["p100"] < 2e-5, st
    # the box-filtered march on the same levels differs (the prefiltered values are in use)
    box = orc.march(s, orc.STATIC, lv, probes[k], d)
    assert orc.rel_err_stats(box, want)["p99"] > 1e-4


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("spec", [dict(index=0, seed=4300, N=48, dim=3, brick=8, n_levels=4, n_dir=16, n_lam=8),
                                  dict(index=1, seed=4301, N=128, dim=2, brick=16, n_levels=5, n_dir=32, n_lam=8)])
def test_line_model_prefilter_matches_oracle(rt, spec, storage):
    import torch
    sc = make_cfg4_scene(spec)
    T = 1e-2
    print("prefilter parity: %dD N=%d L=%d %s" % (sc["dim"], spec["N"], spec["n_levels"], storage), flush=True)
    scene = rt.Scene.from_dict(sc, emission="prefilter")
    scene.build(0, 8, iod_threshold=T, storage=storage)
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    I = scene.trace(dirs, mode="vlm", level_dist=rt.CASCADE_LEVEL_DIST, grade="path").cpu().numpy()
    so = orc.Scene(sc, lam_idx=list(range(8)))
    E = np.zeros((8, so.nvox))
    C = np.zeros_like(E)
    for il in range(8):
        E[il], C[il] = orc.lines_mip0(so, il, 0)
    s, lv = oracle_prefilter(sc, E, C, T, scene.levels(), storage)
    assert (lv > 0).sum() > 4, "the test needs merged blocks"
    s.set_level_dist(rt.CASCADE_LEVEL_DIST, "path")
    probes, k, d = sample_pairs(scene, spec["n_dir"], 1024, 2)
    want = orc.march(s, orc.PREFILTER, lv, probes[k], d)
    st = orc.rel_err_stats(I[d, :, k], want)
    assert st["n_ref_zero_mismatch"] == 0 and st["p100"] < 2e-5, st


def test_prefilter_at_mip0_is_the_static_march(rt):
    import torch
    sc = make_cfg1()
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    a = rt.Scene.from_dict(sc, emission="prefilter")
    b = rt.Scene.from_dict(sc)
    for s in (a, b):
        s.build(0, 8, iod_threshold=1e-2)
    assert torch.equal(a.trace(dirs, mode="level0"), b.trace(dirs, mode="level0"))
    assert a.info["storage_bytes"] == rt.scene_workspace_bytes(sc, emission="prefilter")
    assert a.info["storage_bytes"] > b.info["storage_bytes"]
