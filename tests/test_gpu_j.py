"""Angle-integrated trace (mean intensity J and the diagonal operator psi) on the 2D 64^2 static scene.

J = sum_d w_d I_d and psi = sum_d w_d (1 - exp(-tau of the first segment)) are checked
  - against the same sums of rt_trace's per-direction output (summation order only),
  - against the FP64 oracle on the same adapted cells (the oracle's march and segment lists),
  - chunked (work buffer, fixed-order reduction) vs one chunk, and run-to-run determinism.
"""
import numpy as np
import pytest

import oracle as orc
from synth import make_cfg1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_08498_amd as rt
    rt.lib()
    return rt


@pytest.fixture(scope="module")
def setup(rt):
    import torch
    sc = make_cfg1()
    scene = rt.Scene.from_dict(sc)
    scene.build(0, 8, iod_threshold=1e-2)
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    w = np.linspace(0.5, 1.5, 8).astype(np.float32)
    w /= w.sum()
    return sc, scene, dirs, w


def test_j_equals_weighted_sum_of_traces(rt, setup):
    import torch
    sc, scene, dirs, w = setup
    I = scene.trace(dirs, mode="vlm").double()  # [dir][lam][probe]
    Jref = (torch.from_numpy(w).double().cuda()[:, None, None] * I).sum(0)
    for chunked in (False, True):
        J, psi = scene.trace_j(dirs, weights=w, mode="vlm", chunked=chunked)
        torch.cuda.synchronize()
        rel = ((J.double() - Jref).abs() / Jref.abs().clamp_min(1e-30)).max().item()
        assert rel < 2e-6, (chunked, rel)
        assert torch.all(psi >= 0) and torch.all(psi <= 1)


def test_j_deterministic_and_chunked_matches_single(rt, setup):
    import torch
    sc, scene, dirs, w = setup
    J1, p1 = scene.trace_j(dirs, weights=w, chunked=True)
    J2, p2 = scene.trace_j(dirs, weights=w, chunked=True)
    J3, p3 = scene.trace_j(dirs, weights=w, chunked=False)
    torch.cuda.synchronize()
    assert torch.equal(J1, J2) and torch.equal(p1, p2)
    assert torch.allclose(J1, J3, rtol=2e-6, atol=0) and torch.allclose(p1, p3, rtol=2e-6, atol=1e-9)


def test_j_and_psi_against_oracle(rt, setup):
    import torch
    sc, scene, dirs, w = setup
    s = orc.Scene(sc)
    lvs, st_e, st_c = orc.static_level_values(s, sc["eta"][0:8], sc["chi"][0:8], sc["block_active"], T=1e-2)
    lv = orc.batch_levels(lvs)
    s.set_static_levels(st_e, st_c)
    assert np.array_equal(scene.levels(), lv)
    probes = scene.probe_voxels()
    rng = np.random.default_rng(3)
    pick = np.sort(rng.choice(probes.size, 300, replace=False))
    J, psi = scene.trace_j(dirs, weights=w, probes=torch.from_numpy(probes[pick]).cuda())
    J, psi = J.cpu().numpy(), psi.cpu().numpy()
    nd = sc["dirs"].shape[0]
    vox = np.repeat(probes[pick], nd)
    d = np.tile(np.arange(nd, dtype=np.int32), pick.size)
    I = orc.march(s, orc.STATIC, lv, vox, d).reshape(pick.size, nd, 8)  # [probe][dir][lam]
    Jref = np.einsum("d,pdl->lp", w.astype(np.float64), I)
    assert np.max(np.abs(J - Jref) / np.abs(Jref)) < 2e-5
    # psi: first segment of each ray (oracle segment list) with the oracle's stored level value of chi
    tot = s.level_total
    offs = np.cumsum([0] + [(64 >> m) ** 2 for m in range(4)])
    psi_ref = np.zeros((8, pick.size))
    for i, pv in enumerate(probes[pick]):
        for di in range(nd):
            cells, lvl, t_in, t_out = orc.ray_segments(s, lv, (int(pv) % 64, int(pv) // 64), sc["dirs"][di])
            m = int(lvl[0])
            cx, cy = cells[0, 0] >> m, cells[0, 1] >> m
            chi = np.array([st_c[l][offs[m] + cx + (64 >> m) * cy] for l in range(8)])
            psi_ref[:, i] += w[di] * -np.expm1(-chi * (t_out[0] - t_in[0]) * sc["ds0"])
    assert st_c[0].size == tot
    assert np.max(np.abs(psi - psi_ref)) < 1e-5
