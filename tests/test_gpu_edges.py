"""GPU edge cases: a scene with no active block, empty probe lists, probes inside empty blocks, probe
indices outside the grid.

Rays through empty space carry the boundary intensity unchanged (the recurrence of
Eq. RteIntegral with eta = chi = 0), so these cases have exact answers.
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


def _dirs2(n, seed):
    rng = np.random.default_rng(seed)
    th = rng.uniform(0, 2 * np.pi, n)
    return np.stack([np.cos(th), np.sin(th)], 1).astype(np.float32)


def test_scene_without_active_blocks(rt):
    import torch
    n = 32
    zeros = np.zeros((2, n * n), np.float32)
    sc = dict(dim=2, n=(n, n, 1), brick=8, n_levels=3, model="static", eta=zeros, chi=zeros, ds0=1.0)
    scene = rt.Scene.from_dict(sc)
    assert scene.info["n_active"] == 0 and scene.info["n_probes"] == 0
    scene.build(0, 2, iod_threshold=1e-2)
    assert np.all(scene.levels() == -1)
    dirs = torch.from_numpy(_dirs2(6, 1)).cuda()
    I = scene.trace(dirs, I0=0.6)
    assert tuple(I.shape) == (6, 2, 0)
    probes = np.arange(0, n * n, 37, dtype=np.int32)  # explicit probes anywhere in the (empty) grid
    for grade in ("entry", "path"):
        I = scene.trace(dirs, probes=probes, I0=0.6, level_dist=rt.CASCADE_LEVEL_DIST, grade=grade).cpu().numpy()
        assert np.all(I == np.float32(0.6))
    Ii, Ti = scene.trace_interval(dirs, 2.0, 9.0, probes=probes, I0=0.6)
    assert torch.all(Ti == 1).item()
    # I0 only where the ray leaves the grid inside [2, 9]
    I_all, _ = scene.trace_interval(dirs, 0.0, np.inf, probes=probes, I0=0.6)
    assert torch.all(I_all == np.float32(0.6)).item()
    J, psi = scene.trace_j(dirs, probes=probes, I0=0.6)
    np.testing.assert_allclose(J.cpu().numpy(), 0.6, rtol=1e-6)
    assert torch.all(psi == 0).item()


def test_line_scene_without_active_blocks_reduced_precision(rt):
    """Core and Voigt with no active block: the BF16 copy of an empty parameter chain is a no-op."""
    import torch
    n = 16
    z = np.zeros((2, n * n), np.float32)
    sc = dict(dim=2, n=(n, n, 1), brick=8, n_levels=3, model="lines", profile="voigt", lam=np.array([500.0, 500.01]),
              lam0=np.array([500.0]), eta_star=z[:1], chi_star=z[:1], damp=z[:1], inv_dld=z[:1] + 10.0,
              eta_bg=z[0], chi_bg=z[0], vel=np.zeros((2, n * n), np.float32), dirs=_dirs2(4, 2),
              block_active=np.zeros(4, np.uint8), ds0=1.0, I0=0.0)
    scene = rt.Scene.from_dict(sc, emission="cav")
    assert scene.info["n_active"] == 0
    scene.build(0, 2, storage="bf16")
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    I = scene.trace(dirs, probes=np.array([0, 17, 255], np.int32), I0=0.25).cpu().numpy()
    assert np.all(I == np.float32(0.25))


def test_empty_probe_lists(rt):
    import torch
    sc = make_cfg1()
    scene = rt.Scene.from_dict(sc)
    scene.build(0, 8, iod_threshold=1e-2)
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    none = np.zeros(0, np.int32)
    assert tuple(scene.trace(dirs, probes=none).shape) == (8, 8, 0)
    I, T = scene.trace_interval(dirs, 1.5, 6.0, probes=none)
    assert tuple(I.shape) == (8, 8, 0) and tuple(T.shape) == (8, 8, 0)
    J, psi = scene.trace_j(dirs, probes=none)
    assert tuple(J.shape) == (8, 0)


def test_probe_indices_outside_the_grid(rt):
    """A probe index outside [0, nvox) is not traced: its outputs are NaN in every entry point, the valid
    probes of the same list are unaffected, and each bad index is counted once per call."""
    import torch
    sc = make_cfg1()
    scene = rt.Scene.from_dict(sc)
    scene.build(0, 8, iod_threshold=1e-2)
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    nvox = 64 * 64
    good = np.array([0, 77, 1000, nvox - 1], np.int32)
    bad = np.array([-1, nvox, 2 ** 31 - 1], np.int32)
    mixed = np.array([good[0], bad[0], good[1], bad[1], good[2], bad[2], good[3]], np.int32)
    isbad = np.isin(mixed, bad) & ~np.isin(mixed, good)
    scene.reset_device_error()
    I_ref = scene.trace(dirs, probes=good).cpu().numpy()
    assert scene.bad_probes() == 0
    I = scene.trace(dirs, probes=mixed).cpu().numpy()
    assert scene.bad_probes() == bad.size
    assert np.all(np.isnan(I[:, :, isbad])) and np.array_equal(I[:, :, ~isbad], I_ref)
    Iv, Tv = scene.trace_interval(dirs, 1.5, 6.0, probes=mixed)
    Iv_ref, Tv_ref = scene.trace_interval(dirs, 1.5, 6.0, probes=good)
    assert torch.all(torch.isnan(Iv[:, :, isbad])) and torch.all(torch.isnan(Tv[:, :, isbad]))
    assert torch.equal(Iv[:, :, ~isbad], Iv_ref) and torch.equal(Tv[:, :, ~isbad], Tv_ref)
    J, psi = scene.trace_j(dirs, probes=mixed)
    J_ref, psi_ref = scene.trace_j(dirs, probes=good)
    assert torch.all(torch.isnan(J[:, isbad])) and torch.equal(J[:, ~isbad], J_ref)
    assert torch.equal(psi[:, ~isbad], psi_ref)
    assert scene.bad_probes() == 3 * bad.size
    scene.reset_device_error()
    assert scene.bad_probes() == 0 and scene.device_error() == (0, -1)


def test_probes_inside_empty_blocks(rt):
    """Probe voxels in empty blocks: the ray starts in empty space; intensities against the oracle on the same
    cells, and I0 alone for rays that meet no active block."""
    import torch
    sc = make_cfg1()
    T = 1e-2
    scene = rt.Scene.from_dict(sc)
    scene.build(0, 8, iod_threshold=T)
    empty = np.nonzero(sc["block_active"] == 0)[0]
    rng = np.random.default_rng(4)
    vox = []
    for b in rng.choice(empty, 6, replace=False):
        bx, by = int(b) % 8, int(b) // 8
        for _ in range(20):
            vox.append((bx * 8 + int(rng.integers(0, 8))) + 64 * (by * 8 + int(rng.integers(0, 8))))
    vox = np.array(vox, np.int32)
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    I = scene.trace(dirs, probes=vox, I0=0.3).cpu().numpy()  # [dir][lam][probe]
    s = orc.Scene(sc)
    lvs, st_e, st_c = orc.static_level_values(s, sc["eta"][:8], sc["chi"][:8], sc["block_active"], T=T)
    lv = orc.batch_levels(lvs)
    assert np.array_equal(lv, scene.levels())
    s.set_static_levels(st_e, st_c)
    s.s.I0 = 0.3
    d = np.repeat(np.arange(8, dtype=np.int32), vox.size)
    ref = orc.march(s, orc.STATIC, lv, np.tile(vox, 8), d).reshape(8, vox.size, 8).transpose(0, 2, 1)
    st = orc.rel_err_stats(I, ref)
    assert st["n_ref_zero_mismatch"] == 0 and st["p100"] < 2e-5, st
    assert np.any(I == np.float32(0.3))  # some rays cross only empty blocks


def test_invalid_inputs_rejected_at_create(rt):
    """Negative or non-finite emissivity / opacity / line parameters, and non-finite velocities, are rejected
    when the scene is created (a device pass over every input value)."""
    n = 32
    rng = np.random.default_rng(5)
    eta = rng.uniform(0.1, 1.0, (2, n * n)).astype(np.float32)
    chi = rng.uniform(0.1, 1.0, (2, n * n)).astype(np.float32)
    base = dict(dim=2, n=(n, n, 1), brick=8, n_levels=3, model="static", ds0=1.0)
    rt.Scene.from_dict(dict(base, eta=eta, chi=chi))  # valid
    for name, arr, idx, val in (("chi", chi, (0, 5), np.nan), ("chi", chi, (1, 9), np.inf),
                                ("eta", eta, (1, 7), -1e-3), ("eta", eta, (0, 0), -np.inf)):
        bad = arr.copy()
        bad[idx] = val
        kw = dict(eta=eta, chi=chi)
        kw[name] = bad
        with pytest.raises(RuntimeError, match="negative or non-finite"):
            rt.Scene.from_dict(dict(base, **kw))
    from test_gpu_lines import cav_scene
    sc = cav_scene(n=16)
    rt.Scene.from_dict(sc, emission="cav")  # valid
    for key, val in (("damp", -0.1), ("vel", np.nan), ("inv_dld", np.inf), ("chi_bg", -1.0)):
        bad = dict(sc)
        arr = np.array(sc[key], np.float32, copy=True)
        arr.reshape(-1)[123] = val
        bad[key] = arr
        with pytest.raises(RuntimeError, match="negative or non-finite"):
            rt.Scene.from_dict(bad, emission="cav")
