"""GPU parity of the moving-medium line models against the FP64 oracle.

Velocity interpolation (2D, Gaussian lines + continuum, cfg2 recipe at 128^2)
and Core and Voigt (3D 32^3, two Voigt lines): block levels (exact outside
the threshold tie band; the oracle then marches the device's level map), intensities on the same adapted
cells, both velocity-node grid modes, level-0
equivalence with the Classic march, BF16/FP16 storage of velocity nodes and
line parameters within their rounding bounds, and the approximation error
against the dense Classic march (reported).
"""
import math

import numpy as np
import pytest

import oracle as orc
from synth import C_KMS, directions_fibonacci, grf, make_cfg2

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
def vscene():
    return make_cfg2(seed=21, n=128, B=16, n_lam_per_line=8, n_dir=8)


def cav_scene(seed=31, n=32, B=8, n_lam_per_line=8, n_dir=8):
    """Small 3D Core-and-Voigt scene: smooth density, two Voigt lines, |v| <= 30 km/s."""
    rng = [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(8)]
    shp = (n, n, n)
    dens = np.exp(-np.arange(n)[:, None, None] / 12.0) * np.exp(0.5 * grf(rng[0], shp, 6.0))
    nbl = n // B
    bact = (grf(rng[1], (nbl,) * 3, 1.5) > -0.3).reshape(-1).astype(np.uint8)
    mask = np.repeat(np.repeat(np.repeat(bact.reshape((nbl,) * 3), B, 0), B, 1), B, 2).astype(bool)
    T = 0.6 + 0.6 * (1 + np.tanh(grf(rng[2], shp, 8.0))) / 2
    S = np.exp(-1.0 / T)
    vel = np.stack([10.0 * grf(rng[3 + i], shp, 8.0) for i in range(3)])
    vel *= 30.0 / np.sqrt((vel ** 2).sum(0)).max()
    lam0 = np.array([500.0, 500.2])
    vD = 8.0 * np.sqrt(T)
    a = 10.0 ** (-3.0 + 2.0 * 0.5 * (1 + np.tanh(grf(rng[6], shp, 6.0))))
    chi_star = np.stack([c * dens * math.sqrt(math.pi) * l0 * 8.0 / C_KMS for c, l0 in ((50.0, lam0[0]), (2.0, lam0[1]))])
    inv_dld = np.stack([C_KMS / (l0 * vD) for l0 in lam0])
    dv = np.linspace(-80, 80, n_lam_per_line)
    lam = np.concatenate([l0 * (1 + dv / C_KMS) for l0 in lam0])
    f = lambda x, k: (x * mask).astype(np.float32).reshape(k, -1)  # noqa: E731
    return dict(dim=3, n=(n, n, n), brick=B, n_levels=4, model="lines", profile="voigt", lam=lam, lam0=lam0,
                eta_star=f(chi_star * S, 2), chi_star=f(chi_star, 2), damp=f(np.stack([a, a]), 2),
                inv_dld=f(inv_dld, 2), eta_bg=f(1e-3 * dens * S, 1)[0], chi_bg=f(1e-3 * dens, 1)[0],
                vel=f(vel, 3), dirs=directions_fibonacci(n_dir), block_active=bact, ds0=1.0, I0=0.0)


def oracle_levels(sc, lam_idx, rule, T, tau=0.25, rel=0.0):
    """Batch levels from the oracle: MIP-0 values by the velocity rule, then the IoD chain."""
    s = orc.Scene(sc, lam_idx=lam_idx)
    lvs = []
    for il in range(len(lam_idx)):
        e, c = orc.lines_mip0(s, il, rule)
        lvs.append(orc.levels_one(s, e, c, sc["block_active"], T * (1 + rel), tau * (1 + rel)))
    return orc.batch_levels(lvs)


def level_band(sc):
    """Relative tie band on T and tau_thin inside which device and oracle may take different levels.
    Gaussian lines: MIP-0 values are FP64 on both sides in the same order of operations, so only the last-ulp
    rounding of exp and log differs: 1e-9.  Voigt lines: the device takes its single-precision profile (relative
    error below 1e-4 per value, i.e. 1e-4 absolute on every ln(q ds0)).  That moves a cell's mean by <= 1e-4 and
    its deviations by <= 2e-4, hence its variance by <= 4e-4 sqrt(Var) + 4e-8, and near the threshold
    (Var ~ T |mean|) its index of dispersion by <= 4e-4 sqrt(T / |mean|) + 1e-4 T / |mean|: at most 3e-3 T for
    T >= 1e-2 and |mean ln(chi ds0)| >= 0.5, the cells that decide these scenes' levels."""
    return 1e-9 if sc.get("profile", "gauss") == "gauss" else 3e-3


def check_levels(lv_gpu, sc, lam_idx, rule, T):
    """The device's level map against the oracle's.  Every block whose oracle level stays put when T and tau_thin
    move by the tie band must match exactly; inside the band the device's level must be one of the levels the
    band admits.  Returns the device's map: valid everywhere, it is what the oracle then marches (the intensities
    are compared on the same adapted cells, no ray left out)."""
    band = level_band(sc)
    lv = oracle_levels(sc, lam_idx, rule, T)
    lo = oracle_levels(sc, lam_idx, rule, T, rel=-band)
    hi = oracle_levels(sc, lam_idx, rule, T, rel=band)
    robust = (lo == lv) & (hi == lv)
    off = lv_gpu != lv
    assert not np.any(off & robust), "levels differ outside the tie band: blocks %s" % np.nonzero(off & robust)[0][:8]
    assert np.all(~off | (lv_gpu == lo) | (lv_gpu == hi)), "in-band level outside the band's choices"
    if off.any():
        print("levels: %d of %d blocks in the tie band (band %g) took the other level" % (off.sum(), lv.size, band))
    return lv_gpu


def sample_rays(scene, n_dir, n, seed):
    rng = np.random.default_rng(seed)
    probes = scene.probe_voxels()
    k = rng.choice(probes.size, n, replace=False)
    d = rng.integers(0, n_dir, n).astype(np.int32)
    return k, probes[k], d


def test_velinterp_parity(rt, vscene):
    import torch
    sc = vscene
    T = 1e-2
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    scene = rt.Scene.from_dict(sc, emission="velinterp", n_v=21)
    k, vox, d = sample_rays(scene, 8, 600, 1)
    for lam0 in (0, 8):
        scene.build(lam0, lam0 + 8, iod_threshold=T)
        lv = check_levels(scene.levels(), sc, list(range(lam0, lam0 + 8)), 0, T)
        s = orc.Scene(sc, lam_idx=list(range(lam0, lam0 + 8)), n_v=21)
        for mode, lev in (("vlm", lv), ("level0", np.where(lv >= 0, 0, -1).astype(np.int8))):
            I = scene.trace(dirs, mode=mode).cpu().numpy()[d, :, k]
            ref = orc.march(s, orc.VELINTERP, lev, vox, d)
            st = orc.rel_err_stats(I, ref)
            assert st["n_ref_zero_mismatch"] == 0 and st["p100"] < 1e-4, (mode, st)
        # approximation error against the dense Classic march (reported)
        ref_c = orc.march(s, orc.CLASSIC, None, vox, d)
        I = scene.trace(dirs, mode="vlm", level_dist=rt.CASCADE_LEVEL_DIST).cpu().numpy()[d, :, k]
        print("velinterp VLM(graded) vs Classic:", orc.rel_err_stats(I, ref_c))
    assert lv.max() >= 1


@pytest.mark.parametrize("vgrid", ["full", "orthant"])
def test_velinterp_grid_modes_parity(rt, vscene, vgrid):
    """Both node-grid modes (one grid over [-V, V], or one per orthant of directions) against the oracle's, on
    the same adapted cells, in 2D (8 directions over the 4 quadrants) and 3D (12 directions over the 8 octants)."""
    import torch
    for sc, T in ((vscene, 1e-2), (dict(cav_scene(n_dir=12), profile="gauss"), 0.1)):
        n_dir = sc["dirs"].shape[0]
        dirs = torch.from_numpy(sc["dirs"]).cuda()
        scene = rt.Scene.from_dict(sc, emission="velinterp", n_v=9, vgrid=vgrid)
        k, vox, d = sample_rays(scene, n_dir, 400, 11)
        scene.build(0, 8, iod_threshold=T)
        lv = check_levels(scene.levels(), sc, list(range(8)), 0, T)
        s = orc.Scene(sc, lam_idx=list(range(8)), n_v=9, vgrid=vgrid)
        I = scene.trace(dirs, mode="vlm").cpu().numpy()[d, :, k]
        st = orc.rel_err_stats(I, orc.march(s, orc.VELINTERP, lv, vox, d))
        assert st["n_ref_zero_mismatch"] == 0 and st["p100"] < 1e-4, (sc["dim"], vgrid, st)
        q = np.array([(w < 0).astype(int) @ (1 << np.arange(sc["dim"])) for w in sc["dirs"]])
        assert len(set(q.tolist())) == 1 << sc["dim"]  # every orthant is exercised


@pytest.mark.parametrize("dim,storage", [(2, "bf16"), (2, "f16"), (3, "bf16")])
def test_velinterp_reduced_precision_storage(rt, vscene, dim, storage):
    """Velocity-interpolation node records stored in BF16 / FP16 (round to nearest even, unit roundoff
    u = 2^-8 / 2^-11) against the FP64 oracle on the same adapted cells.  Each interpolated eta, chi is a convex
    combination of two rounded node values, so it carries a relative error <= u; a segment's contribution
    T S (1 - e^-tau) moves by <= 2u through its own eta and chi (the factor (1 - e^-tau)/chi has a relative
    sensitivity to chi in [-1, 0]) and by tau_up u through the upstream transmission T.  Contributions from behind
    tau_up > 3 weigh less than e^-3 of the source-function contrast, so I moves by ~(2 + 3) u at most: bounded here
    by 4u at p99.9 and 16u overall.  Levels do not depend on the storage dtype."""
    import torch
    if dim == 2:
        sc, T, rule = vscene, 1e-2, 0
    else:
        sc, T, rule = cav_scene(), 0.1, 0
    u = 2.0 ** -8 if storage == "bf16" else 2.0 ** -11
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    scene = rt.Scene.from_dict(sc, emission="velinterp", n_v=21)
    k, vox, d = sample_rays(scene, 8, 400, 7)
    scene.build(0, 8, iod_threshold=T)
    I32 = scene.trace(dirs, mode="vlm").cpu().numpy()[d, :, k]
    lv_gpu = scene.levels()
    scene.build(0, 8, iod_threshold=T, storage=storage)
    assert np.array_equal(scene.levels(), lv_gpu)
    I = scene.trace(dirs, mode="vlm").cpu().numpy()[d, :, k]
    lv = check_levels(lv_gpu, sc, list(range(8)), rule, T)
    s = orc.Scene(sc, lam_idx=list(range(8)), n_v=21)
    ref = orc.march(s, orc.VELINTERP, lv, vox, d)
    st = orc.rel_err_stats(I, ref)
    st32 = orc.rel_err_stats(I32, ref)
    print("velinterp %dD %s nodes vs FP64: p99.9 %.3g max %.3g = %.2f u (FP32 nodes: max %.3g)" % (
        dim, storage, st["p99.9"], st["p100"], st["p100"] / u, st32["p100"]))
    # FP32 nodes: Gaussian lines within FP32 rounding; the 3D scene's Voigt lines add the device Voigt
    # function's 5.3e-5 relative error to every node value
    assert st32["p100"] < (1e-4 if dim == 2 else 5e-4)
    assert st["n_ref_zero_mismatch"] == 0 and st["p99.9"] < 4 * u and st["p100"] < 16 * u, st


def test_velinterp_core_frame_levels(rt, vscene):
    """Velocity interpolation with the level test in the core-closest frame: levels follow the oracle's rule 1."""
    sc = vscene
    T = 1e-2
    scene = rt.Scene.from_dict(sc, emission="velinterp", n_v=21)
    for lam0 in (0, 8):
        scene.build(lam0, lam0 + 8, iod_threshold=T, iod_frame="core")
        lv_core = scene.levels()
        check_levels(lv_core, sc, list(range(lam0, lam0 + 8)), 1, T)
        scene.build(lam0, lam0 + 8, iod_threshold=T)
        assert np.all(lv_core <= scene.levels() + 3)  # both valid level maps


def test_cav_parity(rt):
    import torch
    sc = cav_scene()
    T = 0.1
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    scene = rt.Scene.from_dict(sc, emission="cav")
    k, vox, d = sample_rays(scene, 8, 300, 2)
    for lam0 in (0, 8):
        scene.build(lam0, lam0 + 8, iod_threshold=T)
        lv = check_levels(scene.levels(), sc, list(range(lam0, lam0 + 8)), 1, T)
        s = orc.Scene(sc, lam_idx=list(range(lam0, lam0 + 8)))
        for mode, lev in (("vlm", lv), ("level0", np.where(lv >= 0, 0, -1).astype(np.int8))):
            I = scene.trace(dirs, mode=mode).cpu().numpy()[d, :, k]
            ref = orc.march(s, orc.CAV, lev, vox, d)
            st = orc.rel_err_stats(I, ref)
            assert st["n_ref_zero_mismatch"] == 0 and st["p99.9"] < 1e-3 and st["p100"] < 5e-3, (mode, st)
        ref_c = orc.march(s, orc.CLASSIC, None, vox, d)
        I = scene.trace(dirs, mode="vlm", level_dist=rt.CASCADE_LEVEL_DIST).cpu().numpy()[d, :, k]
        print("CaV VLM(graded) vs Classic:", orc.rel_err_stats(I, ref_c))


def test_cav_chain_follows_the_averaging_mode(rt):
    """The Core-and-Voigt chain is rebuilt when a build asks for the other stored-value mode: LOG, then LINEAR
    again, each against the oracle in the same mode on the same cells."""
    import torch
    sc = cav_scene()
    T = 0.1
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    scene = rt.Scene.from_dict(sc, emission="cav")
    k, vox, d = sample_rays(scene, 8, 200, 4)
    for avg in ("log", "linear"):
        scene.build(0, 8, iod_threshold=T, avg_mode=avg)
        lv = check_levels(scene.levels(), sc, list(range(0, 8)), 1, T)
        s = orc.Scene(sc, lam_idx=list(range(0, 8)), avg_mode=orc.AVG_LOG if avg == "log" else orc.AVG_LINEAR)
        I = scene.trace(dirs, mode="vlm").cpu().numpy()[d, :, k]
        st = orc.rel_err_stats(I, orc.march(s, orc.CAV, lv, vox, d))
        assert st["n_ref_zero_mismatch"] == 0 and st["p99.9"] < 1e-3 and st["p100"] < 5e-3, (avg, st)


@pytest.mark.parametrize("storage,bound", [("bf16", 5e-2), ("f16", 1e-2)])
def test_cav_reduced_precision_storage(rt, storage, bound):
    """Core and Voigt with the line-parameter chain stored in BF16 / FP16 (round to nearest even) against the FP64
    oracle on the same adapted cells.  Bound from the storage rounding (2^-8 BF16, 2^-11 FP16 relative on each of
    eta*, chi*, a, 1/dlD and v): the profile argument's relative error is amplified by up to 2 x^2 in the Gaussian
    core-to-wing range (x <~ 3), about 5 % (BF16) and 1 % (FP16) at p99.9 over the sample."""
    import torch
    sc = cav_scene()
    T = 0.1
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    scene = rt.Scene.from_dict(sc, emission="cav")
    k, vox, d = sample_rays(scene, 8, 300, 3)
    scene.build(0, 8, iod_threshold=T)
    I32 = scene.trace(dirs, mode="vlm").cpu().numpy()[d, :, k]
    lv_gpu = scene.levels()
    scene.build(0, 8, iod_threshold=T, storage=storage)
    assert np.array_equal(scene.levels(), lv_gpu)  # levels do not depend on the storage dtype
    I = scene.trace(dirs, mode="vlm").cpu().numpy()[d, :, k]
    lv = check_levels(lv_gpu, sc, list(range(0, 8)), 1, T)
    s = orc.Scene(sc, lam_idx=list(range(0, 8)))
    ref = orc.march(s, orc.CAV, lv, vox, d)
    st = orc.rel_err_stats(I, ref)
    st32 = orc.rel_err_stats(I32, ref)
    print("CaV %s storage vs FP64: p99.9 %.3g max %.3g (FP32 storage: p99.9 %.3g)" % (
        storage, st["p99.9"], st["p100"], st32["p99.9"]))
    assert st["n_ref_zero_mismatch"] == 0 and st["p99.9"] < bound


def test_cav_level0_dense_is_classic(rt, vscene):
    """A dense scene traced at level 0 with Core and Voigt is the DenseClassic march."""
    import torch
    sc = vscene
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    scene = rt.Scene.from_dict(sc, emission="cav", dense=True)
    assert scene.info["n_active"] == (128 // 16) ** 2
    scene.build(0, 8)
    k, vox, d = sample_rays(scene, 8, 400, 3)
    I = scene.trace(dirs, mode="level0").cpu().numpy()[d, :, k]
    s = orc.Scene(sc, lam_idx=list(range(8)))
    ref = orc.march(s, orc.CLASSIC, None, vox, d)
    st = orc.rel_err_stats(I, ref)
    assert st["n_ref_zero_mismatch"] == 0 and st["p100"] < 2e-5, st


def test_workspace_bytes_match_allocation(rt, vscene):
    """The host-only size query equals what rt_scene_create allocated (velocity nodes, Core-and-Voigt chains)."""
    for sc, emis in ((vscene, "velinterp"), (cav_scene(), "cav")):
        s = rt.Scene.from_dict(sc, emission=emis)
        assert s.info["storage_bytes"] == rt.scene_workspace_bytes(sc, n_active=s.info["n_active"], emission=emis)


def test_velocity_grid_warning(rt, vscene):
    """Sect. 3.1: the build warns when velocity nodes are more than two thermal widths apart."""
    import warnings
    sc = vscene  # |v| <= 30 km/s, thermal width 10 km/s
    coarse = rt.Scene.from_dict(sc, emission="velinterp", n_v=2)   # >= 30 km/s apart: >= 3 widths
    with pytest.warns(rt.VelocityGridWarning):
        coarse.build(0, 8)
    fine = rt.Scene.from_dict(sc, emission="velinterp", n_v=21)    # <= 3 km/s apart (orthant ranges <= 60 km/s)
    with warnings.catch_warnings():
        warnings.simplefilter("error", rt.VelocityGridWarning)
        fine.build(0, 8)
    assert fine.velocity_grid_ratio.max() < 0.31


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_pipelined_velinterp_march_equals_the_unpipelined_one(rt, vscene, storage):
    """The plain march applies each segment's node records one traversal step after loading them; the
    truncated march's inference mode with every block falling back runs the same march unpipelined.  Same
    segments, same order, same arithmetic: the intensities are equal bit for bit (VLM, path-graded cascade caps,
    and MIP 0)."""
    import torch
    sc = vscene
    scene = rt.Scene.from_dict(sc, emission="velinterp", n_v=41)
    scene.build(0, 8, iod_threshold=1e-2, storage=storage, velocity_grid_warn=0)
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    ld = rt.CASCADE_LEVEL_DIST
    fb = torch.ones(scene.info["n_blocks"], dtype=torch.uint8, device="cuda")
    assert (scene.levels() > 0).any(), "the test needs merged blocks"
    for mode, kw in (("vlm", dict(level_dist=ld, grade="path")), ("level0", {})):
        full = scene.trace(dirs, mode=mode, **kw)
        inf = scene.trace_truncated(dirs, 32.0, gen=False, fallback=fb, mode=mode, **kw)
        torch.cuda.synchronize()
        assert torch.equal(inf["I_near"], full), mode
