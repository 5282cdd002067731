"""GPU parity of radiance-interval tracing (rt_trace_interval) against the FP64 oracle.

Each ray is traversed over [t1, t2] only (Eq. Ray and the HDDA procedure of
Alg. 1 take [t1, t2]); the cascade layout of Sect. 4.1 gives interval ends
1.5 * 4^c and per-cascade MIP caps [0, 0, 1, 2, 3, 4].  Covered: [0, inf)
equals rt_trace, cascade intervals with per-call caps (plain and
distance-graded) against the oracle on the same cells, composition of the
intervals back into the whole ray, intervals beyond the grid and empty
intervals, argument errors, and the velocity-interpolation and Core-and-Voigt
emission paths.
"""
import numpy as np
import pytest

import oracle as orc
from synth import make_cfg1, make_cfg2
from test_gpu_lines import cav_scene, check_levels, sample_rays
from test_gpu_static import TOL_SAME_CELLS, all_pairs, oracle_batch

pytestmark = pytest.mark.gpu

ENDS = [0.0, 1.5, 6.0, 24.0, 96.0, np.inf]  # cascade intervals; the last runs to the boundary
CAPS = [0, 0, 1, 2, 3]                      # per-cascade maximum MIP level (the paper's schedule, truncated at L - 1)


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_08498_amd as rt
    rt.lib()
    return rt


@pytest.fixture(scope="module")
def cfg1():
    return make_cfg1()


def _check_T(T, Tr, bound, what):
    """Transmittance: relative bound where the FP64 value is representable in FP32 (> 1e-30); where it
    underflows (optically thick intervals, e^-tau < 1e-30) the FP32 value must be below 1e-30 too."""
    T, Tr = np.asarray(T, np.float64), np.asarray(Tr, np.float64)
    big = Tr > 1e-30
    rel = np.abs(T[big] - Tr[big]) / Tr[big]
    assert rel.size == 0 or rel.max() < bound, (what, float(rel.max()))
    assert np.all(T[~big] <= 1e-30), what


def _p100(st):
    """largest relative error (0 when every reference value is 0, e.g. an interval past every exit)"""
    return st.get("p100", 0.0)


def _dir_lam_probe(ref, n_dir, n_probes, nl):
    """oracle [ray = dir-major][lam] -> [dir][lam][probe]"""
    return ref.reshape(n_dir, n_probes, nl).transpose(0, 2, 1)


def test_whole_ray_interval_is_trace(rt, cfg1):
    import torch
    dirs = torch.from_numpy(cfg1["dirs"]).cuda()
    scene = rt.Scene.from_dict(cfg1)
    scene.build(0, 8, iod_threshold=0.1)
    for kw in (dict(mode="vlm"), dict(mode="level0"), dict(mode="vlm", level_dist=rt.CASCADE_LEVEL_DIST),
               dict(mode="vlm", I0=0.7)):
        I = scene.trace(dirs, **kw).cpu().numpy()
        Ii, Ti = scene.trace_interval(dirs, 0.0, np.inf, **kw)
        assert np.array_equal(Ii.cpu().numpy(), I), kw
        T = Ti.cpu().numpy()
        assert np.all((T > 0) & (T <= 1))


@pytest.mark.parametrize("graded", [False, True])
def test_cascade_intervals_static(rt, cfg1, graded):
    import torch
    dirs = torch.from_numpy(cfg1["dirs"]).cuda()
    scene = rt.Scene.from_dict(cfg1)
    probes, vox, d = all_pairs(scene, 8)
    scene.build(0, 8, iod_threshold=0.1)
    s, lv, _, _ = oracle_batch(cfg1, 0, 8, 0.1)
    ld = rt.CASCADE_LEVEL_DIST if graded else None
    s.set_level_dist(ld)
    for I0 in (0.0, 0.7):
        s.s.I0 = I0
        for c in range(len(CAPS)):
            t1, t2 = ENDS[c], ENDS[c + 1]
            I, T = scene.trace_interval(dirs, t1, t2, mode="vlm", max_level=CAPS[c], level_dist=ld, I0=I0)
            Ir, Tr = orc.march_interval(s, orc.STATIC, orc.cap_levels(lv, CAPS[c]), vox, d, t1, t2)
            Ir, Tr = _dir_lam_probe(Ir, 8, probes.size, 8), _dir_lam_probe(Tr, 8, probes.size, 8)
            st = orc.rel_err_stats(I.cpu().numpy(), Ir)
            assert st["n_ref_zero_mismatch"] == 0 and _p100(st) < TOL_SAME_CELLS, (c, I0, st)
            _check_T(T.cpu().numpy(), Tr, TOL_SAME_CELLS, (c, I0))
        # cfg1's longest ray (64 sqrt 2 < 96) has left the grid before the last cascade starts
        I, T = scene.trace_interval(dirs, ENDS[-2], ENDS[-1], mode="vlm", I0=I0)
        assert torch.all(I == 0).item() and torch.all(T == 1).item()


def test_intervals_compose_into_the_ray(rt):
    """Without caps the cascade intervals cover the ray: I = I_0 + T_0 (I_1 + T_1 (...)) equals rt_trace
    up to FP32 rounding (a cell split at an interval end is two exponentials instead of one)."""
    import torch
    sc = make_cfg2(seed=21, n=128, B=16, n_lam_per_line=8, n_dir=8)
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    scene = rt.Scene.from_dict(sc, emission="velinterp", n_v=21)
    scene.build(0, 8, iod_threshold=1e-2)
    for kw in (dict(mode="vlm"), dict(mode="vlm", level_dist=rt.CASCADE_LEVEL_DIST), dict(mode="level0", I0=0.3)):
        full = scene.trace(dirs, **kw).double()
        acc = torch.zeros_like(full)
        trans = torch.ones_like(full)
        for t1, t2 in zip(ENDS[:-1], ENDS[1:]):
            I, T = scene.trace_interval(dirs, t1, t2, **kw)
            acc += trans * I.double()
            trans *= T.double()
        st = orc.rel_err_stats(acc.cpu().numpy(), full.cpu().numpy())
        assert st["n_ref_zero_mismatch"] == 0 and _p100(st) < 5e-5, (kw, st)


def test_interval_edges_and_errors(rt, cfg1):
    import torch
    dirs = torch.from_numpy(cfg1["dirs"]).cuda()
    scene = rt.Scene.from_dict(cfg1)
    scene.build(0, 8, iod_threshold=0.1)
    for t1, t2 in ((1e6, 2e6), (1e6, np.inf), (5.0, 5.0), (0.0, 0.0), (2.5, 2.5)):
        I, T = scene.trace_interval(dirs, t1, t2, I0=0.9)
        assert torch.all(I == 0).item() and torch.all(T == 1).item(), (t1, t2)
    # the whole ray collects I0 through its transmittance
    I, T = scene.trace_interval(dirs, 0.0, np.inf, I0=0.9)
    assert torch.all(I >= 0.9 * T * (1 - 1e-6)).item()
    I_noT, T_none = scene.trace_interval(dirs, 1.5, 6.0, want_T=False)
    I_T, _ = scene.trace_interval(dirs, 1.5, 6.0)
    assert T_none is None and torch.equal(I_noT, I_T)
    for t1, t2 in ((3.0, 2.0), (-1.0, 2.0), (np.inf, np.inf), (np.nan, 1.0), (0.0, np.nan)):
        with pytest.raises(RuntimeError):
            scene.trace_interval(dirs, t1, t2)
    # explicit probe list: the same rays as the all-probe launch
    probes = scene.probe_voxels()
    sel = probes[::7].copy()
    I_all, T_all = scene.trace_interval(dirs, 1.5, 24.0, max_level=1)
    I_sel, T_sel = scene.trace_interval(dirs, 1.5, 24.0, probes=sel, max_level=1)
    assert torch.equal(I_sel, I_all[:, :, ::7]) and torch.equal(T_sel, T_all[:, :, ::7])


@pytest.mark.parametrize("emission", ["velinterp", "cav"])
def test_cascade_intervals_lines(rt, emission):
    import torch
    if emission == "velinterp":
        sc = make_cfg2(seed=21, n=128, B=16, n_lam_per_line=8, n_dir=8)
        T, kind, rule, kw = 1e-2, orc.VELINTERP, 0, dict(n_v=21)
    else:
        sc = cav_scene()
        T, kind, rule, kw = 0.1, orc.CAV, 1, {}
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    scene = rt.Scene.from_dict(sc, emission=emission, **kw)
    k, vox, d = sample_rays(scene, 8, 400, 5)
    scene.build(0, 8, iod_threshold=T)
    lv = check_levels(scene.levels(), sc, list(range(8)), rule, T)
    s = orc.Scene(sc, lam_idx=list(range(8)), **kw)
    bound = 1e-4 if emission == "velinterp" else 5e-3
    for c in range(len(CAPS)):
        t1, t2 = ENDS[c], ENDS[c + 1]
        I, Tt = scene.trace_interval(dirs, t1, t2, mode="vlm", max_level=CAPS[c])
        I, Tt = I.cpu().numpy()[d, :, k], Tt.cpu().numpy()[d, :, k]
        Ir, Tr = orc.march_interval(s, kind, orc.cap_levels(lv, CAPS[c]), vox, d, t1, t2)
        st = orc.rel_err_stats(I, Ir)
        assert st["n_ref_zero_mismatch"] == 0 and _p100(st) < bound, (c, st)
        _check_T(Tt, Tr, bound, c)


def test_path_graded_visited_cells_bit_exact(rt, cfg1):
    """Path grading: the level cap rises at t = level_dist[m] inside a cell; visited cells and levels equal the
    oracle's bit for bit, segment ends to 1e-13 (the split points are the schedule's values)."""
    import math
    scene = rt.Scene.from_dict(cfg1)
    scene.build(0, 8, iod_threshold=1.0)
    s, lv, _, _ = oracle_batch(cfg1, 0, 8, 1.0)
    assert np.array_equal(scene.levels(), lv)
    rng = np.random.default_rng(8)
    probes = scene.probe_voxels()
    dirs = list(cfg1["dirs"]) + [np.array(v, np.float32) for v in ([1, 0], [0, -1], [math.sqrt(.5), math.sqrt(.5)],
                                                                  [-0.6, 0.8])]
    nchk = nsplit = 0
    for sched in ((0, 6, 24, 96), (0, 2.5, 7, 30), (0, 0, 5, 5)):
        s.set_level_dist(sched, mode="path")
        for w in dirs:
            for pv in rng.choice(probes, 25, replace=False):
                cells, tt = scene.visited(int(pv), w, mode="vlm", level_dist=sched, grade="path")
                oc, ol, oti, oto = orc.ray_segments(s, lv, (int(pv) % 64, int(pv) // 64), w)
                assert len(cells) == len(oc), (sched, pv, w)
                assert np.array_equal(cells[:, :3], oc) and np.array_equal(cells[:, 3], ol)
                np.testing.assert_allclose(tt[:, 0], oti, rtol=1e-13, atol=1e-13)
                np.testing.assert_allclose(tt[:, 1], oto, rtol=1e-13, atol=1e-13)
                nsplit += int(np.isin(oti, np.array(sched[1:], np.float64)).sum())
                nchk += 1
    s.set_level_dist(None)
    assert nchk > 700 and nsplit > 50


def test_path_graded_intensities_and_cascades(rt, cfg1):
    """Path-graded whole-ray march against the oracle on the same cells, and against the composition of the
    capped cascade intervals on the GPU (FP32 rounding only)."""
    import torch
    dirs = torch.from_numpy(cfg1["dirs"]).cuda()
    scene = rt.Scene.from_dict(cfg1)
    probes, vox, d = all_pairs(scene, 8)
    scene.build(0, 8, iod_threshold=0.1)
    s, lv, _, _ = oracle_batch(cfg1, 0, 8, 0.1)
    LD = rt.CASCADE_LEVEL_DIST
    s.set_level_dist(LD, mode="path")
    I = scene.trace(dirs, mode="vlm", level_dist=LD, grade="path")
    ref = _dir_lam_probe(orc.march(s, orc.STATIC, lv, vox, d), 8, probes.size, 8)
    st = orc.rel_err_stats(I.cpu().numpy(), ref)
    assert st["n_ref_zero_mismatch"] == 0 and _p100(st) < TOL_SAME_CELLS, st
    acc = torch.zeros_like(I, dtype=torch.float64)
    trans = torch.ones_like(acc)
    for c in range(len(CAPS)):
        Ic, Tc = scene.trace_interval(dirs, ENDS[c], ENDS[c + 1], mode="vlm", max_level=CAPS[c])
        acc += trans * Ic.double()
        trans *= Tc.double()
    st = orc.rel_err_stats(acc.cpu().numpy(), I.double().cpu().numpy())
    assert _p100(st) < 5e-5, st
    # path grading coarsens no later than entry grading: never more segments
    sp = torch.zeros(5, dtype=torch.int64, device="cuda")
    se = torch.zeros(5, dtype=torch.int64, device="cuda")
    scene.trace(dirs, mode="vlm", level_dist=LD, grade="path", stats=sp)
    scene.trace(dirs, mode="vlm", level_dist=LD, stats=se)
    assert sp[0].item() <= se[0].item()
    # the same rule inside an interval: [6, 96] path-graded equals [6, 24] capped at 1 composed with [24, 96] at 2
    I1, T1 = scene.trace_interval(dirs, 6.0, 96.0, mode="vlm", level_dist=LD, grade="path")
    Ia, Ta = scene.trace_interval(dirs, 6.0, 24.0, mode="vlm", max_level=1)
    Ib, Tb = scene.trace_interval(dirs, 24.0, 96.0, mode="vlm", max_level=2)
    comp = (Ia.double() + Ta.double() * Ib.double()).cpu().numpy()
    st = orc.rel_err_stats(comp, I1.double().cpu().numpy())
    assert st["n_ref_zero_mismatch"] == 0 and _p100(st) < 5e-5, st
    _check_T(T1.cpu().numpy(), (Ta.double() * Tb.double()).cpu().numpy(), 5e-5, "T [6, 96]")


@pytest.mark.parametrize("emission", ["velinterp", "cav"])
def test_path_graded_lines(rt, emission):
    import torch
    if emission == "velinterp":
        sc = make_cfg2(seed=21, n=128, B=16, n_lam_per_line=8, n_dir=8)
        T, kind, rule, kw = 1e-2, orc.VELINTERP, 0, dict(n_v=21)
    else:
        sc = cav_scene()
        T, kind, rule, kw = 0.1, orc.CAV, 1, {}
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    scene = rt.Scene.from_dict(sc, emission=emission, **kw)
    k, vox, d = sample_rays(scene, 8, 400, 6)
    scene.build(0, 8, iod_threshold=T)
    lv = check_levels(scene.levels(), sc, list(range(8)), rule, T)
    s = orc.Scene(sc, lam_idx=list(range(8)), **kw)
    s.set_level_dist(rt.CASCADE_LEVEL_DIST, mode="path")
    I = scene.trace(dirs, mode="vlm", level_dist=rt.CASCADE_LEVEL_DIST, grade="path").cpu().numpy()[d, :, k]
    ref = orc.march(s, kind, lv, vox, d)
    st = orc.rel_err_stats(I, ref)
    bound = 1e-4 if emission == "velinterp" else 5e-3
    assert st["n_ref_zero_mismatch"] == 0 and _p100(st) < bound, st


@pytest.mark.parametrize("grade", ["entry", "path"])
def test_intervals_compose_in_3d(rt, grade):
    """3D Core and Voigt, distance-graded: the whole ray equals its cascade intervals composed (the start block of
    each interval keeps the cap of the path length at which the ray entered it, or the cap along the path)."""
    import torch
    sc = cav_scene()
    dirs = torch.from_numpy(sc["dirs"]).cuda()
    scene = rt.Scene.from_dict(sc, emission="cav")
    scene.build(0, 8, iod_threshold=0.1)
    ld = (0.0, 2.0, 6.0, 12.0)
    kw = dict(mode="vlm", level_dist=ld, grade=grade)
    full = scene.trace(dirs, **kw).double()
    ends = [0.0, 1.5, 4.0, 9.0, 20.0, np.inf]
    acc = torch.zeros_like(full)
    trans = torch.ones_like(full)
    for t1, t2 in zip(ends[:-1], ends[1:]):
        I, T = scene.trace_interval(dirs, t1, t2, **kw)
        acc += trans * I.double()
        trans *= T.double()
    st = orc.rel_err_stats(acc.cpu().numpy(), full.cpu().numpy())
    assert st["n_ref_zero_mismatch"] == 0 and _p100(st) < 5e-4, st
