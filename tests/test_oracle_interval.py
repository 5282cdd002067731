"""Pins of the oracle's radiance-interval march (CPU only).

The traversal of Sect. 2.3 (Eq. Ray, Alg. 1) runs over a path interval
[t1, t2]; the deployment of Sect. 4.1 splits each ray into cascade intervals
whose end distances grow by 4 per cascade from 1.5 voxels.  What the
mathematics fixes, independently of the oracle's own code:
  - the whole ray [0, inf) is the long-characteristic march;
  - transfer over consecutive intervals composes: I = I_a + T_a I_b and
    T = T_a T_b (the formal solution's semigroup property);
  - a homogeneous medium has I = S (1 - e^-chi L), T = e^-chi L over the
    interval's path length L inside the grid;
  - the clipped cell list equals the exact-rational one clipped to [t1, t2];
  - a fine midpoint quadrature of the integral form, with each sample's cell
    found by flooring the sample point, converges to the same I.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle.exact import adapted_cells_exact, ray_cells_exact

from test_oracle_march import _rand_dirs, static_scene

CASCADE_ENDS = [1.5 * 4 ** c for c in range(5)]  # 1.5, 6, 24, 96, 384; the last cascade runs to the boundary


def _cfg1_static(orc, T=1e-2):
    from synth import make_cfg1
    sc = make_cfg1()
    s = orc.Scene(sc)
    lvs, st_e, st_c = orc.static_level_values(s, sc["eta"], sc["chi"], sc["block_active"], T=T)
    s.set_static_levels(st_e, st_c)
    return sc, s, orc.batch_levels(lvs)


def test_whole_ray_is_the_march(orc):
    sc, s, lv = _cfg1_static(orc)
    rng = np.random.default_rng(21)
    vox = rng.integers(0, 4096, size=400).astype(np.int32)
    d = rng.integers(0, 8, size=400).astype(np.int32)
    for levels in (None, lv):
        I_full = orc.march(s, orc.STATIC, levels, vox, d)
        I, T = orc.march_interval(s, orc.STATIC, levels, vox, d, 0.0, np.inf)
        assert np.array_equal(I, I_full)
        assert np.all((T > 0) & (T <= 1))


@pytest.mark.parametrize("graded", [False, True])
def test_cascade_intervals_compose(orc, graded):
    """I over [0, inf) = I_0 + T_0 (I_1 + T_1 (I_2 + ...)) over the cascade intervals."""
    sc, s, lv = _cfg1_static(orc)
    if graded:
        s.set_level_dist((0, 3, 9, 27))
    rng = np.random.default_rng(22)
    vox = rng.integers(0, 4096, size=500).astype(np.int32)
    d = rng.integers(0, 8, size=500).astype(np.int32)
    for I0 in (0.0, 0.7):
        s.s.I0 = I0
        I_full, T_full = orc.march_interval(s, orc.STATIC, lv, vox, d, 0.0, np.inf)
        ends = [0.0] + CASCADE_ENDS + [np.inf]
        parts = [orc.march_interval(s, orc.STATIC, lv, vox, d, a, b) for a, b in zip(ends[:-1], ends[1:])]
        I, T = np.zeros_like(I_full), np.ones_like(I_full)
        for Ic, Tc in parts:
            I += T * Ic
            T *= Tc
        np.testing.assert_allclose(I, I_full, rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(T, T_full, rtol=1e-12, atol=0)
    s.s.I0 = 0.0


def test_homogeneous_interval_closed_form(orc):
    rng = np.random.default_rng(23)
    n = (16, 16)
    eta0, chi0, I0 = float(np.float32(0.37)), float(np.float32(0.23)), 0.8
    sc = static_scene(n, 8, np.full((1, 16, 16), eta0), np.full((1, 16, 16), chi0), I0=I0)
    S = eta0 / chi0
    for trial in range(60):
        pv = (int(rng.integers(0, 16)), int(rng.integers(0, 16)))
        th = rng.uniform(0, 2 * np.pi)
        w = np.array([np.cos(th), np.sin(th)], np.float32)
        sc["dirs"] = w[None]
        s = orc.Scene(sc)
        s.set_static_levels(sc["eta"].astype(np.float64), sc["chi"].astype(np.float64))
        _, ti, to = ray_cells_exact(2, n, pv, w)
        texit = float(to[-1])
        t1 = float(rng.uniform(0, 1.2 * texit))
        t2 = t1 + float(rng.uniform(0, 12))
        vox = np.array([pv[0] + 16 * pv[1]], np.int32)
        I, T = orc.march_interval(s, orc.STATIC, None, vox, np.zeros(1, np.int32), t1, t2)
        L = max(0.0, min(t2, texit) - t1)
        Tref = math.exp(-chi0 * L)
        Iref = S * (1 - Tref) + (I0 * Tref if t1 < texit <= t2 else 0.0)
        assert T[0, 0] == pytest.approx(Tref, rel=1e-13, abs=0)
        assert I[0, 0] == pytest.approx(Iref, rel=1e-12, abs=1e-300)
        if t1 >= texit:
            assert I[0, 0] == 0.0 and T[0, 0] == 1.0


@pytest.mark.parametrize("case", ["random2d", "random3d"])
def test_interval_cells_match_exact(orc, case):
    """Static values per adapted cell; the march over [t1, t2] equals the recurrence over the
    exact-rational adapted cells clipped to [t1, t2]."""
    rng = np.random.default_rng({"random2d": 24, "random3d": 25}[case])
    if case == "random2d":
        n, B, nl = (64, 64), 16, 5
        lv = rng.integers(-1, 5, size=16).astype(np.int8)
    else:
        n, B, nl = (16, 16, 16), 8, 4
        lv = rng.integers(-1, 4, size=8).astype(np.int8)
    dim = len(n)
    nvox = int(np.prod(n))
    eta = rng.uniform(0.1, 1.0, size=(1, nvox))
    chi = rng.uniform(0.05, 0.6, size=(1, nvox))
    sc = static_scene(n, B, eta, chi, n_levels=nl)
    dirs = _rand_dirs(rng, dim, 8)
    sc["dirs"] = np.asarray(dirs, np.float32)
    s = orc.Scene(sc)
    tot = s.level_total
    # independent random stored values per level cell (the march only indexes them)
    st_e = rng.uniform(0.1, 1.0, size=(1, tot))
    st_c = rng.uniform(0.05, 0.6, size=(1, tot))
    s.set_static_levels(st_e, st_c)
    offs = np.concatenate([[0], np.cumsum([int(np.prod([v >> m for v in n])) for m in range(nl)])])

    def value(arr, c, m):
        nm = [v >> m for v in n]
        idx = 0
        mul = 1
        for a in range(dim):
            idx += (c[a] >> m) * mul
            mul *= nm[a]
        return arr[0, offs[m] + idx]

    for k, w in enumerate(dirs):
        for _ in range(4):
            pv = tuple(int(rng.integers(0, n[a])) for a in range(dim))
            vox = np.array([pv[0] + n[0] * (pv[1] + (n[1] * pv[2] if dim > 2 else 0))], np.int32)
            t1 = float(rng.uniform(0, 30))
            t2 = t1 + float(rng.uniform(0, 30))
            I, T = orc.march_interval(s, orc.STATIC, lv, vox, np.array([k], np.int32), t1, t2)
            ex = adapted_cells_exact(dim, n, B, lv, pv, w)
            f1, f2 = Fraction(t1), Fraction(t2)
            segs = []
            for cc, L, a, b in ex:
                lo, hi = max(a, f1), min(b, f2)
                if hi > lo:
                    segs.append((cc, L, float(hi - lo)))
            Iref, Tref = 0.0, 1.0
            for cc, L, ln in reversed(segs):
                e, x = value(st_e, cc, L), value(st_c, cc, L)
                Iref = Iref * math.exp(-x * ln) + (e / x) * (-math.expm1(-x * ln))
                Tref *= math.exp(-x * ln)
            assert I[0, 0] == pytest.approx(Iref, rel=1e-12, abs=1e-300), (pv, w, t1, t2)
            assert T[0, 0] == pytest.approx(Tref, rel=1e-12, abs=0)


def test_interval_quadrature(orc):
    """Midpoint quadrature of I = int_{t1}^{t2} eta(x(t)) exp(-int_{t1}^{t} chi) dt, each sample's
    voxel found by flooring x(t): independent of plane crossings and of the recurrence."""
    rng = np.random.default_rng(26)
    n = (16, 16)
    eta = rng.uniform(0.05, 1.0, size=(1, 16, 16))
    chi = rng.uniform(0.05, 0.5, size=(1, 16, 16))
    sc = static_scene(n, 8, eta, chi)
    dirs = _rand_dirs(rng, 2, 6)
    sc["dirs"] = np.asarray(dirs, np.float32)
    s = orc.Scene(sc)
    s.set_static_levels(sc["eta"].astype(np.float64), sc["chi"].astype(np.float64))
    e2, c2 = eta[0], chi[0]  # [y][x]
    for k, w in enumerate(dirs):
        pv = (int(rng.integers(0, 16)), int(rng.integers(0, 16)))
        _, _, to = ray_cells_exact(2, n, pv, w)
        texit = float(to[-1])
        t1 = float(rng.uniform(0, 0.5 * texit))
        t2 = float(rng.uniform(t1, texit + 4))
        I, T = orc.march_interval(s, orc.STATIC, None, np.array([pv[0] + 16 * pv[1]], np.int32),
                                  np.array([k], np.int32), t1, t2)
        L = min(t2, texit) - t1
        m = 400000
        h = L / m
        t = t1 + (np.arange(m) + 0.5) * h
        x = np.floor(pv[0] + 0.5 - t * float(w[0])).astype(int).clip(0, 15)
        y = np.floor(pv[1] + 0.5 - t * float(w[1])).astype(int).clip(0, 15)
        ee, cc = e2[y, x], c2[y, x]
        tau_before = np.concatenate([[0.0], np.cumsum(cc * h)[:-1]])
        Iq = float(np.sum(ee * np.exp(-tau_before) * h))
        Tq = math.exp(-float(np.sum(cc * h)))
        assert I[0, 0] == pytest.approx(Iq, rel=2e-4), (pv, w, t1, t2)
        assert T[0, 0] == pytest.approx(Tq, rel=2e-4)


def test_interval_boundary_intensity_once(orc):
    """I0 enters only through the interval in which the ray leaves the grid."""
    n = (8, 8)
    sc = static_scene(n, 8, np.zeros((1, 64)), np.zeros((1, 64)), I0=2.5)
    sc["dirs"] = np.array([[1.0, 0.0]], np.float32)
    s = orc.Scene(sc)
    s.set_static_levels(sc["eta"].astype(np.float64), sc["chi"].astype(np.float64))
    vox = np.array([5 + 8 * 3], np.int32)  # centre x = 5.5: leaves through x = 0 at t = 5.5
    d = np.zeros(1, np.int32)
    for (t1, t2), want in (((0.0, 5.0), 0.0), ((5.0, 6.0), 2.5), ((5.5, 9.0), 0.0), ((0.0, 5.5), 2.5),
                           ((6.0, 1e9), 0.0)):
        I, T = orc.march_interval(s, orc.STATIC, None, vox, d, t1, t2)
        assert I[0, 0] == want and T[0, 0] == 1.0, (t1, t2)
    with pytest.raises(AssertionError):
        orc.march_interval(s, orc.STATIC, None, vox, d, 3.0, 2.0)


@pytest.mark.parametrize("case", ["random2d", "random3d"])
@pytest.mark.parametrize("sched", [(0, 6, 24, 96, 384), (0, 2.5, 7, 30), (0, 0, 5, 5)])
def test_path_graded_cells_match_exact(orc, case, sched):
    """Path grading: the level cap rises exactly at t = level_dist[m], splitting the voxel piece there."""
    rng = np.random.default_rng({"random2d": 27, "random3d": 28}[case])
    if case == "random2d":
        n, B, nl = (64, 64), 16, 5
        lv = rng.integers(-1, 5, size=16).astype(np.int8)
    else:
        n, B, nl = (16, 16, 16), 8, 4
        lv = rng.integers(-1, 4, size=8).astype(np.int8)
    dim = len(n)
    sc = static_scene(n, B, np.zeros((1,) + n), np.zeros((1,) + n), n_levels=nl)
    s = orc.Scene(sc)
    s.set_level_dist(sched, mode="path")
    nsplit = 0
    for w in _rand_dirs(rng, dim, 8):
        for _ in range(5):
            pv = tuple(int(rng.integers(0, n[a])) for a in range(dim))
            cells, lvl, ti, to = orc.ray_segments(s, lv, pv, w)
            ex = adapted_cells_exact(dim, n, B, lv, pv, w, level_dist=sched, grade="path")
            assert len(ex) == len(cells), (pv, w)
            for i, (cc, L, a, b) in enumerate(ex):
                assert list(cells[i]) == cc and lvl[i] == L
                assert ti[i] == pytest.approx(float(a), rel=1e-14, abs=1e-14)
                assert to[i] == pytest.approx(float(b), rel=1e-14, abs=1e-14)
                nsplit += any(float(a) == x for x in sched[1:])
            ent = adapted_cells_exact(dim, n, B, lv, pv, w, level_dist=sched, grade="entry")
            # entry grading holds each block at the cap of its entry point: never coarser than path grading
            assert sum(float(b - a) * (1 << L) for _, L, a, b in ent) <= sum(
                float(b - a) * (1 << L) for _, L, a, b in ex) + 1e-9
    assert nsplit > 0


def test_path_graded_march_is_composed_cascades(orc):
    """Whole-ray march with path grading {0, 6, 24, 96} = the cascade intervals [0,1.5], [1.5,6], [6,24],
    [24,96], [96,inf) each capped at its cascade level, composed (I = I_a + T_a I_b)."""
    sc, s, lv = _cfg1_static(orc)
    rng = np.random.default_rng(29)
    vox = rng.integers(0, 4096, size=500).astype(np.int32)
    d = rng.integers(0, 8, size=500).astype(np.int32)
    s.set_level_dist((0, 6, 24, 96), mode="path")
    for I0 in (0.0, 0.4):
        s.s.I0 = I0
        I_path = orc.march(s, orc.STATIC, lv, vox, d)
        s.set_level_dist(None)
        ends = [0.0] + CASCADE_ENDS[:4] + [np.inf]
        caps = [0, 0, 1, 2, 3]
        I, T = np.zeros_like(I_path), np.ones_like(I_path)
        for c in range(5):
            Ic, Tc = orc.march_interval(s, orc.STATIC, orc.cap_levels(lv, caps[c]), vox, d, ends[c], ends[c + 1])
            I += T * Ic
            T *= Tc
        np.testing.assert_allclose(I, I_path, rtol=1e-12, atol=1e-300)
        s.set_level_dist((0, 6, 24, 96), mode="path")
        # entry grading is a different (coarser-later) rule: it differs on some rays
        s.set_level_dist((0, 6, 24, 96), mode="entry")
        I_entry = orc.march(s, orc.STATIC, lv, vox, d)
        assert np.any(np.abs(I_entry - I_path) > 1e-9 * np.abs(I_path))
        s.set_level_dist((0, 6, 24, 96), mode="path")
    s.s.I0 = 0.0
