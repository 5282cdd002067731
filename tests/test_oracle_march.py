"""Pins of the oracle's traversal and piecewise-constant march (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

from oracle.exact import adapted_cells_exact, ray_cells_exact

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def static_scene(n, B, eta, chi, I0=0.0, n_levels=1):
    """Single-resolution static scene dict with per-wavelength arrays [n_lam][nvox]."""
    dim = len(n)
    n3 = tuple(n) + (1,) * (3 - dim)
    eta = np.asarray(eta, np.float32).reshape(eta.shape[0], -1)
    chi = np.asarray(chi, np.float32).reshape(chi.shape[0], -1)
    nb = int(np.prod([v // B for v in n]))
    return dict(dim=dim, n=n3, brick=B, n_levels=n_levels, model="static", eta=eta, chi=chi,
                dirs=np.zeros((1, dim), np.float32), block_active=np.ones(nb, np.uint8), ds0=1.0, I0=I0)


# ---------------------------------------------------------------------------
def test_homogeneous_slab_closed_form(orc):
    """I = I0 exp(-chi L) + S (1 - exp(-chi L)) for any subdivision of the path (Eq. RteIntegral)."""
    rng = np.random.default_rng(11)
    n = (16, 16)
    eta0, chi0, I0 = float(np.float32(0.37)), float(np.float32(0.23)), 0.8
    sc = static_scene(n, 8, np.full((1, 16, 16), eta0), np.full((1, 16, 16), chi0), I0=I0)
    for trial in range(40):
        pv = (int(rng.integers(0, 16)), int(rng.integers(0, 16)))
        th = rng.uniform(0, 2 * np.pi)
        w = np.array([np.cos(th), np.sin(th)], np.float32)
        if trial == 0:
            w = np.array([1.0, 0.0], np.float32)
        if trial == 1:
            w = np.array([math.sqrt(0.5), math.sqrt(0.5)], np.float32)
        sc["dirs"] = w[None]
        s = orc.Scene(sc)
        s.set_static_levels(sc["eta"].astype(np.float64), sc["chi"].astype(np.float64))
        vox = np.array([pv[0] + 16 * pv[1]], np.int32)
        I = orc.march(s, orc.STATIC, None, vox, np.zeros(1, np.int32))[0, 0]
        _, ti, to = ray_cells_exact(2, n, pv, w)
        L = float(to[-1])
        S = eta0 / chi0
        Iref = I0 * math.exp(-chi0 * L) + S * (1 - math.exp(-chi0 * L))
        assert I == pytest.approx(Iref, rel=1e-13, abs=0)


def test_pass_through_empty_space(orc):
    """eta = chi = 0 everywhere: the boundary intensity arrives unchanged, bit for bit."""
    rng = np.random.default_rng(12)
    n = (8, 8, 8)
    for I0 in (0.0, 1.0, 3.141592653589793):
        sc = static_scene(n, 8, np.zeros((2, 512)), np.zeros((2, 512)), I0=I0)
        dirs = rng.normal(size=(5, 3))
        dirs = (dirs / np.linalg.norm(dirs, axis=1, keepdims=True)).astype(np.float32)
        sc["dirs"] = dirs
        s = orc.Scene(sc)
        s.set_static_levels(sc["eta"].astype(np.float64), sc["chi"].astype(np.float64))
        vox = rng.integers(0, 512, size=5).astype(np.int32)
        I = orc.march(s, orc.STATIC, None, vox, np.arange(5, dtype=np.int32))
        assert np.all(I == I0)


def test_two_slab_order_dependence(orc):
    """Voxel values of the worked example (S = 10, chi = 0.2 vs S = 2/7, chi = 1.4):
    light-then-dark differs from dark-then-light (Sect. 1.1), each matching the
    two-slab closed form."""
    g = json.load(open(os.path.join(GOLD, "worked_example_t1.json")))["voxels"]
    g = {k: float(np.float32(v)) for k, v in g.items()}
    n = (16, 16)
    eta = np.zeros((1, 16, 16))
    chi = np.zeros((1, 16, 16))
    eta[0, :, :8], chi[0, :, :8] = g["eta_AB"], g["chi_AB"]
    eta[0, :, 8:], chi[0, :, 8:] = g["eta_CD"], g["chi_CD"]
    sc = static_scene(n, 8, eta, chi)
    SA, tA = g["eta_AB"] / g["chi_AB"], g["chi_AB"]
    SC, tC = g["eta_CD"] / g["chi_CD"], g["chi_CD"]
    # probe at x = 15 (dark side), light along +x: upwind path 8 light then 7.5 dark
    sc["dirs"] = np.array([[1.0, 0.0], [-1.0, 0.0]], np.float32)
    s = orc.Scene(sc)
    s.set_static_levels(eta.reshape(1, -1), chi.reshape(1, -1))
    I = orc.march(s, orc.STATIC, None, np.array([15 + 16 * 3, 0 + 16 * 3], np.int32), np.array([0, 1], np.int32))
    I1 = SA * (1 - math.exp(-tA * 8))
    ref_ld = I1 * math.exp(-tC * 7.5) + SC * (1 - math.exp(-tC * 7.5))
    I2 = SC * (1 - math.exp(-tC * 8))
    ref_dl = I2 * math.exp(-tA * 7.5) + SA * (1 - math.exp(-tA * 7.5))
    assert I[0, 0] == pytest.approx(ref_ld, rel=1e-13)
    assert I[1, 0] == pytest.approx(ref_dl, rel=1e-13)
    assert abs(I[0, 0] - I[1, 0]) > 1.0


def test_worked_example_average_column(orc):
    """Table 1 'Average' column: homogeneous eta = 1.2, chi = 0.8 over path
    lengths sqrt(6), sqrt(5), sqrt(6)/2 gives 1.29, 1.25, 0.94."""
    g = json.load(open(os.path.join(GOLD, "worked_example_t1.json")))
    eb, cb = g["average"]["eta"], g["average"]["chi"]
    printed = g["average_column"]
    n = (8, 8)
    sc = static_scene(n, 8, np.full((1, 8, 8), eb), np.full((1, 8, 8), cb))
    for name, L in (("alpha", math.sqrt(6)), ("gamma", math.sqrt(5)), ("delta", math.sqrt(6) / 2)):
        # probe (0, 7): exits through x = 0 after 0.5/w_x when 0.5/w_x * w_y < 7.5
        wx = 0.5 / L
        w = np.array([wx, math.sqrt(1 - wx * wx)], np.float32)
        sc["dirs"] = w[None]
        s = orc.Scene(sc)
        s.set_static_levels(sc["eta"].astype(np.float64), sc["chi"].astype(np.float64))
        I = orc.march(s, orc.STATIC, None, np.array([0 + 8 * 7], np.int32), np.zeros(1, np.int32))[0, 0]
        assert round(I, 2) == pytest.approx(printed[name], abs=1e-12)


def _rand_dirs(rng, dim, k):
    d = rng.normal(size=(k, dim))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    special = []
    for a in range(dim):
        e = np.zeros(dim)
        e[a] = 1
        special += [e, -e]
    if dim == 2:
        s = math.sqrt(0.5)
        special += [np.array([s, s]), np.array([-s, s]), np.array([0.6, -0.8])]
    else:
        s = 1 / math.sqrt(3)
        special += [np.array([s, s, s]), np.array([-s, s, -s]), np.array([0.6, 0.8, 0.0]), np.array([0.0, -0.6, 0.8])]
    return np.concatenate([d, np.array(special)]).astype(np.float32)


@pytest.mark.parametrize("n", [(8, 8), (16, 16), (12, 20), (8, 8, 8), (8, 16, 8)])
def test_dense_cells_match_exact_rationals(orc, n):
    rng = np.random.default_rng(hash(n) % 2 ** 32)
    dim = len(n)
    for w in _rand_dirs(rng, dim, 12):
        for _ in range(4):
            pv = tuple(int(rng.integers(0, n[a])) for a in range(dim))
            cells, ti, to = orc.ray_cells(dim, n, pv, w)
            ec, eti, eto = ray_cells_exact(dim, n, pv, w)
            assert len(cells) == len(ec), (pv, w)
            assert np.array_equal(cells, np.array(ec, np.int32)), (pv, w)
            np.testing.assert_allclose(ti, [float(x) for x in eti], rtol=1e-14, atol=1e-14)
            np.testing.assert_allclose(to, [float(x) for x in eto], rtol=1e-14, atol=1e-14)


def hdda_example_levels():
    g = json.load(open(os.path.join(GOLD, "hdda_example_blocks.json")))
    lv = np.zeros(16, np.int8)
    for b in g["empty_blocks"]:
        lv[b] = -1
    for b, cps in g["block_cells_per_side"].items():
        lv[int(b)] = int(round(math.log2(g["brick"] // cps)))
    return lv


def test_hdda_example_block_map():
    lv = hdda_example_levels()
    assert lv[9] == 1 and lv[10] == 2 and (lv == -1).sum() == 7 and (lv == 0).sum() == 7


@pytest.mark.parametrize("case", ["example", "random2d", "random3d"])
def test_adapted_cells_match_exact(orc, case):
    rng = np.random.default_rng({"example": 1, "random2d": 2, "random3d": 3}[case])
    if case == "example":
        n, B, lv = (32, 32), 8, hdda_example_levels()
    elif case == "random2d":
        n, B = (64, 64), 16
        lv = rng.integers(-1, 5, size=16).astype(np.int8)
    else:
        n, B = (16, 16, 16), 8
        lv = rng.integers(-1, 4, size=8).astype(np.int8)
    dim = len(n)
    sc = static_scene(n, B, np.zeros((1,) + n), np.zeros((1,) + n), n_levels=5)
    s = orc.Scene(sc)
    for w in _rand_dirs(rng, dim, 10):
        for _ in range(5):
            pv = tuple(int(rng.integers(0, n[a])) for a in range(dim))
            cells, lvl, ti, to = orc.ray_segments(s, lv, pv, w)
            ex = adapted_cells_exact(dim, n, B, lv, pv, w)
            assert len(ex) == len(cells)
            for i, (cc, L, a, b) in enumerate(ex):
                assert list(cells[i]) == cc and lvl[i] == L
                assert ti[i] == pytest.approx(float(a), rel=1e-14, abs=1e-14)
                assert to[i] == pytest.approx(float(b), rel=1e-14, abs=1e-14)


@pytest.mark.parametrize("sched", [(0, 6, 24, 96, 384), (0, 2, 8, 32), (0, 0, 5, 5)])
def test_graded_cap_matches_exact(orc, sched):
    """Distance-graded cap: a block's level is capped by the path length at which the ray enters it."""
    rng = np.random.default_rng(11)
    n, B = (64, 64), 16
    lv = rng.integers(-1, 5, size=16).astype(np.int8)
    sc = static_scene(n, B, np.zeros((1,) + n), np.zeros((1,) + n), n_levels=5)
    s = orc.Scene(sc)
    s.set_level_dist(sched)
    for w in _rand_dirs(rng, 2, 10):
        for _ in range(5):
            pv = (int(rng.integers(0, 64)), int(rng.integers(0, 64)))
            cells, lvl, ti, to = orc.ray_segments(s, lv, pv, w)
            ex = adapted_cells_exact(2, n, B, lv, pv, w, level_dist=sched)
            assert len(ex) == len(cells)
            for i, (cc, L, a, b) in enumerate(ex):
                assert list(cells[i]) == cc and lvl[i] == L
    # the probe's own block is never coarsened when level_dist[1] > 0
    if sched[1] > 0:
        for _ in range(50):
            pv = (int(rng.integers(0, 64)), int(rng.integers(0, 64)))
            cells, lvl, ti, to = orc.ray_segments(s, lv, pv, np.array([0.6, 0.8], np.float32))
            if len(lvl) and ti[0] == 0.0:
                assert lvl[0] == 0


def test_single_resolution_is_aw87(orc):
    """All levels 0 and no empty blocks: the adapted list is the dense list (Sect. 2.3)."""
    rng = np.random.default_rng(5)
    n, B = (32, 32), 8
    sc = static_scene(n, B, np.zeros((1,) + n), np.zeros((1,) + n), n_levels=4)
    s = orc.Scene(sc)
    lv = np.zeros(16, np.int8)
    for w in _rand_dirs(rng, 2, 10):
        pv = (int(rng.integers(0, 32)), int(rng.integers(0, 32)))
        c1, l1, a1, b1 = orc.ray_segments(s, lv, pv, w)
        c2, a2, b2 = orc.ray_cells(2, n, pv, w)
        assert np.array_equal(c1, c2) and np.all(l1 == 0)
        assert np.array_equal(a1, a2) and np.array_equal(b1, b2)


def test_vlm_all_level0_equals_dense_bitwise(orc):
    """With every block at level 0 the VLM march is the dense march bit for bit."""
    from synth import make_cfg1
    sc = make_cfg1()
    s = orc.Scene(sc)
    lvs, st_e, st_c = orc.static_level_values(s, sc["eta"], sc["chi"], np.ones(64, np.uint8), T=1e-2)
    s.set_static_levels(st_e, st_c)
    rng = np.random.default_rng(3)
    vox = rng.integers(0, 4096, size=300).astype(np.int32)
    d = rng.integers(0, 8, size=300).astype(np.int32)
    I_dense = orc.march(s, orc.STATIC, None, vox, d)
    I_l0 = orc.march(s, orc.STATIC, np.zeros(64, np.int8), vox, d)
    assert np.array_equal(I_dense, I_l0)
