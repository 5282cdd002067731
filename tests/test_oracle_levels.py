"""Pins of the oracle's mip chain, index of dispersion and VLM level selection."""
import json
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def scene(n, B, L):
    dim = len(n)
    n3 = tuple(n) + (1,) * (3 - dim)
    return dict(dim=dim, n=n3, brick=B, n_levels=L, model="static", dirs=np.zeros((1, dim), np.float32),
                ds0=1.0, I0=0.0)


def test_constant_field_mips_equal_the_field(orc):
    """Sect. 2.1: a homogeneous region averages exactly; every active block takes the top level."""
    for n, B, L in (((64, 64), 16, 5), ((32, 32, 32), 8, 4)):
        sc = scene(n, B, L)
        s = orc.Scene(sc)
        nvox = int(np.prod(n))
        nb = int(np.prod([v // B for v in n]))
        act = np.ones(nb, np.uint8)
        act[::3] = 0
        e0, c0 = float(np.float32(0.7)), float(np.float32(3.3))
        lv, oe, oc, clamped = orc.levels_one(s, np.full(nvox, e0), np.full(nvox, c0), act, T=1e-12,
                                             want_values=True)
        assert clamped == 0
        assert np.all(lv[act == 0] == -1) and np.all(lv[act == 1] == L - 1)
        # exp(log(q)) returns q to within 2 ulp
        np.testing.assert_allclose(oe, e0, rtol=4.5e-16, atol=0)
        np.testing.assert_allclose(oc, c0, rtol=4.5e-16, atol=0)
        # a cap limits the level
        lv2 = orc.levels_one(s, np.full(nvox, e0), np.full(nvox, c0), act, T=1e-12, cap=1)
        assert np.all(lv2[act == 1] == 1)


def ramp_iod(m, cx, c, g):
    """Closed form for ln chi = c + g x at level m: the 2^D children differ by
    2^(m-1) in x, so Var = (2^(m-2) g)^2; the mean over [cx, cx + 2^m) is
    c + g (cx + (2^m - 1)/2)."""
    var = (2.0 ** (m - 2) * g) ** 2
    return abs(var / (c + g * (cx + ((1 << m) - 1) / 2.0)))


def ramp_expected(n, B, L, c, g, T):
    nbx, nby = n[0] // B, n[1] // B
    out = np.zeros(nbx * nby, np.int8)
    for bx in range(nbx):
        lv = 0
        for m in range(1, L):
            iods = [ramp_iod(m, cx, c, g) for cx in range(bx * B, (bx + 1) * B, 1 << m)]
            assert all(abs(v - T) > 1e-6 * T for v in iods)
            if max(iods) > T:
                break
            lv = m
        out[bx::nbx] = lv
    return out


def test_linear_ramp_variance(orc):
    """ln chi = c + g x: the IoD at each level follows the closed form; levels agree."""
    n, B, L = (128, 32), 16, 5
    c, g = 3.0, 1.0 / 32.0
    # threshold halfway between two block maxima of the level-3 IoD
    bmax = sorted(max(ramp_iod(3, cx, c, g) for cx in range(bx * B, (bx + 1) * B, 8)) for bx in range(8))
    T = 0.5 * (bmax[3] + bmax[4])
    xs = np.arange(n[0])
    lnchi = c + g * xs[None, :] * np.ones((n[1], 1))
    chi = np.exp(lnchi).reshape(-1)
    eta = np.full(chi.size, 2.0)
    s = orc.Scene(scene(n, B, L))
    lv = orc.levels_one(s, eta, chi, np.ones(16, np.uint8), T=T, tau_thin=0.25)
    exp = ramp_expected(n, B, L, c, g, T)
    assert np.array_equal(lv, exp), (lv, exp)
    assert len(set(exp.tolist())) > 1  # the ramp separates the blocks


def test_iod_hand_case(orc):
    """Children ln chi = {1, 3, 1, 3}: mean 2, population variance 1, IoD 0.5."""
    n, B, L = (2, 2), 2, 2
    sc = scene(n, B, L)
    s = orc.Scene(sc)
    chi = np.exp(np.array([1.0, 3.0, 1.0, 3.0]))
    eta = np.full(4, 5.0)
    assert orc.levels_one(s, eta, chi, np.ones(1, np.uint8), T=0.49)[0] == 0
    assert orc.levels_one(s, eta, chi, np.ones(1, np.uint8), T=0.51)[0] == 1
    # mean of ln values exactly 0 with a spread: IoD infinite, never merged
    chi0 = np.exp(np.array([-1.0, 1.0, -1.0, 1.0]))
    assert orc.levels_one(s, np.full(4, 5.0), chi0, np.ones(1, np.uint8), T=1e300)[0] == 0
    # identical children: Var = 0 -> IoD 0 even at T = 0
    assert orc.levels_one(s, np.full(4, 5.0), np.full(4, 7.0), np.ones(1, np.uint8), T=0.0)[0] == 1


def test_thin_bypass(orc):
    """Sect. 2.2: cells with chi ds < 0.25 are always averaged, whatever their IoD."""
    rng = np.random.default_rng(4)
    n, B, L = (32, 32), 16, 5
    sc = scene(n, B, L)
    s = orc.Scene(sc)
    eta = np.exp(rng.normal(0, 3, size=32 * 32))  # wildly varying: IoD fails everywhere
    for chi0, expect in ((0.01, 4), (0.05, 2), (0.2, 0), (0.1, 1)):
        # chi * 2^m < 0.25 holds up to m = floor(log2(0.25 / chi))
        lv = orc.levels_one(s, eta, np.full(32 * 32, chi0), np.ones(4, np.uint8), T=1e-3)
        assert np.all(lv == expect), (chi0, lv)


def test_thin_bypass_uses_box_filtered_chi(orc):
    """The thin test measures a merged cell's optical side with the box-filtered (arithmetic mean) chi of Sect. 2.1:
    one dense voxel among thin ones keeps its block at full resolution, even though the geometric mean of chi
    (the stored value in LOG mode) is far below the threshold."""
    n, B, L = (2, 2), 2, 2
    s = orc.Scene(scene(n, B, L), avg_mode=orc.AVG_LOG)
    eta = np.array([1.0, 1e-3, 2e-3, 3e-3])  # IoD of ln eta fails
    chi = np.array([0.2, 1e-6, 1e-6, 1e-6])  # mean 0.05 -> 0.05 x 2 = 0.1 < 0.25; geometric mean ~ 1e-5
    assert orc.levels_one(s, eta, chi, np.ones(1, np.uint8), T=1e-2)[0] == 1
    chi = np.array([0.6, 1e-6, 1e-6, 1e-6])  # mean 0.15 -> 0.3 >= 0.25: not thin, IoD decides -> level 0
    assert orc.levels_one(s, eta, chi, np.ones(1, np.uint8), T=1e-2)[0] == 0
    # the same cell with a uniform thin chi is averaged
    assert orc.levels_one(s, eta, np.full(4, 0.1), np.ones(1, np.uint8), T=1e-2)[0] == 1


def test_state_packing_512(orc):
    """3 bits per block, 21 blocks per 64-bit word: 512^2 with 16^2 blocks -> 49 words, 392 B."""
    g = json.load(open(os.path.join(GOLD, "block_state_packing.json")))
    nb = (g["grid"][0] // g["brick"]) * (g["grid"][1] // g["brick"])
    rng = np.random.default_rng(0)
    lv = rng.integers(-1, 5, size=nb)
    words = orc.pack_states(lv)
    assert words.size == g["words"] and words.nbytes == g["bytes"]
    # unpack
    back = np.array([int((int(words[b // 21]) >> (3 * (b % 21))) & 7) - 1 for b in range(nb)])
    assert np.array_equal(back, lv)
    assert int(words[-1]) >> (3 * (nb - 21 * (g["words"] - 1))) == 0  # unused high bits stay clear


def test_mip_storage_factors(orc):
    """Sect. 2.1: whole chain costs 1.33x MIP 0 in 2D (levels 0-4) and 1.14x in 3D (levels 0-3)."""
    g = json.load(open(os.path.join(GOLD, "block_state_packing.json")))
    s2 = orc.Scene(scene((512, 512), 16, 5))
    assert round(s2.level_total / 512 ** 2, 2) == g["mip_storage_factor_2d_levels_0_4"]
    s3 = orc.Scene(scene((64, 64, 64), 8, 4))
    assert round(s3.level_total / 64 ** 3, 2) == g["mip_storage_factor_3d"]


def test_level_values_log_and_linear(orc):
    """Level-1 stored value of children {a, b, c, d}: geometric mean (LOG) or arithmetic mean (LINEAR)."""
    n, B, L = (2, 2), 2, 2
    q = np.array([1.0, 2.0, 4.0, 8.0])
    s = orc.Scene(scene(n, B, L), avg_mode=orc.AVG_LOG)
    _, oe, oc, _ = orc.levels_one(s, q, q * 3, np.ones(1, np.uint8), T=1.0, want_values=True)
    assert oe[4] == pytest.approx(64.0 ** 0.25, rel=1e-15)
    assert oc[4] == pytest.approx(3 * 64.0 ** 0.25, rel=1e-15)
    s = orc.Scene(scene(n, B, L), avg_mode=orc.AVG_LINEAR)
    _, oe, oc, _ = orc.levels_one(s, q, q * 3, np.ones(1, np.uint8), T=1.0, want_values=True)
    assert oe[4] == 3.75 and oc[4] == 11.25


def test_zero_in_active_block_is_clamped_and_counted(orc):
    n, B, L = (4, 4), 4, 3
    s = orc.Scene(scene(n, B, L))
    e = np.ones(16)
    c = np.ones(16)
    c[5] = 0.0
    lv, _, _, clamped = orc.levels_one(s, e, c, np.ones(1, np.uint8), T=1.0, want_values=True)
    assert clamped == 1  # flagged; a zero child makes the log mean tiny (thin), so no level is asserted


def test_morton_order_pins():
    """Sect. 2.3.1 orders active blocks by Morton code: the z-order of a 4 x 4 and a 2 x 2 x 2 block grid
    written out by hand, and the probe order of an all-probes trace (blocks in that order, voxels x fastest)."""
    from oracle.order import morton_order, probe_voxels
    assert list(morton_order((4, 4))) == [0, 1, 4, 5, 2, 3, 6, 7, 8, 9, 12, 13, 10, 11, 14, 15]
    assert list(morton_order((2, 2, 2))) == [0, 1, 2, 3, 4, 5, 6, 7]
    # 4 x 2: x has two bits, y one; codes x0 | y0 << 1 | x1 << 2
    assert list(morton_order((4, 2))) == [0, 1, 4, 5, 2, 3, 6, 7]
    sc = dict(dim=2, n=(4, 4, 1), brick=2, block_active=np.array([0, 1, 1, 1], np.uint8))
    assert list(probe_voxels(sc)) == [2, 3, 6, 7, 8, 9, 12, 13, 10, 11, 14, 15]
