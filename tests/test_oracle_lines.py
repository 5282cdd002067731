"""Pins of the oracle's line model: Voigt function, Doppler shift, velocity
interpolation and Core-and-Voigt (CPU only)."""
import math

import numpy as np
import pytest
from scipy.special import erfcx, wofz

from synth import C_KMS


def tiny_lines_scene(n=(32, 32), B=8, L=3, profile="gauss", seed=0, vmax=20.0, n_lines=1, uniform_v=None,
                     lam0=(500.0,), n_lam=12, dv_span=40.0):
    rng = np.random.default_rng(seed)
    dim = len(n)
    nvox = int(np.prod(n))
    n3 = tuple(n) + (1,) * (3 - dim)
    chi_star = np.exp(rng.normal(-1.0, 0.7, size=(n_lines, nvox)))
    S = np.exp(-1.0 / rng.uniform(0.5, 2.0, size=nvox))
    eta_star = chi_star * S
    chi_bg = np.exp(rng.normal(-5.0, 0.3, size=nvox))
    eta_bg = chi_bg * S
    vth = 8.0
    lam0 = np.array(lam0[:n_lines], np.float64)
    inv_dld = np.stack([np.full(nvox, C_KMS / (l0 * vth)) for l0 in lam0])
    damp = np.exp(rng.uniform(np.log(1e-3), np.log(1e-1), size=(n_lines, nvox)))
    if uniform_v is not None:
        vel = np.stack([np.full(nvox, uniform_v[a]) for a in range(dim)])
    else:
        vel = rng.uniform(-vmax / math.sqrt(dim), vmax / math.sqrt(dim), size=(dim, nvox))
    dv = np.linspace(-dv_span, dv_span, n_lam)
    lam = np.concatenate([l0 * (1.0 + dv / C_KMS) for l0 in lam0])
    th = 2 * np.pi * (np.arange(8) + 0.5) / 8
    dirs = np.stack([np.cos(th), np.sin(th)], 1).astype(np.float32) if dim == 2 else \
        (lambda d: (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32))(rng.normal(size=(8, 3)))
    nb = int(np.prod([v // B for v in n]))
    f = lambda a: np.ascontiguousarray(a, np.float32)  # noqa: E731
    return dict(dim=dim, n=n3, brick=B, n_levels=L, model="lines", profile=profile, lam=lam, lam0=lam0,
                eta_star=f(eta_star), chi_star=f(chi_star), damp=f(damp), inv_dld=f(inv_dld), eta_bg=f(eta_bg),
                chi_bg=f(chi_bg), vel=f(vel), dirs=dirs, block_active=np.ones(nb, np.uint8), ds0=1.0, I0=0.0)


# ---------------------------------------------------------------------------
# Voigt
# ---------------------------------------------------------------------------
def test_voigt_matches_scipy_faddeeva(orc):
    x = np.linspace(-60, 60, 4001)
    for a in (1e-4, 1e-3, 1e-2, 0.1, 0.5, 1.0):
        H = orc.voigt_h(a, x)
        ref = wofz(x + 1j * a).real
        assert np.max(np.abs(H - ref) / ref) < 1e-9, a


def test_voigt_special_cases(orc):
    x = np.linspace(-6, 6, 241)
    # a = 0: Gaussian
    np.testing.assert_allclose(orc.voigt_h(0.0, x), np.exp(-x * x), rtol=1e-10, atol=1e-15)
    # x = 0: exp(a^2) erfc(a)
    a = np.array([1e-3, 0.01, 0.1, 0.5, 1.0, 2.0])
    np.testing.assert_allclose(orc.voigt_h(a, 0.0), erfcx(a), rtol=1e-10)
    # far wing: w ~ i / (sqrt(pi) z)  ->  H ~ a / (sqrt(pi) (a^2 + x^2))
    a0, xw = 0.05, 400.0
    assert orc.voigt_h(a0, xw) == pytest.approx(a0 / (math.sqrt(math.pi) * (a0 ** 2 + xw ** 2)), rel=1e-4)
    # normalisation: integral of H over x is sqrt(pi)
    xs = np.linspace(-2000, 2000, 400001)
    I = np.trapezoid(orc.voigt_h(0.02, xs), xs)
    assert I == pytest.approx(math.sqrt(math.pi), rel=2e-5)


def test_cav_wavelength_scalings(orc):
    """Sect. 3.2: eta*, chi* scale as lam0/lam and the damping as (lam/lam0)^2.
    Checked in the Lorentzian wing, where H ~ a(lam) / (sqrt(pi) x^2)."""
    sc = tiny_lines_scene(n=(8, 8), B=8, L=1, profile="voigt", uniform_v=(0.0, 0.0))
    nvox = 64
    lam0, lam = 1.0, 1.2
    sc["lam0"] = np.array([lam0])
    sc["lam"] = np.array([lam])
    inv_dld, a0, chis = 250.0, 0.02, 3.0
    sc["inv_dld"][:] = inv_dld
    sc["damp"][:] = a0
    sc["chi_star"][:] = chis
    sc["chi_bg"][:] = 0.0
    sc["eta_bg"][:] = 0.0
    s = orc.Scene(sc)
    e, c = orc.lines_mip0(s, 0, 0)
    x = (lam - lam0) * inv_dld
    aL = a0 * (lam / lam0) ** 2
    H = aL / (math.sqrt(math.pi) * (aL * aL + x * x)) * (1 + 1.5 / x ** 2)
    expect = (lam0 / lam) * chis * H * inv_dld / math.sqrt(math.pi)
    np.testing.assert_allclose(c, expect, rtol=2e-4)
    assert c.shape == (nvox,)


def test_line_centre_normalisation(orc):
    """At the rest wavelength and zero velocity: chi = bg + chi* H(a,0)/(sqrt(pi) dlD) (Voigt),
    chi = bg + chi* (peak-normalised Gaussian)."""
    for prof in ("voigt", "gauss"):
        sc = tiny_lines_scene(n=(8, 8), B=8, L=1, profile=prof, uniform_v=(0.0, 0.0))
        sc["lam"] = np.array([sc["lam0"][0]])
        s = orc.Scene(sc)
        e, c = orc.lines_mip0(s, 0, 0)
        cs = sc["chi_star"][0].astype(np.float64)
        bg = sc["chi_bg"].astype(np.float64)
        if prof == "voigt":
            peak = erfcx(sc["damp"][0].astype(np.float64)) * sc["inv_dld"][0].astype(np.float64) / math.sqrt(math.pi)
        else:
            peak = 1.0
        np.testing.assert_allclose(c, bg + cs * peak, rtol=1e-9)


# ---------------------------------------------------------------------------
# Doppler shift
# ---------------------------------------------------------------------------
def test_uniform_velocity_is_a_wavelength_shift(orc):
    """Classic march with uniform v along w at lam equals the v = 0 march at
    lam' = lam + lam0 u / c (profile argument lam + (v.w/c) lam0, Sect. 3.2)."""
    v = (12.0, -7.0)
    scv = tiny_lines_scene(n=(16, 16), B=8, L=1, profile="gauss", uniform_v=v)
    sc0 = tiny_lines_scene(n=(16, 16), B=8, L=1, profile="gauss", uniform_v=(0.0, 0.0))
    w = scv["dirs"][3].astype(np.float64)
    u = v[0] * w[0] + v[1] * w[1]
    lam0 = scv["lam0"][0]
    sc0["lam"] = scv["lam"] + lam0 * u / C_KMS
    s_v, s_0 = orc.Scene(scv), orc.Scene(sc0)
    vox = np.arange(0, 256, 7).astype(np.int32)
    d = np.full(vox.size, 3, np.int32)
    Iv = orc.march(s_v, orc.CLASSIC, None, vox, d)
    I0 = orc.march(s_0, orc.CLASSIC, None, vox, d)
    np.testing.assert_allclose(Iv, I0, rtol=1e-9)
    # the opposite sign would not agree
    sc0["lam"] = scv["lam"] - lam0 * u / C_KMS
    I0b = orc.march(orc.Scene(sc0), orc.CLASSIC, None, vox, d)
    assert np.max(np.abs(I0b - Iv) / np.abs(Iv)) > 1e-2


def test_core_closest_shift_rule(orc):
    """Sect. 3.2 IoD frame: each line is shifted by the velocity in [-|v|, |v|]
    nearest the line core; reachable cores give chi = bg + chi* exactly (Gaussian peak)."""
    sc = tiny_lines_scene(n=(8, 8), B=8, L=1, profile="gauss", uniform_v=(3.0, 4.0))  # |v| = 5
    lam0 = sc["lam0"][0]
    sc["lam"] = np.array([lam0 * (1 - 4.0 / C_KMS), lam0 * (1 - 9.0 / C_KMS)])
    s = orc.Scene(sc)
    e, c = orc.lines_mip0(s, 0, 1)
    np.testing.assert_allclose(c, sc["chi_bg"].astype(np.float64) + sc["chi_star"][0], rtol=1e-12)
    e2, c2 = orc.lines_mip0(s, 1, 1)
    x = 4.0 / 8.0  # clamped at u = 5: offset 4 km/s over a thermal width of 8 km/s
    np.testing.assert_allclose(c2, sc["chi_bg"].astype(np.float64) + sc["chi_star"][0] * math.exp(-x * x),
                               rtol=1e-6)


# ---------------------------------------------------------------------------
# velocity interpolation and Core-and-Voigt
# ---------------------------------------------------------------------------
def _rest_static_levels(orc, sc, s, lam_count, T=1e-2):
    lvs, st_e, st_c = [], [], []
    for il in range(lam_count):
        e0, c0 = orc.lines_mip0(s, il, 0)
        lv, oe, oc, _ = orc.levels_one(s, e0, c0, sc["block_active"], T, 0.25, -1, want_values=True)
        lvs.append(lv)
        st_e.append(oe)
        st_c.append(oc)
    return orc.batch_levels(lvs), np.array(st_e), np.array(st_c)


def test_velinterp_zero_velocity_is_the_static_march(orc):
    """v = 0: every node grid collapses (V = 0) and velocity interpolation is the
    rest-frame VLM march."""
    sc = tiny_lines_scene(n=(32, 32), B=8, L=4, profile="gauss", uniform_v=(0.0, 0.0), n_lam=6)
    s = orc.Scene(sc)
    lv, st_e, st_c = _rest_static_levels(orc, sc, s, s.s.n_lam, T=5.0)
    assert lv.max() > 0
    rng = np.random.default_rng(1)
    vox = rng.integers(0, 1024, 60).astype(np.int32)
    d = rng.integers(0, 8, 60).astype(np.int32)
    Ivi = orc.march(s, orc.VELINTERP, lv, vox, d)
    s.set_static_levels(st_e, st_c)
    Ist = orc.march(s, orc.STATIC, lv, vox, d)
    np.testing.assert_allclose(Ivi, Ist, rtol=1e-12)


def test_velinterp_converges_second_order(orc):
    """Linear interpolation between n_v nodes: the error against the Classic march
    at level 0 falls ~4x per halving of the node spacing."""
    sc = tiny_lines_scene(n=(16, 16), B=8, L=1, profile="gauss", vmax=25.0, n_lam=8, dv_span=25.0)
    rng = np.random.default_rng(2)
    vox = rng.integers(0, 256, 80).astype(np.int32)
    d = rng.integers(0, 8, 80).astype(np.int32)
    ref = orc.march(orc.Scene(sc), orc.CLASSIC, None, vox, d)
    errs = []
    for nv in (9, 17, 33, 65):
        I = orc.march(orc.Scene(sc, n_v=nv), orc.VELINTERP, None, vox, d)
        errs.append(np.max(np.abs(I - ref) / np.abs(ref)))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert errs[-1] < 1e-2
    assert all(3.0 < r < 5.5 for r in ratios), (errs, ratios)


def test_cav_level0_is_classic(orc):
    """Core and Voigt at MIP 0 evaluates each voxel's own parameters: identical to Classic."""
    for prof in ("gauss", "voigt"):
        sc = tiny_lines_scene(n=(16, 16), B=8, L=3, profile=prof, n_lines=2, lam0=(500.0, 500.1))
        s = orc.Scene(sc)
        rng = np.random.default_rng(3)
        vox = rng.integers(0, 256, 40).astype(np.int32)
        d = rng.integers(0, 8, 40).astype(np.int32)
        I_c = orc.march(s, orc.CLASSIC, None, vox, d)
        I_cav = orc.march(s, orc.CAV, np.zeros(4, np.int8), vox, d)
        assert np.array_equal(I_c, I_cav)


def test_cav_constant_parameters_any_level(orc):
    """Homogeneous line parameters: Core-and-Voigt at any level equals Classic (Sect. 1.1:
    averaging homogeneous parameters is exact)."""
    sc = tiny_lines_scene(n=(16, 16), B=8, L=4, profile="voigt", uniform_v=(5.0, -3.0))
    for k in ("eta_star", "chi_star", "damp", "inv_dld"):
        sc[k][:] = sc[k][0, 0]
    for k in ("eta_bg", "chi_bg"):
        sc[k][:] = sc[k][0]
    s = orc.Scene(sc)
    rng = np.random.default_rng(4)
    vox = rng.integers(0, 256, 40).astype(np.int32)
    d = rng.integers(0, 8, 40).astype(np.int32)
    I_c = orc.march(s, orc.CLASSIC, None, vox, d)
    I_cav = orc.march(s, orc.CAV, np.full(4, 3, np.int8), vox, d)
    np.testing.assert_allclose(I_cav, I_c, rtol=1e-12)


# ---------------------------------------------------------------------------
# velocity interpolation at merged levels (Sect. 3.1; orthant grids, Sect. 4.1)
# ---------------------------------------------------------------------------
AXIS_DIRS = np.array([[1.0, 0.0], [-1.0, 0.0], [0.0, 1.0], [0.0, -1.0]], np.float32)


def _shifted_static_march(orc, sc, u, level, vox, d):
    """The static march, every block at `level`, of the scene with v = 0 observed at
    lam' = lam + lam0 u / c (a uniform projected velocity u is a pure wavelength shift),
    whose level values are box filters of the MIP-0 values: what a velocity-interpolation
    node at projected velocity u holds."""
    sc0 = dict(sc)
    sc0["vel"] = np.zeros_like(sc["vel"])
    sc0["lam"] = sc["lam"] + sc["lam0"][0] * u / C_KMS
    s0 = orc.Scene(sc0)
    lvs, st_e, st_c = orc.static_level_values(s0, np.array([orc.lines_mip0(s0, il, 0)[0] for il in range(s0.s.n_lam)]),
                                              np.array([orc.lines_mip0(s0, il, 0)[1] for il in range(s0.s.n_lam)]),
                                              sc["block_active"], T=0.0)
    s0.set_static_levels(st_e, st_c)
    lv = np.full(sc["block_active"].size, level, np.int8)
    return orc.march(s0, orc.STATIC, lv, vox, d)


@pytest.mark.parametrize("vgrid,n_v", [("full", 9), ("orthant", 9)])
def test_velinterp_uniform_velocity_node_any_level(orc, vgrid, n_v):
    """Uniform v along x: rays along +-x project u = +-V, the end nodes of the full
    grid and of both x-orthant grids; rays along y project u = 0, the middle node of
    the full grid and an end node of the orthant grids.  At every level the
    velocity-interpolation march then equals the static march of the Doppler-shifted
    scene with box-filtered level values."""
    V = 12.0
    sc = tiny_lines_scene(n=(32, 32), B=8, L=4, profile="gauss", uniform_v=(V, 0.0), n_lam=6)
    sc["dirs"] = AXIS_DIRS
    s = orc.Scene(sc, n_v=n_v, vgrid=vgrid)
    rng = np.random.default_rng(5)
    vox = rng.integers(0, 1024, 48).astype(np.int32)
    for d_idx in range(4):
        u = float(np.dot(np.array([V, 0.0]), AXIS_DIRS[d_idx].astype(np.float64)))
        d = np.full(vox.size, d_idx, np.int32)
        for level in range(4):
            lv = np.full(16, level, np.int8)
            got = orc.march(s, orc.VELINTERP, lv, vox, d)
            ref = _shifted_static_march(orc, sc, u, level, vox, d)
            np.testing.assert_allclose(got, ref, rtol=1e-9, err_msg="%s dir %d level %d" % (vgrid, d_idx, level))


@pytest.mark.parametrize("vgrid,n_v", [("full", 7), ("orthant", 5)])
def test_velinterp_mixed_speeds_in_a_cell(orc, vgrid, n_v):
    """Cells mixing speeds: v_x = -1 on voxels with even x and y, +3 elsewhere (v_y = 0), so
    every merged cell has mean velocity vbar = (2, 0), V = max |v| = 3 and x-orthant ranges
    [-1, 3] (w_x > 0) and [-3, 1] (w_x < 0).  With 7 full-grid nodes (spacing 1) or 5
    orthant nodes (spacing 1) a ray along +-x projects u = vbar . w = +-2 onto a node, whose
    value is the cell's box filter of eta, chi with every voxel at u.  A grid over the mean
    speed (2.5) instead of the maximum, a different vbar, voxels taken at their own
    velocities, or a wrong orthant range would put u between nodes or change the node."""
    sc = tiny_lines_scene(n=(32, 32), B=8, L=4, profile="gauss", uniform_v=(3.0, 0.0), n_lam=6)
    x = np.arange(32)
    slow = ((x[None, :] % 2 == 0) & (x[:, None] % 2 == 0)).ravel()  # [y][x] flattened, x fastest
    sc["vel"][0, slow] = -1.0
    sc["dirs"] = AXIS_DIRS
    s = orc.Scene(sc, n_v=n_v, vgrid=vgrid)
    rng = np.random.default_rng(6)
    vox = rng.integers(0, 1024, 48).astype(np.int32)
    for d_idx, u in ((0, 2.0), (1, -2.0)):
        d = np.full(vox.size, d_idx, np.int32)
        for level in (1, 2, 3):
            lv = np.full(16, level, np.int8)
            got = orc.march(s, orc.VELINTERP, lv, vox, d)
            ref = _shifted_static_march(orc, sc, u, level, vox, d)
            np.testing.assert_allclose(got, ref, rtol=1e-9, err_msg="%s dir %d level %d" % (vgrid, d_idx, level))


def test_velinterp_orthant_grid_is_finer(orc):
    """The orthant grids (Sect. 4.1: each quadrant solved with its own grid) span at most the
    full range, so at equal n_v they interpolate at least as finely: at MIP 0 their error
    against Classic is smaller, and both converge to it."""
    sc = tiny_lines_scene(n=(16, 16), B=8, L=1, profile="gauss", vmax=25.0, n_lam=8, dv_span=25.0)
    rng = np.random.default_rng(7)
    vox = rng.integers(0, 256, 80).astype(np.int32)
    d = rng.integers(0, 8, 80).astype(np.int32)
    ref = orc.march(orc.Scene(sc), orc.CLASSIC, None, vox, d)
    err = {}
    for vg in ("full", "orthant"):
        I = orc.march(orc.Scene(sc, n_v=21, vgrid=vg), orc.VELINTERP, None, vox, d)
        err[vg] = np.max(np.abs(I - ref) / np.abs(ref))
    assert err["orthant"] < 0.75 * err["full"], err
    I = orc.march(orc.Scene(sc, n_v=161, vgrid="orthant"), orc.VELINTERP, None, vox, d)
    assert np.max(np.abs(I - ref) / np.abs(ref)) < 1e-3
