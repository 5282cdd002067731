"""Pins of the oracle's prefiltered cells (Sect. 5.1: the transfer precomputed along the +-axes of each cell and
interpolated between them by direction).

  * a homogeneous field: every level's equivalent cell is the field itself, for every signed axis;
  * two voxels with the values of the paper's worked example (Table 1: S = 10, tau = 0.2 and S = 2/7,
    tau = 1.4): the equivalent cell of the pair reproduces the two-slab formal solution in each propagation
    order (light -> dark and dark -> light differ) and the transmittance exp(-(tau1 + tau2));
  * a merged block stratified along one axis, crossed whole by an axis-aligned ray: the prefiltered march
    equals the MIP-0 march (the beam average is exact when every row is the same), for both signs of the
    axis, in 2D and 3D (along z);
  * all levels 0: the prefiltered march is the static march bit for bit;
  * an opaque cell (every row's transmittance underflows) stays finite and, crossed whole along an axis,
    still equals the MIP-0 march (whose last voxel's source function it returns);
A wrong propagation order, a transposed axis, a missing row average or a wrong equivalent emissivity fails one
of them.
"""
import math

import numpy as np
import pytest

import oracle as orc


def scene_dict(dim, n, brick, n_levels, eta, chi, dirs, block_active):
    return dict(dim=dim, n=tuple(n) + (1,) * (3 - len(n)), brick=brick, n_levels=n_levels, model="static",
                eta=eta, chi=chi, dirs=np.asarray(dirs, np.float32), block_active=block_active, ds0=1.0, I0=0.0)


def test_homogeneous_field_is_its_own_prefilter(orc):
    n = (16, 16)
    eta = np.full((1, 256), 0.3)
    chi = np.full((1, 256), 0.7)
    s = orc.Scene(scene_dict(2, n, 8, 4, eta, chi, [[1.0, 0.0]], np.ones(4, np.uint8)))
    pe, pc = orc.prefilter_values(s, eta, chi)
    np.testing.assert_allclose(pe, 0.3, rtol=1e-13)
    np.testing.assert_allclose(pc, 0.7, rtol=1e-13)
    # an empty (zero) field stays zero, and a field with no opacity keeps its emissivity (thin limit)
    pe0, pc0 = orc.prefilter_values(s, np.zeros((1, 256)), np.zeros((1, 256)))
    assert not pe0.any() and not pc0.any()
    pe1, pc1 = orc.prefilter_values(s, eta, np.zeros((1, 256)))
    np.testing.assert_allclose(pe1, 0.3, rtol=1e-13)
    assert not pc1.any()


def test_worked_example_pair_order_dependence(orc):
    """Two voxels (2 x 2 cell, columns x = 0 and x = 1 uniform in y) with Table 1's voxel values."""
    S1, t1, S2, t2 = 10.0, 0.2, 2.0 / 7.0, 1.4
    chi = np.zeros((1, 4))
    eta = np.zeros((1, 4))
    for y in range(2):
        chi[0, 2 * y + 0], eta[0, 2 * y + 0] = t1, S1 * t1
        chi[0, 2 * y + 1], eta[0, 2 * y + 1] = t2, S2 * t2
    s = orc.Scene(scene_dict(2, (2, 2), 2, 2, eta, chi, [[1.0, 0.0]], np.ones(1, np.uint8)))
    pe, pc = orc.prefilter_values(s, eta, chi)
    cell = s.level_total - 1  # the level-1 cell
    L = 2.0
    for k, (Sa, ta, Sb, tb) in ((0, (S1, t1, S2, t2)), (1, (S2, t2, S1, t1))):  # +x: 1 then 2; -x: 2 then 1
        I_exact = Sb * (1 - math.exp(-tb)) + math.exp(-tb) * Sa * (1 - math.exp(-ta))
        chi_eff, eta_eff = pc[0, cell, k], pe[0, cell, k]
        assert chi_eff == pytest.approx((ta + tb) / L, rel=1e-14)
        I_eq = eta_eff / chi_eff * (1 - math.exp(-chi_eff * L))  # the homogeneous cell over its side
        assert I_eq == pytest.approx(I_exact, rel=1e-13)
    assert abs(pe[0, cell, 0] - pe[0, cell, 1]) > 0.1 * pe[0, cell, 0]  # light -> dark differs from dark -> light
    # along y every row is one column: beam average of two different rows
    Ibar = 0.5 * (S1 * (1 - math.exp(-2 * t1)) + S2 * (1 - math.exp(-2 * t2)))
    Tbar = 0.5 * (math.exp(-2 * t1) + math.exp(-2 * t2))
    for k in (2, 3):
        chi_eff, eta_eff = pc[0, cell, k], pe[0, cell, k]
        assert math.exp(-chi_eff * L) == pytest.approx(Tbar, rel=1e-14)
        assert eta_eff / chi_eff * (1 - Tbar) == pytest.approx(Ibar, rel=1e-13)


def stratified(dim, n, axis, seed):
    """eta, chi varying along one axis only (uniform across it), strictly positive."""
    rng = np.random.default_rng(seed)
    prof_c = np.exp(rng.normal(-1.0, 1.0, n[axis]))
    prof_s = rng.uniform(0.2, 2.0, n[axis])
    shape = tuple(reversed(n))  # numpy [z][y][x]
    idx = np.indices(shape)[dim - 1 - axis]
    chi = prof_c[idx].reshape(1, -1)
    eta = (prof_s[idx] * prof_c[idx]).reshape(1, -1)
    return eta, chi


@pytest.mark.parametrize("dim", [2, 3])
def test_axis_ray_through_stratified_merged_block_is_exact(orc, dim):
    """Block 0 merged to one cell (level log2 B), block 1 at MIP 0 holding the probe; axis-aligned rays that cross
    block 0 whole: equal to the MIP-0 march, for the propagation sign that enters block 0 from either face."""
    B = 8
    axis = dim - 1  # y in 2D, z in 3D
    n = [B] * dim
    n[axis] = 2 * B
    eta, chi = stratified(dim, n, axis, 11 + dim)
    nb = 2
    dirs = np.zeros((2, dim), np.float32)
    dirs[0, axis], dirs[1, axis] = 1.0, -1.0
    sc = scene_dict(dim, n, B, 4, eta, chi, dirs, np.ones(nb, np.uint8))
    s = orc.Scene(sc)
    lvs, st_e, st_c = orc.static_level_values(s, eta, chi, sc["block_active"], T=1e-2)
    pe, pc = orc.prefilter_values(s, eta, chi)
    s.set_static_levels(st_e, st_c)
    s.set_prefilter(pe, pc)
    lv0 = np.zeros(nb, np.int8)
    strides = [1, n[0], n[0] * (n[1] if dim > 1 else 1)]
    for merged, probe_block, d in ((0, 1, 0), (1, 0, 1)):
        # +axis propagation: the upwind side is block 0 (merged), probe in block 1; -axis the other way round
        lv = lv0.copy()
        lv[merged] = 3
        rng = np.random.default_rng(5)
        probes = []
        for _ in range(6):
            c = [int(v) for v in rng.integers(0, B, dim)]
            c[axis] += probe_block * B
            probes.append(sum(c[a] * strides[a] for a in range(dim)))
        probes = np.array(probes, np.int32)
        dd = np.full(probes.size, d, np.int32)
        got = orc.march(s, orc.PREFILTER, lv, probes, dd)
        ref = orc.march(s, orc.STATIC, lv0, probes, dd)
        np.testing.assert_allclose(got, ref, rtol=1e-12)
        # the same rays through the box-filtered merged block are not exact (the test has teeth)
        box = orc.march(s, orc.STATIC, lv, probes, dd)
        assert np.max(np.abs(box / ref - 1)) > 1e-3
        # and the other sign's prefiltered values give a different answer
        s2 = orc.Scene(sc)
        s2.set_static_levels(st_e, st_c)
        K = 2 * dim
        swapped_e, swapped_c = pe.copy(), pc.copy()
        swapped_e[..., 2 * axis], swapped_e[..., 2 * axis + 1] = pe[..., 2 * axis + 1], pe[..., 2 * axis]
        swapped_c[..., 2 * axis], swapped_c[..., 2 * axis + 1] = pc[..., 2 * axis + 1], pc[..., 2 * axis]
        assert K == pe.shape[-1]
        s2.set_prefilter(swapped_e, swapped_c)
        wrong = orc.march(s2, orc.PREFILTER, lv, probes, dd)
        assert np.max(np.abs(wrong / ref - 1)) > 1e-3


def test_level0_prefilter_march_is_static_march(orc):
    rng = np.random.default_rng(3)
    n = (32, 32)
    chi = np.exp(rng.normal(-2, 1, (2, 1024)))
    eta = chi * rng.uniform(0.5, 1.5, (2, 1024))
    act = np.ones(16, np.uint8)
    act[5] = 0
    for b in (5,):
        bx, by = b % 4, b // 4
        for y in range(by * 8, by * 8 + 8):
            chi[:, y * 32 + bx * 8: y * 32 + bx * 8 + 8] = 0
            eta[:, y * 32 + bx * 8: y * 32 + bx * 8 + 8] = 0
    th = np.linspace(0.1, 6.0, 7)
    dirs = np.stack([np.cos(th), np.sin(th)], 1).astype(np.float32)
    sc = scene_dict(2, n, 8, 4, eta, chi, dirs, act)
    s = orc.Scene(sc)
    lvs, st_e, st_c = orc.static_level_values(s, eta, chi, act, T=1e-2)
    pe, pc = orc.prefilter_values(s, eta, chi)
    s.set_static_levels(st_e, st_c)
    s.set_prefilter(pe, pc)
    lv = np.where(act > 0, 0, -1).astype(np.int8)
    vox = rng.integers(0, 1024, 64).astype(np.int32)
    vox = vox[act[(vox % 32) // 8 + 4 * ((vox // 32) // 8)] > 0]
    d = rng.integers(0, 7, vox.size).astype(np.int32)
    assert np.array_equal(orc.march(s, orc.PREFILTER, lv, vox, d), orc.march(s, orc.STATIC, lv, vox, d))


def test_opaque_cells_stay_finite_and_exact_along_axes(orc):
    """chi = 100 per voxel: rows of 8 voxels have tau = 800 and T_row = 0 in FP64.  The equivalent cell is finite,
    and an axis ray crossing the merged block whole returns what the MIP-0 march returns."""
    B = 8
    n = (B, 2 * B)
    eta, chi = stratified(2, list(n), 1, 21)
    chi *= 100.0 / chi.min()
    eta *= 100.0 / eta.min()
    thin = np.arange(n[0] * n[1]) >= n[0] * B  # block 1 (y >= B), which holds the probes, stays optically thin
    chi[:, thin] *= 1e-4
    dirs = np.array([[0.0, 1.0], [0.0, -1.0], [0.6, 0.8]], np.float32)
    sc = scene_dict(2, n, B, 4, eta, chi, dirs, np.ones(2, np.uint8))
    s = orc.Scene(sc)
    _, st_e, st_c = orc.static_level_values(s, eta, chi, sc["block_active"], T=1e-2)
    pe, pc = orc.prefilter_values(s, eta, chi)
    assert np.all(np.isfinite(pe)) and np.all(np.isfinite(pc)) and np.all(pc > 0)
    s.set_static_levels(st_e, st_c)
    s.set_prefilter(pe, pc)
    lv = np.array([3, 0], np.int8)
    probes = np.array([9 * B + 3, 12 * B + 5], np.int32)
    ref = orc.march(s, orc.STATIC, np.zeros(2, np.int8), probes, np.zeros(2, np.int32))
    got = orc.march(s, orc.PREFILTER, lv, probes, np.zeros(2, np.int32))
    np.testing.assert_allclose(got, ref, rtol=1e-12)
    got2 = orc.march(s, orc.PREFILTER, lv, probes, np.full(2, 2, np.int32))
    assert np.all(np.isfinite(got2))
