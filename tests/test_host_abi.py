"""Host-only entry points of the C ABI (no device work): size queries and descriptor validation."""
import numpy as np
import pytest

from synth import make_cfg1


@pytest.fixture(scope="module")
def rt():
    import paper_2511_08498_amd as rt
    rt.lib()
    return rt


def _layout_bytes(nb, n_state_words, na, cells, feat_cells, n_lam_batch=8):
    """Device layout of a static scene in its workspace, each piece rounded up to a multiple of 256 B (so
    every piece stays 256-byte aligned): morton, active, slot, active list, active count, levels, states,
    error counters, input-validation counter, level statistics [na][feat cells][8] float4, values
    [na][cells][8][eta, chi] float."""
    a = lambda n: (max(n, 1) + 255) // 256 * 256  # noqa: E731
    return (a(4 * nb) + a(nb) + a(4 * nb) + a(4 * nb) + a(4) + a(nb) + a(8 * n_state_words) + a(32) + a(8)
            + a(16 * na * feat_cells * n_lam_batch) + a(4 * 2 * n_lam_batch * na * cells))


def test_scene_workspace_bytes_static(rt):
    sc = make_cfg1()
    na = int(sc["block_active"].sum())
    # 64^2, 8^2 bricks, 4 levels: 64 + 16 + 4 + 1 cells per brick, level-2 statistics (2^2 cells per brick)
    assert rt.scene_workspace_bytes(sc) == _layout_bytes(64, 4, na, 85, 4)
    assert rt.scene_workspace_bytes(sc, dense=True) == _layout_bytes(64, 4, 64, 85, 4)
    assert rt.scene_workspace_bytes(sc, n_active=0) == _layout_bytes(64, 4, 0, 85, 4)


def test_scene_descriptor_validation(rt):
    sc = make_cfg1()
    cases = [(dict(sc, n=(60, 64, 1)), rt.RT_E_ARG),            # not a multiple of the brick
             (dict(sc, n_levels=5), rt.RT_E_ARG),                 # 8^2 bricks allow levels 0..3
             (dict(sc, dim=3, n=(64, 64, 64), brick=16), rt.RT_E_UNSUPPORTED)]  # 3D uses 8^3 bricks
    for bad, status in cases:
        with pytest.raises(rt.RtError) as e:
            rt.scene_workspace_bytes(bad)
        assert e.value.status == status
    with pytest.raises(rt.RtError) as e:
        rt.scene_workspace_bytes(sc, n_active=65)
    assert e.value.status == rt.RT_E_ARG
    # 8192^2 voxels in 8^2 bricks: 2^20 blocks, whose packed states (399 KB) exceed a compute unit's LDS
    big = dict(sc, n=(8192, 8192, 1), block_active=np.ones(1 << 20, np.uint8))
    with pytest.raises(rt.RtError) as e:
        rt.scene_workspace_bytes(big, n_active=0)
    assert e.value.status == rt.RT_E_UNSUPPORTED and "LDS" in str(e.value)
    # the same grid in 16^2 bricks fits (2^18 blocks, 100 KB of states)
    assert rt.scene_workspace_bytes(dict(big, brick=16, block_active=np.ones(1 << 18, np.uint8)), n_active=0) > 0


def test_nrc_workspace_bytes(rt):
    B = 16384
    # weights/Adam/gradient (FP32, padded to 256) + BF16 copy, activations, output gradient,
    # per-chunk gradient partials (256 chunks of the padded parameter layout), loss partials
    npad = (rt.nrc_num_params() + 255) // 256 * 256
    expect = (4 * 4 * npad + 2 * npad + 2 * B * 256 + 4 * 4 * B * 64 + 2 * 4 * B * 64 + 4 * B + 4 * 256 * npad
              + 4 * 512)
    assert rt.nrc_workspace_bytes(B) == expect
    for bad in (0, 300, 1 << 20):
        with pytest.raises(rt.RtError):
            rt.nrc_workspace_bytes(bad)


def test_velocity_grid_ratio():
    """Node spacing against the thermal width c / (lam0 inv_dld) (Sect. 3.1 warning rule): 2 |v| / (n_v - 1) for
    the full grid; the widest orthant range / (n_v - 1) for orthant grids."""
    import paper_2511_08498_amd as rt
    nvox = 50
    vel = np.zeros((2, nvox), np.float32)
    vel[0, 7] = 30.0                                  # 30 km/s in one voxel: spacing 3 km/s with 21 nodes
    lam0 = np.array([500.0, 600.0])
    idl = np.zeros((2, nvox), np.float32)
    idl[0] = rt.C_KMS / (500.0 * 1.0)                 # line 0: thermal width 1 km/s
    idl[1] = rt.C_KMS / (600.0 * 10.0)                # line 1: 10 km/s
    idl[1, 3] = 0.0                                   # no line in this voxel: ignored
    r = rt.velocity_grid_ratio(vel, idl, lam0, 21, vgrid="full")
    np.testing.assert_allclose(r, [3.0, 0.3], rtol=1e-5)
    # v along x: the orthant ranges are [0, 30] (w_x > 0) and [-30, 0] (w_x < 0), spacing 1.5 km/s
    r = rt.velocity_grid_ratio(vel, idl, lam0, 21, vgrid="orthant")
    np.testing.assert_allclose(r, [1.5, 0.15], rtol=1e-5)
    # v at 45 degrees: the quadrants across it see [-30/sqrt 2, 30/sqrt 2], the widest range
    vel[:, 7] = 30.0 / np.sqrt(2.0)
    r = rt.velocity_grid_ratio(vel, idl, lam0, 21, vgrid="orthant")
    np.testing.assert_allclose(r, [1.5 * np.sqrt(2.0), 0.15 * np.sqrt(2.0)], rtol=1e-5)
    for vg in ("full", "orthant"):
        assert np.all(rt.velocity_grid_ratio(np.zeros((2, nvox), np.float32), idl, lam0, 21, vgrid=vg) == 0)


def test_create_refuses_a_bad_workspace(rt):
    """Scene creation takes a caller-owned workspace: a null, misaligned or too small one is refused on the
    host before any device work (the input pointers are never dereferenced here)."""
    import ctypes
    sc = make_cfg1()
    d, _, _ = rt._scene_desc(sc["dim"], sc["n"], sc["brick"], sc["n_levels"], "static", "static", "gauss", 21,
                             False, 1.0, 16, None, None)
    inp = rt.RtSceneInputs()
    inp.d_eta, inp.d_chi = 0x100000, 0x200000  # not dereferenced: the workspace check comes first
    need = ctypes.c_size_t(0)
    rt._check(rt.lib().rt_scene_workspace_bytes(ctypes.byref(d), 0, ctypes.byref(need)))
    na = ctypes.c_int64(-1)
    h = ctypes.c_void_p()
    for ws, nbytes, msg in ((None, need.value, b"null workspace"), (0x300010, need.value, b"aligned"),
                            (0x300000, 256, b"needed")):
        st = rt.lib().rt_scene_count_active(ctypes.byref(d), ctypes.byref(inp), ws, nbytes, None, ctypes.byref(na))
        assert st == rt.RT_E_ARG and msg in rt.lib().rt_last_error(), rt.lib().rt_last_error()
        st = rt.lib().rt_scene_create(ctypes.byref(d), ctypes.byref(inp), ws, nbytes, None, ctypes.byref(h))
        assert st == rt.RT_E_ARG and msg in rt.lib().rt_last_error()
    assert na.value == -1 and not h.value
    for bad in (0, -1):
        v = ctypes.c_size_t(0)
        assert rt.lib().rt_batch_workspace_bytes(bad, ctypes.byref(v)) == rt.RT_E_ARG
    v = ctypes.c_size_t(0)
    rt._check(rt.lib().rt_batch_workspace_bytes(3, ctypes.byref(v)))
    assert v.value % 256 == 0 and v.value >= 3 * 64
