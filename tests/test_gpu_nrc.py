"""GPU tests of the truncated march and the neural radiance cache.

Truncated march (2D 64^2 scene, 8x8 bricks, 8 wavelengths, 8 directions,
truncation at path length 32):
  - generation mode: I_near + T_near I_far equals the full march to FP32
    rounding (the formal solution splits exactly at any point), rays that need
    no query reproduce it bit for bit;
  - truncation points and query flags against the FP64 oracle's segment lists,
    level statistics at the truncation point against their definition;
  - inference mode with every block flagged for fallback is the plain march,
    bit for bit; the near part equals generation mode's bit for bit.
Cache (BF16 matrix cores):
  - forward pass against the FP64 network with the same BF16 roundings;
  - gradients against the FP64 analytic gradients (relative L2 per tensor);
  - training lowers the loss; weights round-trip;
  - compose / validate / fallback plumbing and the gain over dropping the far field.
"""
import numpy as np
import pytest

import oracle as orc
from oracle import nrc as onrc
from synth import make_cfg1

pytestmark = pytest.mark.gpu

T_TRUNC = 32.0
# composition of near and far parts vs the single march: FP32 rounding of two
# products and a sum over a few hundred segments
TOL_COMPOSE = 1e-5


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
    full = scene.trace(dirs, mode="vlm")
    gen = scene.trace_truncated(dirs, T_TRUNC, gen=True)
    torch.cuda.synchronize()
    return sc, scene, dirs, full, gen


def _rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-30)


def test_generation_mode_composes_to_full_march(rt, setup):
    sc, scene, dirs, full, gen = setup
    I = full.cpu().numpy().astype(np.float64)
    In, Tn, If = (gen[k].cpu().numpy().astype(np.float64) for k in ("I_near", "T_near", "I_far"))
    flag = gen["feat"].cpu().numpy()[..., 3]
    # 0, or 1 + the index of an active block
    assert np.all(flag == np.round(flag)) and np.all((flag == 0) | sc["block_active"][np.maximum(flag.astype(int) - 1, 0)].astype(bool))
    q = flag[:, None, :] > 0
    assert 0.2 < q.mean() < 0.95  # both kinds of rays are present
    comp = In + Tn * If
    assert np.max(_rel(comp, I)) < TOL_COMPOSE
    # rays with no query: the near part is the whole march, bit for bit
    nq = np.broadcast_to(~q, I.shape)
    assert np.array_equal(gen["I_near"].cpu().numpy()[nq], full.cpu().numpy()[nq])
    assert np.all(Tn[nq] == 0.0) and np.all(If[nq] == 0.0)  # I0 = 0
    # transmittances are probabilities; the far field of a query ray is what lies beyond
    assert np.all((Tn >= 0) & (Tn <= 1))
    assert np.all(If >= 0)


def test_truncation_points_match_oracle_segments(rt, setup):
    sc, scene, dirs, full, gen = setup
    s = orc.Scene(sc)
    lvs, st_e, st_c = orc.static_level_values(s, sc["eta"][0:8], sc["chi"][0:8], sc["block_active"], T=1e-2)
    lv = orc.batch_levels(lvs)
    assert np.array_equal(scene.levels(), lv)
    feat = gen["feat"].cpu().numpy()
    fstat = gen["fstat"].cpu().numpy()
    probes = scene.probe_voxels()
    rng = np.random.default_rng(11)
    with np.errstate(divide="ignore"):  # empty bricks (chi = eta = 0) are never a truncation cell
        lchi = np.log(sc["chi"][0:8].astype(np.float64) * sc["ds0"])
        leta = np.log(sc["eta"][0:8].astype(np.float64) * sc["ds0"])
    n_q = 0
    for d in range(dirs.shape[0]):
        w = sc["dirs"][d]
        for pi in rng.choice(probes.size, 120, replace=False):
            pv = (int(probes[pi]) % 64, int(probes[pi]) // 64)
            cells, lvl, t_in, t_out = orc.ray_segments(s, lv, pv, w)
            k = np.nonzero(t_out > T_TRUNC)[0]
            if k.size == 0:
                assert feat[d, pi, 3] == 0.0
                continue
            k = k[0]
            n_q += 1
            # the block holding the truncation cell, recorded as 1 + its index
            assert feat[d, pi, 3] == 1 + cells[k, 0] // 8 + 8 * (cells[k, 1] // 8)
            ts = max(t_in[k], T_TRUNC)
            x = np.array(pv, np.float64) + 0.5 - ts * w.astype(np.float64)
            assert np.max(np.abs(feat[d, pi, :2] - x)) < 2e-5
            # level-2 statistics of the cell holding the truncation cell's corner:
            # mean and population variance of its four level-1 log means
            cx, cy = (cells[k, 0] >> 2) << 2, (cells[k, 1] >> 2) << 2
            for l in range(8):
                for f, src in ((0, lchi), (2, leta)):
                    g = src[l].reshape(64, 64)[cy:cy + 4, cx:cx + 4]
                    m1 = np.array([g[j:j + 2, i:i + 2].mean() for j in (0, 2) for i in (0, 2)])
                    mean, var = m1.mean(), ((m1 - m1.mean()) ** 2).mean()
                    assert abs(fstat[d, l, pi, f] - mean) <= 1e-5 * max(1.0, abs(mean))
                    assert abs(fstat[d, l, pi, f + 1] - var) <= 1e-5 * max(1.0, var) + 1e-6
    assert n_q > 300


def test_fallback_everywhere_is_the_plain_march(rt, setup):
    import torch
    sc, scene, dirs, full, gen = setup
    fb = torch.ones(scene.info["n_blocks"], dtype=torch.uint8, device="cuda")
    inf = scene.trace_truncated(dirs, T_TRUNC, gen=False, fallback=fb)
    torch.cuda.synchronize()
    assert torch.equal(inf["I_near"], full)
    assert torch.all(inf["T_near"] == 0)
    assert torch.all(inf["feat"][..., 3] == 0)


def test_inference_near_part_equals_generation(rt, setup):
    import torch
    sc, scene, dirs, full, gen = setup
    inf = scene.trace_truncated(dirs, T_TRUNC, gen=False)
    torch.cuda.synchronize()
    for k in ("I_near", "T_near", "feat", "fstat"):
        assert torch.equal(inf[k], gen[k]), k


def _raw_rows(rng, n):
    raw = np.zeros((n, 12), np.float32)
    raw[:, 0:3] = rng.random((n, 3))
    w = rng.normal(size=(n, 3))
    raw[:, 3:6] = w / np.linalg.norm(w, axis=1, keepdims=True)
    raw[:, 6] = rng.random(n)
    raw[:, 7:11] = rng.normal(size=(n, 4)) * 0.3
    raw[:, 11] = 1.0
    return raw


def _emulated_params(w):
    """The GPU multiplies BF16 copies of the four weight matrices; biases and the
    output layer stay FP32."""
    p = w.astype(np.float64)
    for k in ("W1", "W2", "W3", "W4"):
        o, n = onrc.OFF[k]
        p[o:o + n] = onrc.bf16_round(p[o:o + n])
    return p


def test_forward_matches_oracle(rt):
    nn = rt.Nrc(max_batch=8192, freq_max=32.0, seed=7)
    rng = np.random.default_rng(1)
    raw = _raw_rows(rng, 4133)  # several 16-row tiles and a ragged tail
    y = nn.predict(raw).cpu().numpy().astype(np.float64)
    p = _emulated_params(nn.get_weights())
    X = onrc.encode(raw[:, :11].astype(np.float64), 32.0)
    y_em, _, _ = onrc.forward(p, X, onrc.bf16_round)
    y64, _, _ = onrc.forward(nn.get_weights().astype(np.float64), X)
    # same roundings: only FP32 summation order and the fast sine move a BF16 rounding now and then
    assert np.max(np.abs(y - y_em)) < 2e-3
    assert np.mean(np.abs(y - y_em)) < 5e-5
    # against the unrounded FP64 network: BF16 quantisation
    assert np.linalg.norm(y - y64) / np.linalg.norm(y64) < 2e-2


@pytest.mark.parametrize("rows", [512, 16640])
def test_gradients_match_oracle(rt, rows):
    """512 rows: eight 64-row chunks, one per workgroup.  16640 rows: 260 chunks on 256 workgroups, so four
    workgroups add a second chunk to their partial; the gradients are also the same bits on a second call."""
    nn = rt.Nrc(max_batch=16640, freq_max=16.0, seed=3)
    rng = np.random.default_rng(2)
    raw = _raw_rows(rng, rows)
    raw[::7, 11] = 0.0  # ignored rows
    tgt = (rng.normal(size=rows) * 0.3).astype(np.float32)
    g = nn.gradients(raw, tgt).cpu().numpy().astype(np.float64)
    assert np.array_equal(nn.gradients(raw, tgt).cpu().numpy(), g.astype(np.float32))
    p = _emulated_params(nn.get_weights())
    X = onrc.encode(raw[:, :11].astype(np.float64), 16.0)
    g_ref = onrc.gradients(p, X, tgt.astype(np.float64), raw[:, 11].astype(np.float64), onrc.bf16_round)
    rel = {}
    for k, (o, n) in onrc.OFF.items():
        a, b = g[o:o + n], g_ref[o:o + n]
        rel[k] = np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-30)
    print("gradient relative L2 error per tensor:", {k: "%.2e" % v for k, v in rel.items()})
    for k, (o, n) in onrc.OFF.items():
        a, b = g[o:o + n], g_ref[o:o + n]
        assert np.linalg.norm(a - b) <= 1e-2 * np.linalg.norm(b) + 1e-7, (k, rel)


def test_checkpoint_resume_is_bit_exact(rt, tmp_path):
    """Weights, Adam moments and step count saved to .npz and loaded into a new cache with the same descriptor:
    the resumed training repeats the uninterrupted one bit for bit (no float atomics, counter-based batches)."""
    rng = np.random.default_rng(6)
    raw = _raw_rows(rng, 32768)
    tgt = (0.2 * np.sin(2 * np.pi * raw[:, 1]) - 0.3).astype(np.float32)
    nn = rt.Nrc(max_batch=4096, freq_max=8.0, seed=9)
    nn.train(raw, tgt, steps=25, batch=2048, lr=2e-3)
    path = str(tmp_path / "nrc.npz")
    nn.save_checkpoint(path)
    nn.train(raw, tgt, steps=25, batch=2048, lr=2e-3)
    a = nn.get_state()
    nn2 = rt.Nrc(max_batch=4096, freq_max=8.0, seed=9)
    nn2.load_checkpoint(path)
    assert nn2.get_state()["step"] == 25
    nn2.train(raw, tgt, steps=25, batch=2048, lr=2e-3)
    b = nn2.get_state()
    assert a["step"] == b["step"] == 50
    for k in ("w", "m", "v"):
        assert np.array_equal(a[k], b[k]), k
    with np.load(path, allow_pickle=False) as z:
        assert sorted(z.files) == ["m", "step", "v", "w"]


def test_training_lowers_loss_and_weights_round_trip(rt):
    nn = rt.Nrc(max_batch=8192, freq_max=8.0, seed=5)
    rng = np.random.default_rng(4)
    raw = _raw_rows(rng, 65536)
    tgt = (0.3 * np.sin(2 * np.pi * raw[:, 0]) * np.cos(2 * np.pi * raw[:, 1]) + 0.2 * raw[:, 3]
           - 0.1 * raw[:, 6] - 0.4).astype(np.float32)
    nn.train(raw, tgt, steps=1, batch=4096, lr=2e-3)
    l0 = nn.loss()
    nn.train(raw, tgt, steps=400, batch=4096, lr=2e-3)
    l1 = nn.loss()
    assert l1 < 0.05 * l0
    held = _raw_rows(np.random.default_rng(99), 4096)
    th = 0.3 * np.sin(2 * np.pi * held[:, 0]) * np.cos(2 * np.pi * held[:, 1]) + 0.2 * held[:, 3] - 0.1 * held[:, 6] - 0.4
    yh = nn.predict(held).cpu().numpy()
    assert np.mean((yh - th) ** 2) < 0.1 * np.var(th)
    w = nn.get_weights()
    nn2 = rt.Nrc(max_batch=256, freq_max=8.0, seed=123)
    nn2.set_weights(w)
    assert np.array_equal(nn2.get_weights(), w)
    import torch
    assert torch.equal(nn2.predict(held), nn.predict(held))


def test_cache_compose_validate_and_gain(rt, setup):
    import torch
    sc, scene, dirs, full, gen = setup
    nd, nl, npb = full.shape
    rows = nd * nl * npb
    raw = torch.zeros((rows, 12), device="cuda")
    tgt = torch.zeros(rows, device="cuda")
    nn = rt.Nrc(max_batch=8192, freq_max=32.0, seed=9)
    nn.pack(scene, gen, raw, tgt, 0)
    torch.cuda.synchronize()
    # packed rows: flag column equals the query flag of (dir, probe), targets ln(I_far)/10
    flag = (gen["feat"][..., 3] > 0).float()
    assert torch.equal(raw[:, 11].view(nd, nl, npb), flag[:, None, :].expand(nd, nl, npb))
    If = gen["I_far"]
    qm = flag[:, None, :].expand(nd, nl, npb) > 0
    assert torch.allclose(tgt.view(nd, nl, npb)[qm], torch.log(torch.clamp(If[qm], min=1e-30)) * 0.1,
                          rtol=1e-5, atol=1e-6)
    nn.train(raw, tgt, steps=600, batch=8192, lr=2e-3)
    inf = scene.trace_truncated(dirs, T_TRUNC, gen=False)
    I_nrc = nn.compose(scene, inf)
    # compose = I_near + T_near exp(10 y) with y the network's output on the packed row
    y = nn.predict(raw).view(nd, nl, npb)
    expect = torch.where(qm, inf["I_near"] + inf["T_near"] * torch.exp(10 * torch.clamp(y, -8, 8)), inf["I_near"])
    assert torch.allclose(I_nrc, expect, rtol=2e-5, atol=0)
    # gain: the cache beats dropping the far field where the far field matters
    I = full.double()
    e_nrc = ((I_nrc.double() - I).abs() / I.abs().clamp_min(1e-30))[qm]
    e_cut = ((inf["I_near"].double() - I).abs() / I.abs().clamp_min(1e-30))[qm]
    sel = e_cut > 1e-2
    assert sel.sum() > 100
    med_nrc, med_cut = e_nrc[sel].median().item(), e_cut[sel].median().item()
    print("median rel err: cache %.3e, far field dropped %.3e" % (med_nrc, med_cut))
    assert med_nrc < 0.5 * med_cut
    # held-out check: flagged blocks fall back to the full march, bit for bit
    fb = torch.zeros(scene.info["n_blocks"], dtype=torch.uint8, device="cuda")
    pred, err = nn.validate(scene, gen, 5e-3, fb)
    assert torch.allclose(pred, I_nrc, rtol=1e-5, atol=0)
    flagged = fb.cpu().numpy().astype(bool)
    assert 0 < flagged.sum()
    inf2 = scene.trace_truncated(dirs, T_TRUNC, gen=False, fallback=fb)
    I2 = nn.compose(scene, inf2)
    ft = gen["feat"].cpu().numpy()
    blk = np.maximum(ft[..., 3].astype(int) - 1, 0)
    fell = (ft[..., 3] > 0) & flagged[blk]
    fell3 = np.broadcast_to(fell[:, None, :], full.shape)
    assert fell.sum() > 0
    assert np.array_equal(I2.cpu().numpy()[fell3], full.cpu().numpy()[fell3])
    keep = np.broadcast_to((ft[..., 3] > 0)[:, None, :] & ~fell3, full.shape)
    assert np.array_equal(I2.cpu().numpy()[keep], I_nrc.cpu().numpy()[keep])
    # every held-out error above the threshold lies in a flagged block
    e = err.cpu().numpy()
    bad = (e > 5e-3) & np.broadcast_to((ft[..., 3] > 0)[:, None, :], full.shape)
    assert np.all(np.broadcast_to(flagged[blk][:, None, :], full.shape)[bad])
    # checks per block are counted, and blocks with fewer than min_queries checks fall back too
    cnt = torch.zeros(scene.info["n_blocks"], dtype=torch.int32, device="cuda")
    fb2 = torch.zeros_like(fb)
    nn.validate(scene, gen, 5e-3, fb2, count=cnt)
    q = ft[..., 3] > 0
    want = np.bincount(blk[q], minlength=scene.info["n_blocks"]) * full.shape[1]  # one per (query, wavelength)
    assert np.array_equal(cnt.cpu().numpy(), want)
    assert torch.equal(fb2, fb)
    k = 3 * full.shape[1]
    nn.fallback_unverified(scene, cnt, k, fb2)
    assert np.array_equal(fb2.cpu().numpy().astype(bool), flagged | (want < k))
