"""Pins of the FP64 network oracle (CPU): the encoding's special values, BF16
rounding, the forward pass and gradients against autograd (an independent
implementation), and the analytic gradients against central differences."""
import numpy as np
import pytest

from oracle import nrc


def _rows(rng, n):
    raw = np.zeros((n, 11))
    raw[:, 0:3] = rng.random((n, 3))
    w = rng.normal(size=(n, 3))
    raw[:, 3:6] = w / np.linalg.norm(w, axis=1, keepdims=True)
    raw[:, 6] = rng.random(n)
    raw[:, 7:11] = rng.normal(size=(n, 4)) * 0.3
    return raw


def _params(rng, scale=0.2):
    return rng.normal(size=nrc.NPARAMS) * scale


def test_parameter_count():
    assert nrc.NPARAMS == 256 * 64 + 64 + 3 * (64 * 64 + 64) + 64 + 1 == 28993


def test_encode_special_values():
    raw = np.zeros((3, 11))
    raw[1, 0] = 0.25
    raw[2, 7:11] = [1.5, -2.0, 0.25, 3.0]
    X = nrc.encode(raw, 32.0)
    assert X.shape == (3, 256)
    # zero input: sin 0 = 0, cos 0 = 1 for all 7 quantities and 16 frequencies
    assert np.all(X[0, 0:224:2] == 0.0) and np.all(X[0, 1:224:2] == 1.0)
    # lowest frequency is 1 cycle per unit: a quarter turn
    assert abs(X[1, 0] - 1.0) < 1e-15 and abs(X[1, 1]) < 1e-15
    # frequency j is fmax^(j/15): the top one is fmax (32 x 0.25 = 8 whole turns)
    assert abs(X[1, 30]) < 1e-12 and abs(X[1, 31] - 1.0) < 1e-12
    # frequency 5 is 32^(1/3) = 2^(5/3): sin(2 pi 0.25 2^(5/3))
    assert abs(X[1, 10] - np.sin(2 * np.pi * 0.25 * 2 ** (5 / 3))) < 1e-14
    assert np.array_equal(X[2, 224:228], raw[2, 7:11]) and np.all(X[:, 228:] == 0.0)


def test_bf16_round_ties_to_even():
    u = 2.0 ** -8
    x = np.array([1.0, 1 + u, 1 + 3 * u, 1 + 1.5 * u, -(1 + 3 * u), 3.0e38])
    r = nrc.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                 # tie -> even mantissa (1.0)
    assert r[2] == 1 + 4 * u           # tie between 1+2^-7 and 1+2^-6 -> 1+2^-6
    assert r[3] == 1 + 2 * u           # above the tie -> up
    assert r[4] == -(1 + 4 * u)
    assert np.isfinite(r[5])


def test_forward_and_gradients_match_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    p = _params(rng)
    X = nrc.encode(_rows(rng, 40), 16.0)
    t = rng.normal(size=40) * 0.3
    wt = (rng.random(40) > 0.2).astype(np.float64)
    y, _, _ = nrc.forward(p, X)
    g = nrc.gradients(p, X, t, wt)
    P = nrc.unpack(p)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in P.items()}
    H = torch.tensor(X)
    for L in range(1, 5):
        H = torch.nn.functional.silu(torch.nn.functional.linear(H, tp["W%d" % L], tp["b%d" % L]))
    yt = H @ tp["w5"] + tp["b5"][0]
    lt = (torch.tensor(wt) * (yt - torch.tensor(t)) ** 2).sum() / 40
    lt.backward()
    assert np.max(np.abs(yt.detach().numpy() - y)) < 1e-12
    assert abs(lt.item() - nrc.loss(p, X, t, wt)) < 1e-12
    for k, (o, n) in nrc.OFF.items():
        ga = tp[k].grad.numpy().ravel()
        assert np.max(np.abs(ga - g[o:o + n])) <= 1e-12 * max(1.0, np.max(np.abs(ga))), k


def test_gradients_match_central_differences():
    rng = np.random.default_rng(5)
    p = _params(rng)
    X = nrc.encode(_rows(rng, 24), 8.0)
    t = rng.normal(size=24) * 0.3
    wt = np.ones(24)
    g = nrc.gradients(p, X, t, wt)
    idx = np.concatenate([rng.integers(o, o + n, size=min(n, 12)) for o, n in nrc.OFF.values()])
    fd = nrc.finite_difference(p, X, t, wt, idx, h=1e-6)
    scale = np.max(np.abs(g))
    assert np.max(np.abs(fd - g[idx])) < 1e-6 * scale


def test_rounded_forward_rounds_every_product_input():
    rng = np.random.default_rng(7)
    p = _params(rng)
    X = nrc.encode(_rows(rng, 16), 8.0)
    _, _, Hs = nrc.forward(p, X, nrc.bf16_round)
    for H in Hs:
        assert np.array_equal(H, nrc.bf16_round(H))
    y0, _, _ = nrc.forward(p, X)
    y1, _, _ = nrc.forward(p, X, nrc.bf16_round)
    # BF16 rounding moves the output by a fraction of a percent, not more
    assert 0 < np.max(np.abs(y1 - y0)) < 0.05 * np.max(np.abs(y0))
