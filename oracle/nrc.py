"""FP64 numpy reference of the neural-radiance-cache network (test infrastructure).

Only tests may import it.  The paper does not describe this cache (it is an
extension of the formal solution: a learned far field at a truncation
point); the network is restated here from its definition, in FP64,
independently of the HIP kernels:
  input  = 16 log-spaced frequencies f_j = fmax^(j/15), j = 0..15, of
           sin(2 pi f_j v), cos(2 pi f_j v) for v in (x, y, z, w_x, w_y, w_z,
           wavelength offset)  (224 values, ordered quantity, frequency,
           sin/cos), then the 4 level statistics, then zeros up to 256;
  hidden = 4 layers of 64 with SiLU(z) = z / (1 + e^-z);
  output = one linear unit, predicting ln(I_far) / 10;
  loss   = sum_r w_r (y_r - t_r)^2 / R over a batch of R rows.
Weights may be rounded to BF16 first (the GPU multiplies BF16 weights), and
`rnd` (e.g. bf16_round) may be applied to every matrix-product input (the
encoded features and each hidden activation), which is where a BF16
matrix-core forward rounds; the backward pass then uses those rounded
activations as the layer inputs.  The analytic backward pass is checked
against central finite differences and against autograd.
"""
from __future__ import annotations

import numpy as np

FEAT, HID, NFREQ = 256, 64, 16
OFF = {}
_o = 0
for _name, _size in (("W1", HID * FEAT), ("b1", HID), ("W2", HID * HID), ("b2", HID), ("W3", HID * HID),
                     ("b3", HID), ("W4", HID * HID), ("b4", HID), ("w5", HID), ("b5", 1)):
    OFF[_name] = (_o, _size)
    _o += _size
NPARAMS = _o


def unpack(p):
    """Parameter vector -> dict of arrays (W as [out][in])."""
    d = {}
    for k, (o, n) in OFF.items():
        v = p[o:o + n]
        if k == "W1":
            v = v.reshape(HID, FEAT)
        elif k[0] == "W":
            v = v.reshape(HID, HID)
        d[k] = v
    return d


def bf16_round(x):
    """Round float32/float64 values to the nearest BF16 (ties to even)."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def encode(raw, freq_max):
    """raw [n][>=11] -> encoded inputs [n][256] (FP64)."""
    raw = np.asarray(raw, np.float64)
    n = raw.shape[0]
    X = np.zeros((n, FEAT))
    f = freq_max ** (np.arange(NFREQ) / 15.0)
    for q in range(7):
        ang = 2 * np.pi * raw[:, q:q + 1] * f[None, :]
        X[:, 32 * q:32 * q + 32:2] = np.sin(ang)
        X[:, 32 * q + 1:32 * q + 32:2] = np.cos(ang)
    X[:, 224:228] = raw[:, 7:11]
    return X


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def _ident(x):
    return x


def forward(p, X, rnd=_ident):
    """y [n], pre-activations Zs[4], layer inputs Hs[5] (Hs[0] = rnd(X), Hs[4] = rnd(h4))."""
    P = unpack(p)
    H = rnd(X)
    Zs, Hs = [], [H]
    for L in range(1, 5):
        Z = H @ P["W%d" % L].T + P["b%d" % L]
        H = rnd(silu(Z))
        Zs.append(Z)
        Hs.append(H)
    y = H @ P["w5"] + P["b5"][0]
    return y, Zs, Hs


def loss(p, X, target, weight, rnd=_ident):
    y, _, _ = forward(p, X, rnd)
    return float(np.sum(weight * (y - target) ** 2) / X.shape[0])


def gradients(p, X, target, weight, rnd=_ident):
    """Analytic gradient of `loss` with respect to the parameter vector (rounding
    treated as the identity in the backward pass)."""
    P = unpack(p)
    y, Zs, Hs = forward(p, X, rnd)
    R = X.shape[0]
    dy = 2.0 * weight * (y - target) / R
    g = np.zeros_like(p)
    o, n = OFF["w5"]
    g[o:o + n] = Hs[4].T @ dy
    g[OFF["b5"][0]] = dy.sum()
    dH = np.outer(dy, P["w5"])
    for L in range(4, 0, -1):
        dZ = dH * silu_grad(Zs[L - 1])
        o, n = OFF["W%d" % L]
        g[o:o + n] = (dZ.T @ Hs[L - 1]).ravel()
        o, n = OFF["b%d" % L]
        g[o:o + n] = dZ.sum(axis=0)
        dH = dZ @ P["W%d" % L]
    return g


def finite_difference(p, X, target, weight, idx, h=1e-6):
    out = []
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        out.append((loss(pp, X, target, weight) - loss(pm, X, target, weight)) / (2 * h))
    return np.array(out)
