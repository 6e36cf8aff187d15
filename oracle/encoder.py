"""FP64 reference of the learned frequency proposal (test infrastructure).

The network is the set encoder the GPU kernels implement: per-point features
-> Linear(80, 64) -> ReLU -> Linear(64, 128) -> ReLU -> mean over the points
of a light curve -> Linear(128, 1024) logits over log-spaced frequency bins
(the first layer's bias is the weight row of a constant-one feature),
trained with softmax cross-entropy against the bin of the full-grid Super
Smoother best frequency.  Everything here is plain numpy in float64, written
as the definition (no fusion), with an analytic backward pass that the tests
check against central finite differences.  Only the test suite may import it.

With bf16=True the operands that the matrix cores take in BF16 (features,
W1, W2, the hidden layer, and in the backward pass the two gated
activation gradients) are rounded to BF16 (round to nearest, ties to even)
before the FP64 products; everything else stays FP64.  This isolates the
rounding that the BF16 precision of the network fixes from any other
difference.

Feature vector of point i of an object (80 slots, the last 13 zero):
  sin(2 pi g_m tt_i), cos(2 pi g_m tt_i) for the M = 32 frequencies g_m
  log-spaced over [f_lo, f_hi] (slots 2m and 2m+1),
  (y_i - ybar)/sigma and e_i/sigma (slots 64, 65), with ybar the
  e^-2-weighted mean, sigma = sqrt(sum w (y - ybar)^2 / sum w), tt = t - min t,
  and the constant 1 (slot 66).
Parameters, flat float order: w1[80,64], w2[64,128], b2[128], w3[128,1024],
b3[1024] (row-major, input dimension first; row 66 of w1 is the first
layer's bias).
"""
from __future__ import annotations

import numpy as np

M_FREQ = 32
K1, H1, H2, BINS = 80, 64, 128, 1024
ONE_SLOT = 66
SHAPES = (("w1", (K1, H1)), ("w2", (H1, H2)), ("b2", (H2,)),
          ("w3", (H2, BINS)), ("b3", (BINS,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def round_bf16(a):
    """Rounds to the nearest BF16 value (8 significant bits, ties to even)."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64)).reshape(np.shape(a))


def _q(a, on):
    return round_bf16(a) if on else a


def unpack(flat):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def feature_freqs(f_lo, f_hi):
    return np.exp(np.linspace(np.log(f_lo), np.log(f_hi), M_FREQ))


def features(t, y, e, f_lo, f_hi):
    """[n, 80] features of one light curve."""
    t, y, e = (np.asarray(a, dtype=np.float64) for a in (t, y, e))
    w = 1.0 / (e * e)
    ybar = np.sum(w * y) / np.sum(w)
    sigma = np.sqrt(np.sum(w * (y - ybar) ** 2) / np.sum(w))
    tt = t - t.min()
    g = feature_freqs(f_lo, f_hi)
    ph = np.mod(np.outer(tt, g), 1.0)
    x = np.zeros((t.size, K1))
    x[:, 0:2 * M_FREQ:2] = np.sin(2 * np.pi * ph)
    x[:, 1:2 * M_FREQ:2] = np.cos(2 * np.pi * ph)
    x[:, 64] = (y - ybar) / sigma
    x[:, 65] = e / sigma
    x[:, ONE_SLOT] = 1.0
    return x


def bin_of(f, f_lo, f_hi):
    b = np.floor(BINS * np.log(np.asarray(f) / f_lo) / np.log(f_hi / f_lo)).astype(np.int64)
    return np.clip(b, 0, BINS - 1)


def bin_edges(f_lo, f_hi):
    return f_lo * (f_hi / f_lo) ** (np.arange(BINS + 1) / BINS)


def forward(params, feats, bf16=False):
    """feats: list of [n_o, 80] arrays.  Returns (logits [B, 1024], cache)."""
    p = unpack(params)
    w1, w2 = _q(p["w1"], bf16), _q(p["w2"], bf16)
    cache = []
    emb = np.zeros((len(feats), H2))
    for o, x in enumerate(feats):
        x = _q(x, bf16)
        a1 = x @ w1
        h1 = _q(np.maximum(a1, 0.0), bf16)
        a2 = h1 @ w2 + p["b2"]
        h2 = np.maximum(a2, 0.0)
        emb[o] = h2.mean(axis=0)
        cache.append((x, a1, h1, a2))
    logits = emb @ p["w3"] + p["b3"]
    return logits, (emb, cache)


def loss_and_grad(params, feats, labels, bf16=False):
    """Mean softmax cross-entropy over the batch and its gradient (flat)."""
    p = unpack(params)
    w2 = _q(p["w2"], bf16)
    logits, (emb, cache) = forward(params, feats, bf16)
    B = logits.shape[0]
    z = logits - logits.max(axis=1, keepdims=True)
    lse = np.log(np.exp(z).sum(axis=1))
    loss = float(np.mean(lse - z[np.arange(B), labels]))
    prob = np.exp(z - lse[:, None])
    dlog = prob
    dlog[np.arange(B), labels] -= 1.0
    dlog /= B
    g = {name: np.zeros(shp) for name, shp in SHAPES}
    g["w3"] = emb.T @ dlog
    g["b3"] = dlog.sum(axis=0)
    demb = dlog @ p["w3"].T
    for o, (x, a1, h1, a2) in enumerate(cache):
        n = x.shape[0]
        da2 = np.broadcast_to(demb[o] / n, a2.shape) * (a2 > 0)
        g["b2"] += da2.sum(axis=0)
        da2 = _q(da2, bf16)
        g["w2"] += h1.T @ da2
        da1 = _q((da2 @ w2.T) * (a1 > 0), bf16)
        g["w1"] += x.T @ da1
    return loss, pack(g)


def init_params(seed=0):
    """He-style initialisation (zero biases; rows 66..79 of w1 zero)."""
    rng = np.random.default_rng(seed)
    p = {"w1": rng.normal(0, np.sqrt(2.0 / 66), (K1, H1)),
         "w2": rng.normal(0, np.sqrt(2.0 / H1), (H1, H2)), "b2": np.zeros(H2),
         "w3": rng.normal(0, np.sqrt(1.0 / H2), (H2, BINS)), "b3": np.zeros(BINS)}
    p["w1"][ONE_SLOT:] = 0.0
    return pack(p)


def adam_step(params, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
