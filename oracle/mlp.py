"""Reference of the per-material surrogate network (beyond the paper).

The paper caches sub-graph outputs exactly; the surrogate is an added model
that approximates the deep cacheable sub-graphs of a material from UV and is
trusted only where its measured error is small.  Definitions used by both
this reference and the HIP kernels:

  features   x = [sin(w_k u), cos(w_k u), sin(w_k v), cos(w_k v)] for
             k = 0..7, w_k = 2 pi 2^(k - 4)  (32 values; periods 16 .. 1/8 UV)
  network    h1 = relu(W1 x + b1)   W1: 64 x 32
             h2 = relu(W2 h1 + b2)  W2: 64 x 64
             y  = W3 h2 + b3        W3: 4 x 64
  loss       L = sum over used channels of (y - t)^2 / N   (N = used entries)
  optimiser  Adam (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master weights

FP16 rounding points of the GPU path (``round16=True``): x, the weights, h1
and h2 are rounded to binary16 before each product; products accumulate in
FP32 (here FP64).  In the backward pass the output gradient is
2 (y - t) * mask (the 1/N factor is applied to the weight gradients in FP32,
which keeps the FP16 values in the normal range); dH2 and dH1 are rounded to
binary16 before their products.

Batch sampling uses a counter-based generator so both sides draw the same
indices: index(step, i) = mix64(seed ^ (step << 32 | i)) mod n_train, with the
SplitMix64 finalizer (see hashing.py).

Shading with the network: a missed (not bypassed) surrogated output of a
trusted material takes the network's value, unless the hit is audited:
hit h of frame f is audited when mix64(((f << 32) | h) ^ SEED_AUDIT) >> 58 is 0
(one in 64); audited hits are evaluated by the graph as usual.
"""
import numpy as np

from .hashing import mix64

N_FEAT, N_HID, N_OUT = 32, 64, 4
N_PARAMS = 6532
SEED_AUDIT = 0xD6E8FEB86659FD93
_SHAPES = ((64, 32), (64,), (64, 64), (64,), (4, 64), (4,))
OMEGA = 2.0 * np.pi * 2.0 ** (np.arange(8) - 4.0)


def features(uv):
    uv = np.asarray(uv, dtype=np.float64)
    cols = []
    for w in OMEGA:
        cols += [np.sin(w * uv[:, 0]), np.cos(w * uv[:, 0]), np.sin(w * uv[:, 1]),
                 np.cos(w * uv[:, 1])]
    return np.stack(cols, 1)


def f16(a):
    return np.asarray(a, dtype=np.float64).astype(np.float16).astype(np.float64)


def forward(params, x, round16=False):
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    r = f16 if round16 else (lambda a: np.asarray(a, dtype=np.float64))
    x = r(x)
    a1 = x @ r(W1).T + b1
    h1 = r(np.maximum(a1, 0.0))
    a2 = h1 @ r(W2).T + b2
    h2 = r(np.maximum(a2, 0.0))
    y = h2 @ r(W3).T + b3
    return y, dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2)


def loss_and_grads(params, x, target, mask, round16=False):
    """mask [n, 4] of 0/1: used output channels.  Returns (loss, grads list)."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    r = f16 if round16 else (lambda a: np.asarray(a, dtype=np.float64))
    y, c = forward(params, x, round16)
    mask = np.asarray(mask, dtype=np.float64)
    n_used = max(mask.sum(), 1.0)
    diff = (y - target) * mask
    loss = float((diff ** 2).sum() / n_used)
    dy = r(2.0 * diff)                             # scaled by N (applied below)
    gW3 = dy.T @ c["h2"]
    gb3 = dy.sum(0)
    dh2 = r((dy @ r(W3)) * (c["a2"] > 0))
    gW2 = dh2.T @ c["h1"]
    gb2 = dh2.sum(0)
    dh1 = r((dh2 @ r(W2)) * (c["a1"] > 0))
    gW1 = dh1.T @ c["x"]
    gb1 = dh1.sum(0)
    grads = [g / n_used for g in (gW1, gb1, gW2, gb2, gW3, gb3)]
    return loss, grads


def adam_update(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mh = mm / (1 - b1 ** step)
        vh = vv / (1 - b2 ** step)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v


def unflatten(flat):
    """Flat parameter vector (W1, b1, W2, b2, W3, b3; W row-major [out][in]) -> list."""
    flat = np.asarray(flat, dtype=np.float64).ravel()
    out, k = [], 0
    for shp in _SHAPES:
        n = int(np.prod(shp))
        out.append(flat[k:k + n].reshape(shp))
        k += n
    assert k == N_PARAMS
    return out


def flatten(params):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in params])


def audited(frame, h):
    h = np.asarray(h, dtype=np.uint64)
    z = mix64(((np.uint64(frame) << np.uint64(32)) | h) ^ np.uint64(SEED_AUDIT))
    return (z >> np.uint64(58)) == 0


def targets(records, ordmap):
    """Training targets and channel masks of log records.

    records: structured array with fields ordinal and value[4]; ordmap: dict
    ordinal -> (first channel, width).  Returns (target [n, 4], mask [n, 4]).
    """
    n = len(records)
    t = np.zeros((n, N_OUT))
    m = np.zeros((n, N_OUT))
    for i in range(n):
        o = int(records["ordinal"][i])
        if o not in ordmap:
            continue
        base, width = ordmap[o]
        t[i, base:base + width] = records["value"][i][:width]
        m[i, base:base + width] = 1.0
    return t, m


def batch_indices(seed, step, batch, n_train):
    i = np.arange(batch, dtype=np.uint64)
    z = mix64(np.uint64(seed) ^ ((np.uint64(step) << np.uint64(32)) | i))
    return (z % np.uint64(n_train)).astype(np.int64)
