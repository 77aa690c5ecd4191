"""CPU reference of the per-variable fix predictor (float64 arithmetic).

TEST INFRASTRUCTURE ONLY: used by the test suite to check the GPU kernels.

Model (12 features padded to 16 -> 64 -> 64 -> 1):
    h1 = relu(W1 f + b1);  h2 = relu(W2 bf16(h1) + b2);  logit = w3 . h2 + b3
Rounding points (the GPU takes the same decisions in the same precision):
    f, W1, W2, w3 are bfloat16 values; h1 is rounded to bfloat16 before it
    enters the second product; h2 and the logit stay full precision.
Loss: binary cross-entropy with logits and a positive-class weight pw,
averaged over the minibatch:
    L = mean( -pw y log s(z) - (1 - y) log(1 - s(z)) ),
    dL/dz = (s(z) (pw y + 1 - y) - pw y) / B.
Backward rounding points: dh2 and dh1 are rounded to bfloat16 where they
enter products (dW2 = dh2 h1^T, dh1 = W2^T dh2, dW1 = dh1 f^T); bias
gradients use the unrounded values.  Adam (Kingma and Ba 2015) with bias
correction updates float32 master weights.
"""
from __future__ import annotations

import numpy as np

NF = 16  # padded feature width
H = 64


def bf16(a):
    """Round float values to bfloat16 (round to nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed: int):
    """Kaiming-uniform weights (bound sqrt(6 / fan_in)) from a seeded PCG64,
    zero biases; float32 master values."""
    rng = np.random.default_rng(seed)
    w1 = rng.uniform(-1, 1, (H, NF)) * np.sqrt(6.0 / 12.0)
    w1[:, 12:] = 0.0
    w2 = rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H)
    w3 = rng.uniform(-1, 1, H) * np.sqrt(6.0 / H)
    p = {"w1": w1, "b1": np.zeros(H), "w2": w2, "b2": np.zeros(H), "w3": w3, "b3": np.zeros(1)}
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def forward(p, f):
    """f: (B, 16) -> logits (B,), with the cache for backward."""
    fb = bf16(f)
    a1 = fb @ bf16(p["w1"]).T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    h1b = bf16(h1)
    a2 = h1b @ bf16(p["w2"]).T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ bf16(p["w3"]) + p["b3"][0]
    return z, (fb, a1, h1b, a2, h2)


def loss_and_grad(p, f, y, pw):
    z, (fb, a1, h1b, a2, h2) = forward(p, f)
    bsz = f.shape[0]
    s = 1.0 / (1.0 + np.exp(-z))
    loss = np.mean(-pw * y * np.log(np.maximum(s, 1e-300)) - (1 - y) * np.log(np.maximum(1 - s, 1e-300)))
    dz = (s * (pw * y + 1.0 - y) - pw * y) / bsz
    g = {}
    g["w3"] = dz @ h2
    g["b3"] = np.array([dz.sum()])
    dh2 = np.outer(dz, bf16(p["w3"])) * (a2 > 0)
    g["b2"] = dh2.sum(axis=0)
    dh2b = bf16(dh2)
    g["w2"] = dh2b.T @ h1b
    dh1 = (dh2b @ bf16(p["w2"])) * (a1 > 0)
    g["b1"] = dh1.sum(axis=0)
    g["w1"] = bf16(dh1).T @ fb
    return loss, g, z


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on float32 master weights; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    out = {}
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        out[k] = (p[k] - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32).astype(np.float64)
    return out


def flat(p):
    """Parameter vector in the library's order: w1 (64x16), b1, w2 (64x64), b2, w3, b3."""
    return np.concatenate([p["w1"].ravel(), p["b1"], p["w2"].ravel(), p["b2"], p["w3"], p["b3"]])


def unflat(v):
    v = np.asarray(v, dtype=np.float64)
    o = 0
    p = {}
    for k, shp in (("w1", (H, NF)), ("b1", (H,)), ("w2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))):
        sz = int(np.prod(shp))
        p[k] = v[o:o + sz].reshape(shp).copy()
        o += sz
    return p


N_PARAMS = H * NF + H + H * H + H + H + 1
