"""Numpy oracle of the candidate-ordering MLP (test infrastructure only).

The network ranks the voxel candidates of a ComputeStep: inputs are the
point and direction in the mother frame (6 numbers) plus a one-hot of the
mother volume (realised as a row gather of the first layer's weights); two
hidden layers of 128 ReLU units; 64 logits, one per candidate position in
the start voxel node.  Training minimises softmax cross-entropy against the
position of the daughter that limited the step, with Adam.

Two versions:
  * ``forward64`` / ``backward64``: plain float64 maths, pinned against
    central finite differences;
  * ``forward_bf16`` / ``backward_bf16``: the GPU's numerics -- operands of
    every matrix product rounded to bfloat16 (round to nearest even),
    float32 accumulation and element-wise work -- so the GPU kernels can be
    compared element by element up to accumulation order.
"""
from __future__ import annotations

import numpy as np

NIN = 6
NH = 128
NOUT = 64

PARAMS = ["w1x", "w1m", "b1", "w2", "b2", "w3", "b3"]


def shapes(n_class):
    return {"w1x": (NH, NIN), "w1m": (n_class, NH), "b1": (NH,), "w2": (NH, NH), "b2": (NH,),
            "w3": (NOUT, NH), "b3": (NOUT,)}


def init(n_class, seed=3):
    """He-normal weights (fan-in of the dense inputs), zero biases."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    sh = shapes(n_class)
    p = {}
    p["w1x"] = rng.normal(0, np.sqrt(2.0 / NIN), sh["w1x"])
    p["w1m"] = rng.normal(0, np.sqrt(2.0 / NIN), sh["w1m"]) * 0.1
    p["b1"] = np.zeros(NH)
    p["w2"] = rng.normal(0, np.sqrt(2.0 / NH), sh["w2"])
    p["b2"] = np.zeros(NH)
    p["w3"] = rng.normal(0, np.sqrt(2.0 / NH), sh["w3"])
    p["b3"] = np.zeros(NOUT)
    return {k: v.astype(np.float32) for k, v in p.items()}


def n_params(n_class):
    return sum(int(np.prod(s)) for s in shapes(n_class).values())


# ---------------------------------------------------------------------------
# float64 reference
# ---------------------------------------------------------------------------

def forward64(p, x, cls):
    a1 = x @ p["w1x"].T + p["w1m"][cls] + p["b1"]
    h1 = np.maximum(a1, 0)
    a2 = h1 @ p["w2"].T + p["b2"]
    h2 = np.maximum(a2, 0)
    z = h2 @ p["w3"].T + p["b3"]
    return dict(a1=a1, h1=h1, a2=a2, h2=h2, z=z)


def loss64(p, x, cls, label):
    z = forward64(p, x, cls)["z"]
    zm = z - z.max(axis=1, keepdims=True)
    lse = np.log(np.exp(zm).sum(axis=1))
    return float(np.mean(lse - zm[np.arange(len(label)), label]))


def backward64(p, x, cls, label):
    f = forward64(p, x, cls)
    B = x.shape[0]
    z = f["z"] - f["z"].max(axis=1, keepdims=True)
    sm = np.exp(z)
    sm /= sm.sum(axis=1, keepdims=True)
    dz = sm.copy()
    dz[np.arange(B), label] -= 1.0
    dz /= B
    g = {}
    g["w3"] = dz.T @ f["h2"]
    g["b3"] = dz.sum(0)
    da2 = (dz @ p["w3"]) * (f["a2"] > 0)
    g["w2"] = da2.T @ f["h1"]
    g["b2"] = da2.sum(0)
    da1 = (da2 @ p["w2"]) * (f["a1"] > 0)
    g["w1x"] = da1.T @ x
    g["w1m"] = np.zeros_like(p["w1m"], dtype=np.float64)
    np.add.at(g["w1m"], cls, da1)
    g["b1"] = da1.sum(0)
    return g


# ---------------------------------------------------------------------------
# bfloat16 mirror of the GPU numerics
# ---------------------------------------------------------------------------

def bf16(a):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    if nan.any():
        out = out.copy()
        out[nan] = np.float32(np.nan)
    return out


def _mm(a, b):
    return (a.astype(np.float32) @ b.astype(np.float32)).astype(np.float32)


def forward_bf16(p, x, cls):
    f32 = np.float32
    xb = bf16(x)
    a1 = _mm(xb, bf16(p["w1x"]).T) + bf16(p["w1m"])[cls] + p["b1"].astype(f32)
    h1 = np.maximum(a1, f32(0))
    h1b = bf16(h1)
    a2 = _mm(h1b, bf16(p["w2"]).T) + p["b2"].astype(f32)
    h2b = bf16(np.maximum(a2, f32(0)))
    z = _mm(h2b, bf16(p["w3"]).T) + p["b3"].astype(f32)
    return dict(xb=xb, a1=a1, h1b=h1b, a2=a2, h2b=h2b, z=z)


def backward_bf16(p, x, cls, label):
    f32 = np.float32
    f = forward_bf16(p, x, cls)
    B = x.shape[0]
    z = f["z"] - f["z"].max(axis=1, keepdims=True)
    e = np.exp(z).astype(f32)
    sm = e / e.sum(axis=1, keepdims=True)
    dz = sm.astype(f32)
    dz[np.arange(B), label] -= f32(1)
    dz = (dz / f32(B)).astype(f32)
    dzb = bf16(dz)
    g = {}
    g["w3"] = _mm(dzb.T, f["h2b"])
    g["b3"] = dz.sum(0, dtype=f32)
    da2 = _mm(dzb, bf16(p["w3"])) * (f["a2"] > 0)
    da2b = bf16(da2)
    g["w2"] = _mm(da2b.T, f["h1b"])
    g["b2"] = da2.sum(0, dtype=f32)
    da1 = _mm(da2b, bf16(p["w2"])) * (f["a1"] > 0)
    da1b = bf16(da1)
    g["w1x"] = _mm(da1b.T, f["xb"])
    g["w1m"] = np.zeros_like(p["w1m"], dtype=f32)
    np.add.at(g["w1m"], cls, da1.astype(f32))
    g["b1"] = da1.sum(0, dtype=f32)
    zm = f["z"] - f["z"].max(axis=1, keepdims=True)
    loss = float(np.mean(np.log(np.exp(zm).sum(1)) - zm[np.arange(B), label]))
    return g, loss


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (float32), t >= 1 is the step number."""
    f32 = np.float32
    out = {}
    c1 = f32(1 - b1 ** t)
    c2 = f32(1 - b2 ** t)
    for k in PARAMS:
        m[k] = (f32(b1) * m[k] + f32(1 - b1) * g[k]).astype(f32)
        v[k] = (f32(b2) * v[k] + f32(1 - b2) * g[k] * g[k]).astype(f32)
        mh = m[k] / c1
        vh = v[k] / c2
        out[k] = (p[k] - f32(lr) * mh / (np.sqrt(vh) + f32(eps))).astype(f32)
    return out


def predict_order(p, x, cls):
    """Candidate positions sorted by decreasing logit (float64 forward)."""
    z = forward64(p, x, cls)["z"]
    return np.argsort(-z, axis=1, kind="stable")
