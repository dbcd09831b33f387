"""Element-wise tolerances for comparing the ordering network's GPU kernels
with the numpy oracle (test infrastructure, CPU only).

Both sides take the same rounding points (bf16 operands of every matrix
product, round to nearest even; float32 sums and element-wise work), so they
differ only through float32 summation order.  The bound carried here for
every intermediate is a bound on |GPU - oracle| for that element:
  * a float32 sum of n terms lies within gamma_n = n 2^-24 of sum |terms| of
    the exact sum, whatever the order, so two orders differ by at most twice
    that, plus the inputs' own bounds propagated through |weights|;
  * a bf16 rounding gives the identical value on both sides unless the
    interval value +- bound holds a rounding midpoint; then the two may differ
    by one bf16 unit (bound + unit, to be safe);
  * a ReLU whose input interval holds 0 may differ by the interval width in
    the forward pass, and its gradient mask may differ (the whole incoming
    gradient of that element).
"""
from __future__ import annotations

import numpy as np

from oracle import mlp

U = 2.0 ** -24


def gamma(n):
    return n * U / (1 - n * U)


def _ulp_bf16(a):
    """bf16 unit at |a| (8 significant bits); tiny values get the smallest normal's."""
    e = np.floor(np.log2(np.maximum(np.abs(a), 2.0 ** -126)))
    return 2.0 ** (e - 7)


def round_bound(a, err):
    """Bound on |bf16(a') - bf16(a)| for float32 values with |a' - a| <= err."""
    a = np.asarray(a, np.float64)
    r = mlp.bf16(a.astype(np.float32)).astype(np.float64)
    ulp = _ulp_bf16(r)
    # the unit below a power of two is half as large
    pow2 = (np.abs(r) > 0) & (np.abs(r) == 2.0 ** np.floor(np.log2(np.maximum(np.abs(r), 1e-300))))
    ulp_lo = np.where(pow2, ulp / 2, ulp)
    d_mid = ulp_lo / 2 - np.abs(a - r)       # distance from a to the nearest midpoint (lower bound)
    flip = d_mid <= err
    # an exact zero (a ReLU whose input is certainly negative) is zero on both sides
    return np.where(flip & (a != 0), 2 * err + _ulp_bf16(np.abs(r) + err), 0.0)


def forward_bounds(p, x, cls):
    """Oracle forward_bf16 values and bounds of |GPU - oracle| per element, plus
    the ReLU inputs whose sign is not fixed (a1 and a2)."""
    f = mlp.forward_bf16(p, x, cls)
    wb = {k: np.abs(mlp.bf16(p[k])).astype(np.float64) for k in ("w1x", "w1m", "w2", "w3")}
    xb = np.abs(f["xb"]).astype(np.float64)
    s1 = xb @ wb["w1x"].T + wb["w1m"][cls] + np.abs(p["b1"])
    e_a1 = 2 * gamma(x.shape[1] + 2) * s1
    amb1 = np.abs(f["a1"]) <= e_a1
    e_h1 = np.where(amb1, 2 * e_a1, round_bound(np.maximum(f["a1"], 0), e_a1))
    h1b = np.abs(f["h1b"]).astype(np.float64)
    s2 = h1b @ wb["w2"].T + np.abs(p["b2"])
    e_a2 = 2 * gamma(129) * (s2 + e_h1 @ wb["w2"].T) + e_h1 @ wb["w2"].T
    amb2 = np.abs(f["a2"]) <= e_a2
    e_h2 = np.where(amb2, 2 * e_a2, round_bound(np.maximum(f["a2"], 0), e_a2))
    h2b = np.abs(f["h2b"]).astype(np.float64)
    sz = h2b @ wb["w3"].T + np.abs(p["b3"])
    e_z = 2 * gamma(129) * (sz + e_h2 @ wb["w3"].T) + e_h2 @ wb["w3"].T
    return dict(f=f, e_a1=e_a1, e_h1=e_h1, e_a2=e_a2, e_h2=e_h2, e_z=e_z, amb1=amb1, amb2=amb2)


def grad_bounds(p, x, cls, label):
    """Oracle backward_bf16 gradients (mean softmax cross-entropy) and bounds of
    |GPU - oracle| per element."""
    fb = forward_bounds(p, x, cls)
    f = fb["f"]
    g, loss = mlp.backward_bf16(p, x, cls, label)
    B = x.shape[0]
    wb = {k: np.abs(mlp.bf16(p[k])).astype(np.float64) for k in ("w2", "w3")}
    z = f["z"].astype(np.float64)
    zm = z - z.max(1, keepdims=True)
    sm = np.exp(zm) / np.exp(zm).sum(1, keepdims=True)
    # softmax: the logits' bounds (d sm_c = sm_c (dz_c - sum sm dz)) and float32 exp,
    # sum and division (a few units each)
    e_sm = sm * (2 * fb["e_z"].max(1, keepdims=True)) + 16 * U * sm + gamma(64) * sm
    dz = sm.copy()
    dz[np.arange(B), label] -= 1
    dz /= B
    e_dz = e_sm / B + 4 * U * np.abs(dz)
    e_dzb = round_bound(dz, e_dz)
    adzb = np.abs(mlp.bf16(dz.astype(np.float32))).astype(np.float64)
    h2b, h1b, xb = (np.abs(f[k]).astype(np.float64) for k in ("h2b", "h1b", "xb"))
    tol = {}
    tol["w3"] = 2 * gamma(B) * (adzb.T @ h2b) + e_dzb.T @ (h2b + fb["e_h2"]) + adzb.T @ fb["e_h2"]
    tol["b3"] = 2 * gamma(B) * np.abs(dz).sum(0) + e_dz.sum(0)
    # da2 = (dzb w3b) masked by a2 > 0
    pre2 = adzb @ wb["w3"]
    e_pre2 = 2 * gamma(64) * pre2 + e_dzb @ wb["w3"]
    e_da2 = e_pre2 + np.where(fb["amb2"], pre2, 0.0)
    da2 = (mlp.bf16(dz.astype(np.float32)).astype(np.float64) @ mlp.bf16(p["w3"]).astype(np.float64)) \
        * (f["a2"] > 0)
    e_da2b = round_bound(da2, e_da2)
    ada2b = np.abs(mlp.bf16(da2.astype(np.float32))).astype(np.float64)
    tol["w2"] = 2 * gamma(B) * (ada2b.T @ h1b) + e_da2b.T @ (h1b + fb["e_h1"]) + ada2b.T @ fb["e_h1"]
    tol["b2"] = 2 * gamma(B) * np.abs(da2).sum(0) + e_da2.sum(0)
    pre1 = ada2b @ wb["w2"]
    e_pre1 = 2 * gamma(128) * pre1 + e_da2b @ wb["w2"]
    e_da1 = e_pre1 + np.where(fb["amb1"], pre1, 0.0)
    da1 = (mlp.bf16(da2.astype(np.float32)).astype(np.float64) @ mlp.bf16(p["w2"]).astype(np.float64)) \
        * (f["a1"] > 0)
    e_da1b = round_bound(da1, e_da1)
    ada1b = np.abs(mlp.bf16(da1.astype(np.float32))).astype(np.float64)
    tol["w1x"] = 2 * gamma(B) * (ada1b.T @ xb) + e_da1b.T @ xb
    tol["b1"] = 2 * gamma(B) * np.abs(da1).sum(0) + e_da1.sum(0)
    tol["w1m"] = np.zeros(np.shape(g["w1m"]))
    cnt = np.bincount(cls, minlength=np.shape(g["w1m"])[0]).astype(np.float64)
    np.add.at(tol["w1m"], cls, e_da1)
    tol["w1m"] += 2 * gamma(int(cnt.max()) + 1) * np.add.reduceat(
        np.abs(da1)[np.argsort(cls, kind="stable")], np.r_[0, np.cumsum(cnt)[:-1]].astype(int), axis=0) \
        * (cnt[:, None] > 0) if cnt.max() > 0 else 0
    return g, loss, tol


def alt_forward_backward(p, x, cls, label):
    """The same network with every float32 sum taken exactly (float64) and
    rounded once, and the softmax in float64: another float32 evaluation order
    of the oracle's arithmetic, for checking the bounds above on the CPU."""
    f64 = np.float64
    f32 = np.float32
    b = {k: mlp.bf16(p[k]).astype(f64) for k in ("w1x", "w1m", "w2", "w3")}
    xb = mlp.bf16(x).astype(f64)
    a1 = (xb @ b["w1x"].T + b["w1m"][cls] + p["b1"]).astype(f32)
    h1b = mlp.bf16(np.maximum(a1, f32(0))).astype(f64)
    a2 = (h1b @ b["w2"].T + p["b2"]).astype(f32)
    h2b = mlp.bf16(np.maximum(a2, f32(0))).astype(f64)
    z = (h2b @ b["w3"].T + p["b3"]).astype(f32)
    B = x.shape[0]
    zm = z.astype(f64) - z.max(1, keepdims=True)
    sm = np.exp(zm) / np.exp(zm).sum(1, keepdims=True)
    dz = sm.copy()
    dz[np.arange(B), label] -= 1
    dz = (dz / B).astype(f32)
    dzb = mlp.bf16(dz).astype(f64)
    g = {"w3": (dzb.T @ h2b).astype(f32), "b3": dz.astype(f64).sum(0).astype(f32)}
    da2 = ((dzb @ b["w3"]) * (a2 > 0)).astype(f32)
    da2b = mlp.bf16(da2).astype(f64)
    g["w2"] = (da2b.T @ h1b).astype(f32)
    g["b2"] = da2.astype(f64).sum(0).astype(f32)
    da1 = ((da2b @ b["w2"]) * (a1 > 0)).astype(f32)
    da1b = mlp.bf16(da1).astype(f64)
    g["w1x"] = (da1b.T @ xb).astype(f32)
    g["w1m"] = np.zeros(np.shape(p["w1m"]))
    np.add.at(g["w1m"], cls, da1.astype(f64))
    g["w1m"] = g["w1m"].astype(f32)
    g["b1"] = da1.astype(f64).sum(0).astype(f32)
    return z, g


def excess(a, ref, tol):
    """Largest |a - ref| / tol over the elements (<= 1 passes), and the count above 1."""
    d = np.abs(np.asarray(a, np.float64) - np.asarray(ref, np.float64))
    t = np.asarray(tol, np.float64) + 1e-30
    r = d / t
    return float(r.max()), int((d > t).sum())
