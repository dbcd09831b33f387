"""Pins of the numpy MLP oracle: finite differences, bf16 rounding, training."""
import numpy as np

from oracle import mlp


def _batch(rng, B=64, n_class=5):
    x = rng.normal(size=(B, mlp.NIN))
    cls = rng.integers(0, n_class, B)
    label = rng.integers(0, 8, B)
    return x, cls, label


def test_backward64_matches_finite_differences():
    rng = np.random.Generator(np.random.Philox(key=21))
    n_class = 5
    p = {k: v.astype(np.float64) for k, v in mlp.init(n_class, seed=1).items()}
    for k in ["b1", "b2", "b3"]:
        p[k] = rng.normal(0, 0.1, p[k].shape)
    x, cls, label = _batch(rng, n_class=n_class)
    g = mlp.backward64(p, x, cls, label)
    h = 1e-6
    for k in mlp.PARAMS:
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = mlp.loss64(p, x, cls, label)
            flat[i] = old - h
            lm = mlp.loss64(p, x, cls, label)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)) + 1e-9, (k, i, fd, an)


def test_bf16_rounding_nearest_even():
    f = np.float32
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -7 + 2 ** -8, -2.5, 0.0,
                     3.0e38, 1e-40], dtype=f)
    got = mlp.bf16(vals)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> even (1.0)
    assert got[0] == f(1.0) and got[1] == f(1.0)
    assert got[2] == f(1.0 + 2 ** -7)
    # 1 + 2^-7 + 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6 -> even (1 + 2^-6)
    assert got[3] == f(1.0 + 2 ** -6)
    assert got[4] == f(-2.5) and got[5] == f(0.0)
    # every result has a zero low half-word
    assert np.all(got.view(np.uint32) & 0xFFFF == 0)


def test_bf16_backward_close_to_float64():
    rng = np.random.Generator(np.random.Philox(key=22))
    n_class = 7
    p = mlp.init(n_class, seed=2)
    x, cls, label = _batch(rng, B=256, n_class=n_class)
    g16, _ = mlp.backward_bf16(p, x, cls, label)
    g64 = mlp.backward64({k: v.astype(np.float64) for k, v in p.items()}, x, cls, label)
    for k in mlp.PARAMS:
        a, b = g16[k].astype(np.float64), g64[k]
        assert np.linalg.norm(a - b) <= 0.05 * np.linalg.norm(b) + 1e-7, k


def test_adam_training_reduces_loss():
    rng = np.random.Generator(np.random.Philox(key=23))
    n_class = 3
    p = mlp.init(n_class, seed=4)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(val) for k, val in p.items()}
    x = rng.normal(size=(512, mlp.NIN)).astype(np.float32)
    cls = rng.integers(0, n_class, 512)
    label = (x[:, 0] > 0).astype(int) + 2 * (x[:, 3] > 0).astype(int) + cls  # learnable
    l0 = mlp.loss64({k: val.astype(np.float64) for k, val in p.items()}, x, cls, label)
    for t in range(1, 201):
        g, loss = mlp.backward_bf16(p, x, cls, label)
        p = mlp.adam_step(p, g, m, v, t, lr=3e-3)
    l1 = mlp.loss64({k: val.astype(np.float64) for k, val in p.items()}, x, cls, label)
    assert l1 < 0.5 * l0
    assert mlp.n_params(66) == 34112
