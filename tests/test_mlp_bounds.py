"""CPU: the element-wise bounds used to compare the ordering network's GPU
kernels with the numpy oracle.  Another float32 evaluation order of the same
arithmetic (exact sums rounded once, softmax in float64) must stay inside
them, and a planted mistake (a transposed weight matrix) must not."""
import numpy as np

from oracle import mlp
from tests import mlp_bounds as mb


def _case(seed):
    n_class = 66
    p = mlp.init(n_class, seed=seed)
    rng = np.random.Generator(np.random.Philox(key=100 + seed))
    x = rng.normal(size=(512, mlp.NIN)).astype(np.float32)
    cls = rng.integers(0, n_class, 512).astype(np.int32)
    label = rng.integers(0, 64, 512).astype(np.int32)
    return p, x, cls, label


def test_other_summation_order_within_bounds():
    for seed in (4, 5, 6):
        p, x, cls, label = _case(seed)
        fb = mb.forward_bounds(p, x, cls)
        z, g = mb.alt_forward_backward(p, x, cls, label)
        assert mb.excess(z, fb["f"]["z"], fb["e_z"])[1] == 0
        ref, _, tol = mb.grad_bounds(p, x, cls, label)
        for k in mlp.PARAMS:
            assert mb.excess(g[k], ref[k], tol[k])[1] == 0, k
        # and the bounds are tight where they should be: logits within 1 % of |z|
        assert np.median(fb["e_z"] / (np.abs(fb["f"]["z"]) + 1e-3)) < 1e-2


def test_planted_transpose_exceeds_bounds():
    p, x, cls, label = _case(4)
    fb = mb.forward_bounds(p, x, cls)
    ref, _, tol = mb.grad_bounds(p, x, cls, label)
    bad = dict(p)
    bad["w2"] = np.ascontiguousarray(p["w2"].T)
    z, g = mb.alt_forward_backward(bad, x, cls, label)
    assert mb.excess(z, fb["f"]["z"], fb["e_z"])[1] > 1000
    for k in ("w2", "b2", "w3", "b3"):
        assert mb.excess(g[k], ref[k], tol[k])[1] > 0, k
    bad = dict(p)
    bad["w3"] = p["w3"][::-1].copy()     # logits in reversed candidate order
    z, _ = mb.alt_forward_backward(bad, x, cls, label)
    assert mb.excess(z, fb["f"]["z"], fb["e_z"])[1] > 1000
