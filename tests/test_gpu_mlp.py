"""GPU: the ordering network's kernels (bf16 MFMA, FP32 accumulation) against
the numpy oracle, element by element.

Both sides round at the same points, so they differ only by float32
summation order and what it does downstream (a bf16 rounding or a ReLU
decided the other way).  `tests/mlp_bounds.py` carries, for every
intermediate value, a bound on that difference derived from the arithmetic;
each element must lie within its bound.  The relative L2 norm of each
gradient block is checked as well (it catches a wrong first layer, whose
element bounds are the loosest).
"""
import sys

import numpy as np
import pytest

from oracle import mlp
from tests import mlp_bounds as mb

pytestmark = pytest.mark.gpu


def print_case(*a):
    print("CASE", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1209_5235_amd import gnav
    ctx = gnav.Context(0)
    yield torch, gnav, ctx
    ctx.close()


def _data(B, n_class, seed):
    rng = np.random.Generator(np.random.Philox(key=seed))
    x = rng.normal(size=(B, mlp.NIN)).astype(np.float32)
    cls = rng.integers(0, n_class, B).astype(np.int32)
    label = rng.integers(0, 64, B).astype(np.int32)
    return x, cls, label


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


def _params(n_class, seed, bias_seed):
    p = mlp.init(n_class, seed=seed)
    for k in ["b1", "b2", "b3"]:
        p[k] = np.random.default_rng(bias_seed).normal(0, 0.1, p[k].shape).astype(np.float32)
    return p


def _check_logits(z, fb, what):
    ref = fb["f"]["z"]
    worst, n_over = mb.excess(z, ref, fb["e_z"])
    assert n_over == 0, (what, worst, n_over)
    # the argmax wherever the top two logits are further apart than their bounds
    i1 = ref.argmax(1)
    top = np.sort(ref, axis=1)
    e = fb["e_z"].max(1)
    clear = (top[:, -1] - top[:, -2]) > 2 * e
    assert clear.mean() > 0.9, clear.mean()
    return i1, clear


def test_mlp_forward_matches_numpy(dev):
    """gnav_mlp_forward (the training kernels' forward) element by element."""
    torch, gnav, ctx = dev
    print_case("mlp_forward")
    n_class = 66
    p = _params(n_class, 3, 1)
    net = gnav.MLP(ctx, n_class, p, max_batch=1024)
    x, cls, _ = _data(1024, n_class, 5)
    z = net.forward(torch.from_numpy(x).cuda(), torch.from_numpy(cls).cuda()).cpu().numpy()
    i1, clear = _check_logits(z, mb.forward_bounds(p, x, cls), "forward")
    assert np.array_equal(z.argmax(1)[clear], i1[clear])
    net.free()


@pytest.mark.parametrize("n", [1000, 4099])
def test_transport_scoring_matches_numpy(dev, n):
    """gnav_mlp_score runs the device code that the transport and the
    ComputeStep query use for the learned order (16-row MFMA tiles, layers
    computed transposed): logits element by element, and the predicted
    position is the oracle's argmax wherever the top two logits are separated
    (ragged last tile included)."""
    torch, gnav, ctx = dev
    print_case("mlp_score", n)
    n_class = 66
    p = _params(n_class, 11, 2)
    net = gnav.MLP(ctx, n_class, p, max_batch=64)
    x, cls, _ = _data(n, n_class, 9)
    logits, pred = net.score(torch.from_numpy(x).cuda(), torch.from_numpy(cls).cuda())
    z, pred = logits.cpu().numpy(), pred.cpu().numpy()
    i1, clear = _check_logits(z, mb.forward_bounds(p, x, cls), "score")
    assert np.array_equal(pred[clear], i1[clear])
    # the prediction is the first maximum of the logits it returned
    assert np.array_equal(pred, z.argmax(1))
    net.free()


def test_mlp_gradients_match_numpy(dev):
    torch, gnav, ctx = dev
    print_case("mlp_grad")
    n_class = 66
    p = mlp.init(n_class, seed=4)
    net = gnav.MLP(ctx, n_class, p, max_batch=1024)
    x, cls, label = _data(1024, n_class, 6)
    g, loss = net.grad(torch.from_numpy(x).cuda(), torch.from_numpy(cls).cuda(),
                       torch.from_numpy(label).cuda())
    g = net.unflatten(g.cpu().numpy())
    ref, ref_loss, tol = mb.grad_bounds(p, x, cls, label)
    assert abs(float(loss.cpu()[0]) - ref_loss) < 1e-4 * abs(ref_loss)
    for k in mlp.PARAMS:
        worst, n_over = mb.excess(g[k], ref[k], tol[k])
        assert n_over == 0, (k, worst, n_over)
        assert rel(g[k], ref[k]) < 5e-3, (k, rel(g[k], ref[k]))
    net.free()


def test_mlp_training_matches_numpy_adam(dev):
    """Adam on the GPU follows the numpy oracle, element by element over the
    first ten steps, then by its loss curve.

    A component's update lr m/(sqrt(v) + eps) can differ between the two sides
    by at most about lr times the gradient's relative bound (capped at 2 lr,
    a sign flip), summed over the steps so far."""
    torch, gnav, ctx = dev
    print_case("mlp_adam")
    n_class = 3
    lr = 3e-3
    p = mlp.init(n_class, seed=7)
    net = gnav.MLP(ctx, n_class, p, max_batch=512)
    rng = np.random.Generator(np.random.Philox(key=8))
    x = rng.normal(size=(512, mlp.NIN)).astype(np.float32)
    cls = rng.integers(0, n_class, 512).astype(np.int32)
    label = ((x[:, 0] > 0).astype(int) + 2 * (x[:, 3] > 0).astype(int) + cls).astype(np.int32)
    xt, ct, lt = (torch.from_numpy(a).cuda() for a in (x, cls, label))
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(val) for k, val in p.items()}
    pn = dict(p)
    allow = {k: np.zeros(np.shape(p[k])) for k in p}
    losses, ref_losses = [], []
    for t in range(1, 101):
        loss = net.step(xt, ct, lt, lr=lr, want_loss=True)
        losses.append(float(loss.cpu()[0]))
        if t <= 10:
            g, ref_loss, tol = mb.grad_bounds(pn, x, cls, label)
        else:
            g, ref_loss = mlp.backward_bf16(pn, x, cls, label)
        ref_losses.append(ref_loss)
        pn = mlp.adam_step(pn, g, m, v, t, lr=lr)
        if t <= 10:
            got = net.params()
            for k in mlp.PARAMS:
                allow[k] += lr * np.minimum(2.0, 4 * tol[k] / (np.abs(g[k]) + 1e-30))
                worst, n_over = mb.excess(got[k], pn[k], allow[k] + 1e-6 * np.abs(pn[k]))
                assert n_over == 0, (t, k, worst, n_over)
    assert losses[-1] < 0.5 * losses[0]
    assert ref_losses[-1] < 0.5 * ref_losses[0]
    for a, b in zip(losses, ref_losses):
        assert abs(a - b) <= 0.1 * b + 1e-3, (a, b)
    net.free()
