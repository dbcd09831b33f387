"""GPU: the MLP training kernels (bf16 MFMA) against the numpy oracle."""
import sys

import numpy as np
import pytest

from oracle import mlp

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


def test_mlp_forward_matches_numpy(dev):
    torch, gnav, ctx = dev
    print_case("mlp_forward")
    n_class = 66
    p = mlp.init(n_class, seed=3)
    for k in ["b1", "b2", "b3"]:
        p[k] = np.random.default_rng(1).normal(0, 0.1, p[k].shape).astype(np.float32)
    net = gnav.MLP(ctx, n_class, p, max_batch=256)
    x, cls, _ = _data(256, n_class, 5)
    z = net.forward(torch.from_numpy(x).cuda(), torch.from_numpy(cls).cuda()).cpu().numpy()
    ref = mlp.forward_bf16(p, x, cls)["z"]
    assert rel(z, ref) < 1e-3
    # the same argmax for clearly separated logits
    top = np.sort(ref, axis=1)
    clear = (top[:, -1] - top[:, -2]) > 1e-2 * np.abs(top[:, -1]).clip(1e-3)
    assert np.array_equal(z.argmax(1)[clear], ref.argmax(1)[clear])
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
    ref, ref_loss = mlp.backward_bf16(p, x, cls, label)
    assert abs(float(loss.cpu()[0]) - ref_loss) < 1e-4 * abs(ref_loss)
    for k in mlp.PARAMS:
        assert rel(g[k], ref[k]) < 5e-3, (k, rel(g[k], ref[k]))
    net.free()


def test_mlp_training_matches_numpy_adam(dev):
    """Adam on the GPU follows the numpy oracle.

    Adam divides each update by the root of its running squared gradient, so
    components whose gradient is near zero move by about the learning rate
    whatever the sign of the rounding noise: parameters of two runs that differ
    only in accumulation order drift apart over many steps.  The parameters are
    therefore compared element-wise after a few steps, and the long run by its
    loss curve.
    """
    torch, gnav, ctx = dev
    print_case("mlp_adam")
    n_class = 3
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
    losses, ref_losses = [], []
    for t in range(1, 101):
        loss = net.step(xt, ct, lt, lr=3e-3, want_loss=True)
        losses.append(float(loss.cpu()[0]))
        g, ref_loss = mlp.backward_bf16(pn, x, cls, label)
        ref_losses.append(ref_loss)
        pn = mlp.adam_step(pn, g, m, v, t, lr=3e-3)
        if t == 3:
            got = net.params()
            for k in mlp.PARAMS:
                assert rel(got[k], pn[k]) < 1e-2, (k, rel(got[k], pn[k]))
    assert losses[-1] < 0.5 * losses[0]
    assert ref_losses[-1] < 0.5 * ref_losses[0]
    for a, b in zip(losses, ref_losses):
        assert abs(a - b) <= 0.1 * b + 1e-3, (a, b)
    net.free()
