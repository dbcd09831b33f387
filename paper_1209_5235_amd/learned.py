"""Learned candidate ordering: record crossings, train the network on the GPU.

The transport itself records daughter-limited steps (the crossing recorder
of the C ABI); the network is trained with the library's bf16 MFMA kernels
(gnav_mlp_grad / gnav_mlp_adam) and then handed to the transport
(gnav_set_mlp, order 2).  Results of a learned-order run are identical to
the plain voxel walk; only the order in which the start node's candidates
are examined changes.
"""
from __future__ import annotations

import numpy as np

from . import gnav


def init_params(n_class, seed=3):
    """He-normal weights from a stated seed, zero biases (float32)."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    p = {
        "w1x": rng.normal(0, np.sqrt(2.0 / 6), (128, 6)),
        "w1m": rng.normal(0, np.sqrt(2.0 / 6), (n_class, 128)) * 0.1,
        "b1": np.zeros(128),
        "w2": rng.normal(0, np.sqrt(2.0 / 128), (128, 128)),
        "b2": np.zeros(128),
        "w3": rng.normal(0, np.sqrt(2.0 / 128), (64, 128)),
        "b3": np.zeros(64),
    }
    return {k: v.astype(np.float32) for k, v in p.items()}


def record_crossings(ctx, geom_id, prim_dev, n_events, capacity, seed=1, stream=None):
    """Run one plain transport batch with the recorder on; returns the records."""
    import torch
    rec = gnav.make_recorder(capacity, prim_dev["pos"].device)
    tally = ctx.tally_create(n_events)
    ctx.transport_batch(geom_id, prim_dev, tally, seed=seed, record=rec, stream=stream)
    torch.cuda.synchronize()
    tally.free()
    return rec


def records_to_tensors(rec):
    """Device tensors (x [n][6] float32, cls [n], label [n]) from recorder buffers."""
    import torch
    n = min(int(rec["count"].cpu()[0]), rec["cap"])
    raw = rec["rec"][:n]
    cls = raw[:, 0].contiguous()
    feats = raw[:, 1:7].contiguous().view(torch.float32)
    label = raw[:, 7].contiguous()
    return feats, cls, label


def train(ctx, n_class, x, cls, label, epochs=1, batch=4096, lr=1e-3, seed=3, params=None,
          log_every=0):
    """Adam over shuffled mini-batches of the recorded crossings (GPU kernels)."""
    import torch
    net = gnav.MLP(ctx, n_class, params if params is not None else init_params(n_class, seed),
                   max_batch=batch)
    n = (x.shape[0] // batch) * batch
    g = torch.Generator(device=x.device)
    g.manual_seed(seed)
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(x.shape[0], device=x.device, generator=g)[:n]
        xs, cs, ls = x[perm].contiguous(), cls[perm].contiguous(), label[perm].contiguous()
        for i in range(0, n, batch):
            want = log_every and (i // batch) % log_every == 0
            loss = net.step(xs[i:i + batch], cs[i:i + batch], ls[i:i + batch], lr=lr, want_loss=want)
            if want:
                losses.append(float(loss.cpu()[0]))
    return net, losses


def accuracy(net, x, cls, label, batch=4096):
    """Fraction of crossings whose top-scored candidate is the limiting one."""
    import torch
    n = (x.shape[0] // 16) * 16
    hits = 0
    for i in range(0, n, batch):
        j = min(i + batch, n)
        z = net.forward(x[i:j].contiguous(), cls[i:j].contiguous())
        hits += int((z.argmax(1).to(torch.int32) == label[i:j]).sum())
    return hits / max(n, 1)
