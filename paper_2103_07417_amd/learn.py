"""Training of the learned refinement proposal on the GPU.

The network (art.Cnn) is trained with its own BF16 MFMA forward/backward
kernels and Adam on the decisions of the refinement criterion (Sec. 3.2,
Eqs. 5-6): plain adaptive renders are traced, and at every level l where a
learned render runs the network (l + 2 <= N), the level-l features and the
15 per-vertex labels (was each new point of the next two levels traced?)
become one training sample.  Everything runs through the C ABI; this module
only orchestrates.
"""
import numpy as np

from . import art


def network_levels(levels, all_levels=False):
    """Levels l at which a learned render runs the network."""
    return [l for l in range(levels) if l + 2 <= levels or (all_levels and l + 1 <= levels)]


def training_set(cfgs, all_levels=False, stream=None):
    """{(level, H, W): (x, labels, valid)} stacked over the images whose
    level-l grids have the same shape (CUDA tensors)."""
    import torch
    by_level = {}
    for c in cfgs:
        img, lev, ft, st = art.render(c, feat=True, stream=stream)
        ls = network_levels(c["levels"], all_levels)
        # the loop of a learned render: network at l, then at l + 2
        l = 0
        while l < c["levels"]:
            if l in ls:
                x = art.cnn_features(c, img, ft, l, st["n_abs"], stream=stream)
                y, v = art.cnn_labels(c, lev, l, stream=stream)
                by_level.setdefault((l,) + tuple(x.shape[2:]), []).append((x, y, v))
                l += 2
            else:
                l += 1
    return {l: tuple(torch.cat([t[i] for t in items]) for i in range(3))
            for l, items in by_level.items()}


def positive_weight(data):
    """Weight of the positive class: sqrt(negatives / positives), in [1, 20]."""
    pos, n = 0.0, 0.0
    for _, y, v in data.values():
        m = v > 0
        pos += float(y[m].float().sum())
        n += float(m.sum())
    frac = max(pos / max(n, 1.0), 1e-6)
    return float(np.clip((1.0 - frac) / frac, 1.0, 400.0) ** 0.5)


def train(cfgs, steps=400, lr=3e-3, seed=4, net=None, all_levels=False, log=None, stream=None):
    """Train a proposal network on plain renders of cfgs; returns
    (net, dict(loss_first, loss_last, pos_weight, samples))."""
    data = training_set(cfgs, all_levels, stream=stream)
    pw = positive_weight(data)
    net = net or art.Cnn(seed=seed)
    first = {l: net.gradients(*d, pos_weight=pw, stream=stream)[0] for l, d in data.items()}
    for it in range(steps):
        for l, (x, y, v) in data.items():
            net.train_step(x, y, v, lr=lr, pos_weight=pw, want_loss=False, stream=stream)
        if log and (it + 1) % 100 == 0:
            log("train step %d" % (it + 1))
    last = {l: net.gradients(*d, pos_weight=pw, stream=stream)[0] for l, d in data.items()}
    info = dict(loss_first=first, loss_last=last, pos_weight=pw,
                samples={l: int(d[0].shape[0]) for l, d in data.items()})
    return net, info
