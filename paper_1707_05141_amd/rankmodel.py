"""Training the rank-prediction network from generated blocks.

Labels are the ranks that the plain FP64 randomized SVD of this library computes at tolerance eps
(adaptive range finder + exact check, i.e. the exact truncation rank up to near-ties). Features are
the library's probe features. Training runs on the GPU through the library's own forward, backward
and Adam kernels (``RankModel.train``). The margin added to the prediction is calibrated on the
training blocks so that the first sample block covers the rank plus an oversampling of ``oversample``
for the ``coverage`` quantile of the blocks; the rest fall back to adaptive growth. The quantile is
moderate (0.8): for high-rank blocks an overshoot costs more (the small SVD grows with the cube of
the sample count) than the few growth rounds an undershoot adds.
"""
from __future__ import annotations

import numpy as np
import torch

from . import RankModel, pack_colmajor, rank_features, rsvd_packed


def labels_and_features(buf, offs, m, n, eps=1e-6, seed=0, max_rank=64):
    """(features [b, 16] float32 device tensor, ranks [b] int numpy) of a packed batch."""
    res = rsvd_packed(buf, offs, m, n, eps=eps, max_rank=max_rank, seed=seed, want_vectors=False)
    feats = rank_features(buf, offs, m, n, seed=seed)
    torch.cuda.synchronize()
    ok = res["info"].cpu().numpy() == 0
    return feats, res["rank"].cpu().numpy(), ok


def train_packed(buf, offs, m, n, *, eps=1e-6, seed=0, epochs=150, batch=256, lr=2e-3, oversample=6.0,
                 coverage=0.8, device=None, max_rank=64):
    feats, ranks, ok = labels_and_features(buf, offs, m, n, eps=eps, seed=seed, max_rank=max_rank)
    idx = np.nonzero(ok)[0]
    X = feats[torch.from_numpy(idx).to(feats.device)]
    T = torch.from_numpy((ranks[idx] / 16.0).astype(np.float32))
    model = RankModel(device if device is not None else buf.device)
    model.init(seed=seed)
    loss = model.train(X, T, epochs=epochs, batch=min(batch, len(idx)), lr=lr, seed=seed + 1)
    pred = model.forward(X).cpu().numpy() * 16.0
    gap = ranks[idx] - pred
    margin = float(np.quantile(gap, coverage)) + oversample
    p, _ = model.get()
    model.set(p, margin=margin)
    model.stats = dict(train_loss=loss, n=len(idx), margin=margin,
                       mae=float(np.mean(np.abs(gap))), max_under=float(gap.max()))
    return model


def train_from_blocks(mats, **kw):
    """Train from a list of numpy blocks (packed onto the GPU first)."""
    buf, offs, m, n = pack_colmajor(mats)
    return train_packed(buf, offs, m, n, **kw)
