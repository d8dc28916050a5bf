"""Training and use of the learned neighbor proposal (include/vif_learn.h).

Every arithmetic step runs in libvif.so: features, forward and backward
passes, the contrastive loss, Adam, batch assembly, the exact neighbor lists
used as labels, and the proposal search. PyTorch provides device memory and
the uniform random integers that pick queries and random negatives.

Training data: station-network problems like the continental workload (many
seeds, spread over the year; half of them with hyperparameters perturbed around
the workload's: +-1 in log for a and c, +-1 in logit for alpha, beta, gamma),
labelled by the exact search (vif_neighbors with 2m neighbors: the first m are
the positives, the next m the hard negatives), plus random earlier points as
easy negatives.
"""
from __future__ import annotations

import math
import time

from . import _lib as L

# Feature centre: workload-scale coordinates (km) and days, and the continental
# kernel's log hyperparameters (a = 1.0956, c = 2.1277e-3, alpha = 0.75,
# beta = gamma = 0.5). Time is scaled by 5 days, so that one day of lag weighs
# about as much as the few hundred km of distance it is worth in correlation.
CENTRE = (0.0, 0.0, 182.0, 1400.0, 5.0,
          math.log(1.0956), math.log(2.1277e-3), math.log(0.75), math.log(0.5), math.log(0.5))


def training_problems(count=32, n_stations=3340, n_days=30, m=30, first_seed=1):
    """Station-network problems spread over the year; odd seeds draw perturbed
    hyperparameters, even seeds keep the workload's."""
    import synth
    return [Dataset(synth.config_station_days(seed=s, n_stations=n_stations, n_days=n_days, m=m,
                                              perturb=(s % 2 == 1), day0=(37 * s) % (365 - n_days)),
                    m)
            for s in range(first_seed, first_seed + count)]


def init_params(seed=0, device="cuda"):
    """He-style initialisation of the packed parameters (FP32)."""
    import torch
    g = torch.Generator().manual_seed(seed)
    parts = []
    for fan_in, fan_out in ((8, 64), (64, 64), (64, 64), (64, 16)):
        parts.append(torch.randn(fan_in * fan_out, generator=g) * math.sqrt(2.0 / fan_in))
        parts.append(torch.zeros(fan_out))
    p = torch.cat(parts).to(torch.float32)
    assert p.numel() == L.MLP_PARAMS
    return p.to(device)


class Dataset:
    """One labelled problem resident on the GPU."""

    def __init__(self, d, m, device="cuda"):
        import numpy as np
        import torch
        self.n, self.m, self.kern = d["n"], m, d["kern"]
        to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        self.X = (to(d["sx"]), to(d["sy"]), to(d["t"]))
        self.feat = L.vif_mlp_features(*self.X, self.kern, CENTRE)
        self.nbr_ext = L.vif_neighbors(*self.X, self.kern, 2 * m)
        # queries: points with a full extended list (no -1 padding)
        t = d["t"]
        first = int(np.searchsorted(t, t[0] + 2, side="left"))
        self.q_lo = max(first, 2 * m + 1)
        self.rand_window = max(64, int(self.n / max(1.0, t[-1] - t[0] + 1)) * 2)


def train(datasets, steps=2000, batch=256, npos=30, nhard=30, nrand=16, tau=0.5, lr=2e-3,
          seed=0, log_every=200, log=print):
    """Trains the network on the datasets' exact neighbor lists; returns the parameters and
    the loss history."""
    import torch
    dev = datasets[0].feat.device
    params = init_params(seed, dev)
    m1 = torch.zeros_like(params)
    v1 = torch.zeros_like(params)
    gen = torch.Generator(device=dev).manual_seed(seed)
    nneg = nhard + nrand
    hist = []
    t0 = time.perf_counter()
    for step in range(1, steps + 1):
        ds = datasets[(step - 1) % len(datasets)]
        q = torch.randint(ds.q_lo, ds.n, (batch,), generator=gen, device=dev, dtype=torch.int32)
        rnd = torch.randint(0, 2**31 - 1, (batch, nrand), generator=gen, device=dev,
                            dtype=torch.int32)
        Xb = L.vif_mlp_batch(ds.feat, q, ds.nbr_ext, npos, nhard, nrand, rnd, ds.rand_window)
        E, H = L.vif_mlp_forward(params, Xb, want_hidden=True)
        loss, dE = L.vif_mlp_pair_loss(E, npos, nneg, tau)
        grad = L.vif_mlp_backward(params, Xb, H, dE)
        cur_lr = lr * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / steps))
        L.vif_mlp_adam(params, grad, m1, v1, step, cur_lr)
        if step % log_every == 0 or step == steps:
            lv = float(loss.mean())
            hist.append((step, lv))
            log(f"[train] step {step}/{steps} loss {lv:.4f} ({time.perf_counter() - t0:.1f}s)")
    return params, hist


def embed(params, X, kern):
    """Embeddings [n, 16] of the points under kernel `kern`."""
    feat = L.vif_mlp_features(*X, kern, CENTRE)
    E, _ = L.vif_mlp_forward(params, feat)
    return E


def recall(prop, exact):
    """Share of the exact neighbor entries (excluding -1) present in the proposal rows."""
    import torch
    m = exact.shape[1]
    valid = exact >= 0
    hit = torch.zeros_like(exact, dtype=torch.bool)
    for r in range(m):
        hit |= (prop[:, r:r + 1] == exact) & valid
    return float(hit.sum()) / max(1, int(valid.sum()))
