"""Training driver of the edge-screener MLP.

Labels are the exact per-edge pool distances computed on the GPU by
psdf_screen_labels (the quantity the screener ranks by); the network is
trained by the library's own forward / backward / Adam kernels
(psdf_mlp_train_step).  PyTorch only holds the device buffers.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import api, inputs


def training_set(instances, near=1024, far=1024, seed=0, device="cuda"):
    """Device (X, T) for the given (held-out) instances."""
    b = api.Batch(instances, graph=False, device=device)
    st, ed = inputs.screener_training_pairs(instances, near, far, seed)
    X, T = b.labels(st, ed)
    torch.cuda.synchronize()
    b.close()
    ok = torch.isfinite(T) & torch.isfinite(X).all(1)
    return X[ok].contiguous(), T[ok].contiguous()


def train(X, T, epochs=20, batch=4096, lr=2e-3, seed=0, log=None):
    """Train from mlp_init_params(seed) with Adam and a cosine learning-rate
    schedule; returns (theta on the device, per-epoch mean losses)."""
    dev = X.device
    theta = torch.tensor(inputs.mlp_init_params(seed), device=dev)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    n = int(X.shape[0])
    gen = torch.Generator(device="cpu").manual_seed(seed)
    ws = api._mlp_ws(batch, dev)
    loss = torch.zeros(1, device=dev)
    step = 0
    steps_total = epochs * (n // batch)
    hist = []
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(dev)
        acc = torch.zeros(1, device=dev)
        nb = n // batch
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            xb, tb = X[idx].contiguous(), T[idx].contiguous()
            step += 1
            cur = lr * 0.5 * (1.0 + np.cos(np.pi * (step - 1) / max(1, steps_total)))
            api.mlp_train_step(theta, m, v, step, cur, xb, tb, loss=loss, ws=ws)
            acc += loss
        hist.append(float(acc.item()) / max(1, nb))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f} ({time.time() - t0:.1f} s)")
    return theta, hist
