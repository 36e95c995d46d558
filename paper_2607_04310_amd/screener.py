"""Training driver of the edge-screener MLP.

Labels are the exact per-edge pool distances computed on the GPU by
psdf_screen_labels (the quantity the screener ranks by); the network is
trained by the library's own forward / backward / Adam kernels
(psdf_mlp_train_step).  PyTorch only holds the device buffers.
"""
from __future__ import annotations

import json
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


def save_checkpoint(path, theta, m=None, v=None, step=0, seed=0, hist=None):
    """Write the screener's state to a safetensors file: the FP32 master
    weights, their BF16 copy (the operands the kernels use), the Adam moments,
    and (metadata) the step, the training seed and the loss history."""
    from safetensors.torch import save_file
    th = theta.detach().to("cpu", torch.float32).contiguous()
    tensors = {"theta": th, "theta_bf16": th.to(torch.bfloat16).contiguous()}
    if m is not None:
        tensors["adam_m"] = m.detach().to("cpu", torch.float32).contiguous()
    if v is not None:
        tensors["adam_v"] = v.detach().to("cpu", torch.float32).contiguous()
    meta = {"step": str(int(step)), "seed": str(int(seed)),
            "hist": json.dumps([float(x) for x in (hist or [])]),
            "layout": "W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3"}
    save_file(tensors, str(path), metadata=meta)


def load_checkpoint(path, device="cpu"):
    """The state written by save_checkpoint: dict with theta (FP32), theta_bf16,
    adam_m / adam_v (or None), step, seed, hist."""
    from safetensors import safe_open
    out = {}
    with safe_open(str(path), framework="pt", device="cpu") as f:
        meta = f.metadata() or {}
        for k in ("theta", "theta_bf16", "adam_m", "adam_v"):
            out[k] = f.get_tensor(k).to(device) if k in f.keys() else None
    if out["theta"] is None or out["theta"].numel() != inputs.MLP_PARAMS:
        raise ValueError(f"{path}: not a screener checkpoint ({inputs.MLP_PARAMS} parameters)")
    out["step"] = int(meta.get("step", 0))
    out["seed"] = int(meta.get("seed", 0))
    out["hist"] = json.loads(meta.get("hist", "[]"))
    return out


def train(X, T, epochs=20, batch=4096, lr=2e-3, seed=0, log=None, resume=None, state=None):
    """Train from mlp_init_params(seed) (or from the state `resume` returned by
    load_checkpoint: weights, Adam moments and step) with Adam and a cosine
    learning-rate schedule over this call's steps; returns (theta on the
    device, per-epoch mean losses).  A dict passed as `state` receives the
    Adam moments and the step count (for save_checkpoint)."""
    dev = X.device
    if resume is not None:
        theta = resume["theta"].to(dev, torch.float32).clone()
        m = resume["adam_m"].to(dev).clone() if resume["adam_m"] is not None else torch.zeros_like(theta)
        v = resume["adam_v"].to(dev).clone() if resume["adam_v"] is not None else torch.zeros_like(theta)
        step0 = int(resume["step"])
    else:
        theta = torch.tensor(inputs.mlp_init_params(seed), device=dev)
        m = torch.zeros_like(theta)
        v = torch.zeros_like(theta)
        step0 = 0
    n = int(X.shape[0])
    gen = torch.Generator(device="cpu").manual_seed(seed)
    ws = api._mlp_ws(batch, dev)
    loss = torch.zeros(1, device=dev)
    step = step0
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
            cur = lr * 0.5 * (1.0 + np.cos(np.pi * (step - step0 - 1) / max(1, steps_total)))
            api.mlp_train_step(theta, m, v, step, cur, xb, tb, loss=loss, ws=ws)
            acc += loss
        hist.append(float(acc.item()) / max(1, nb))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f} ({time.time() - t0:.1f} s)")
    if state is not None:
        state.update(m=m, v=v, step=step)
    return theta, hist
