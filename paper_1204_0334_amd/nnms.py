"""Learned (neural normalized / offset) min-sum decoding: the autograd
wrapper of the library's training entry points, Adam training on frames that
the GPU generates, and the FER comparison with plain sum-product.

The decoder keeps the flooding schedule of Algorithm 1 and replaces the
horizontal step (Eq. 3) by alpha = w[t, e] * sign * max(min|beta| - b[t, e], 0)
with one (w, b) pair per iteration t and edge class e, the edge's circulant
block (Nachmani et al. 2016, 2018; Lugosch & Gross 2017).  Forward, backward and decoding run in the HIP
library (`ldpc_nms_train_forward`, `ldpc_nms_train_backward`,
`ldpc_nms_decode`); this module holds the optimiser loop.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import fer, ldpc


class IterationLosses(torch.autograd.Function):
    """weights [T, blocks, 2] -> per-iteration BCE losses [T] of the learned
    min-sum decoder on llr [gamma, n] (all-zero codeword).  The backward pass
    is the library's hand-written one, recomputing every `ckpt_every`
    iterations from the checkpoints the forward pass left in `ws`."""

    @staticmethod
    def forward(ctx, weights, g, llr, ckpt_every, ws):
        w = weights.detach().contiguous()
        loss = ldpc.nms_train_forward(g, llr, w, ckpt_every, ws)
        ctx.g, ctx.gamma, ctx.ckpt_every, ctx.ws = g, llr.shape[0], ckpt_every, ws
        ctx.save_for_backward(w)
        return loss

    @staticmethod
    def backward(ctx, dloss):
        (w,) = ctx.saved_tensors
        grad = ldpc.nms_train_backward(ctx.g, ctx.gamma, w, ctx.ckpt_every, dloss.contiguous().float(), ctx.ws)
        return grad, None, None, None, None


def iteration_losses(weights, g, llr, ckpt_every: int, ws):
    return IterationLosses.apply(weights, g, llr, ckpt_every, ws)


def initial_weights(T: int, classes: int, scale: float = 0.8, offset: float = 0.0, device=None):
    """[T, classes, 2]: every class starts at (scale, offset)."""
    w = torch.empty((T, classes, 2), dtype=torch.float32, device=device or "cuda")
    w[..., 0] = scale
    w[..., 1] = offset
    return w


def choose_ckpt_every(g: ldpc.Graph, batch: int, T: int, device=None) -> int:
    """T (every iteration's messages kept: no recomputation in the backward
    pass) when that workspace takes at most half the free device memory,
    else 4 (the last segment kept, earlier ones recomputed from checkpoints).
    The gradient is the same either way."""
    free, _ = torch.cuda.mem_get_info(torch.device(device or "cuda:0"))
    return T if ldpc.nms_train_workspace_size(g, batch, T, T) <= free // 2 else min(4, T)


def train(g: ldpc.Graph, T: int = 12, ckpt_every: int | None = None, frames: int = 1 << 20, batch: int = 1024,
          ebn0_range=(1.0, 2.5), chunk: int = 64, lr: float = 0.01, seed: int = 7, init=None,
          loss_weights=None, log_every: int = 0, device=None, checkpoint_path: str | None = None,
          checkpoint_every: int = 64):
    """Adam on sum_t loss_weights[t] * (BCE of iteration t) (default: the
    mean over iterations), batches of `batch` fresh frames, each run of
    `chunk` frames at an Eb/N0 drawn uniformly from `ebn0_range`.  Scales and
    offsets are kept >= 0 after every step.  Returns (weights [T, blocks, 2],
    history of (frames, loss)).  `ckpt_every` None: choose_ckpt_every.

    With `checkpoint_path`, the weights, the Adam state, the step count, the
    Eb/N0 generator's state and the history are saved there every
    `checkpoint_every` steps and at the end; an existing checkpoint is
    resumed (the frames are counter-based, so a resumed run sees the same
    frames as an uninterrupted one)."""
    dev = torch.device(device or "cuda:0")
    info = g.info
    n, classes, rate = info["n"], info["blocks"], info["design_rate"]
    if batch % chunk:
        raise ValueError("batch must be a multiple of chunk")
    W = (init.clone() if init is not None else initial_weights(T, classes, device=dev)).requires_grad_(True)
    opt = torch.optim.Adam([W], lr=lr)
    if ckpt_every is None:
        ckpt_every = choose_ckpt_every(g, batch, T, dev)
    ws = ldpc.nms_train_workspace(g, batch, T, ckpt_every, dev)
    llr = torch.empty((batch, n), dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed)
    coef = torch.full((T,), 1.0 / T, device=dev) if loss_weights is None else \
        torch.as_tensor(loss_weights, dtype=torch.float32, device=dev)
    history = []
    steps = max(frames // batch, 1)
    first = 0
    if checkpoint_path and os.path.exists(checkpoint_path):
        ck = torch.load(checkpoint_path, map_location=dev, weights_only=True)
        with torch.no_grad():
            W.copy_(ck["weights"])
        opt.load_state_dict(ck["adam"])
        rng.bit_generator.state = json.loads(ck["rng"])
        history = [tuple(h) for h in ck["history"]]
        first = int(ck["step"])

    def save(step_done):
        tmp = checkpoint_path + ".tmp"
        torch.save({"weights": W.detach().clone(), "adam": opt.state_dict(), "step": step_done,
                    "rng": json.dumps(rng.bit_generator.state), "history": [list(h) for h in history]}, tmp)
        os.replace(tmp, checkpoint_path)

    for step in range(first, steps):
        frame0 = step * batch
        for c in range(batch // chunk):
            sigma2 = fer.ebn0_to_sigma2(float(rng.uniform(*ebn0_range)), rate)
            ldpc.awgn_llr(n, chunk, sigma2, seed, frame0 + c * chunk, out=llr[c * chunk:(c + 1) * chunk])
        per = iteration_losses(W, g, llr, ckpt_every, ws)
        loss = (coef * per).sum()
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        with torch.no_grad():
            W.clamp_(min=0.0)
        if log_every and (step % log_every == 0 or step == steps - 1):
            history.append((frame0 + batch, float(loss.detach())))
        if checkpoint_path and ((step + 1) % checkpoint_every == 0 or step == steps - 1):
            save(step + 1)
    return W.detach(), history


def compare_fer(g: ldpc.Graph, weights, ebn0_points, *, sp_iters: int = 30, frames: int = 1 << 20,
                gamma: int = 1024, seed: int = 2024, min_frame_errors: int | None = None):
    """FER of the learned decoder (T = weights.shape[0] iterations) and of
    plain sum-product (`sp_iters` iterations) on the same fresh frames at
    each Eb/N0.  Both run to `frames` frames (or `min_frame_errors`)."""
    out = []
    stop = min_frame_errors if min_frame_errors is not None else 1 << 62
    for k, e in enumerate(ebn0_points):
        s = seed + 1000 * k
        learned = fer.simulate(g, e, decoder="nms", weights=weights, gamma=gamma, seed=s,
                               min_frame_errors=stop, max_frames=frames)
        plain = fer.simulate(g, e, decoder="block", gamma=gamma, iters=sp_iters, seed=s,
                             min_frame_errors=stop, max_frames=frames)
        out.append(dict(ebn0_db=e, learned=learned, plain=plain))
    return out
