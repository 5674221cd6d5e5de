"""numpy FP64 oracle of the Fourier-feature MLP neural field -- TEST INFRASTRUCTURE.

The paper's grid fields are precomputed for fast lookup (section 4,
magnetic field techniques); the learned stand-in for the trilinear gather is
this project's extension.  Network (all FP64 here):

    xhat  = frac((x - o) / (N * spacing))                      in [0, 1)^3
    gamma = [cos(2 pi F xhat), sin(2 pi F xhat)]               F: [64, 3] integers
    h1    = relu(W1 gamma + b1);  h_k = relu(W_k h_{k-1} + b_k), k = 2..4
    out   = W5 h4 + b5;           B_nf = B_rms * out
    loss  = mean over points of |out - B_grid / B_rms|^2

With ``bf16=True`` the inputs of every matrix product (weights, embedding,
activations and back-propagated gradients) are rounded to bfloat16
(round-to-nearest-even) at the same points as the GPU kernels do, while the
arithmetic itself stays FP64.

Only tests/ and bench.py's CPU-baseline leg may import this module.
"""
from __future__ import annotations

import numpy as np


def round_bf16(a):
    """Round FP64 values to the nearest bfloat16 (8 significant bits), ties to even."""
    a = np.asarray(a, np.float64)
    m, e = np.frexp(a)                      # a = m * 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(np.ldexp(m, 8)), e - 8)


def relu(z):
    return np.maximum(z, 0.0)


def embed(xhat, F):
    ang = 2.0 * np.pi * (np.asarray(xhat, np.float64) @ np.asarray(F, np.float64).T)
    return np.concatenate([np.cos(ang), np.sin(ang)], axis=1)


def normalized_position(pos, n, spacing, origin=(0.0, 0.0, 0.0)):
    box = np.asarray(n, np.float64) * spacing
    f = (np.asarray(pos, np.float64) - np.asarray(origin)[None, :]) / box
    return f - np.floor(f)


def forward(weights, biases, xhat, F, bf16=False):
    """Returns (out [n,3], cache) for backward."""
    rnd = round_bf16 if bf16 else (lambda v: v)
    a = rnd(embed(xhat, F))
    acts = [a]
    pre = []
    nl = len(weights)
    for k in range(nl):
        W = rnd(np.asarray(weights[k], np.float64))
        z = a @ W.T + np.asarray(biases[k], np.float64)[None, :]
        pre.append(z)
        if k < nl - 1:
            a = rnd(relu(z))
            acts.append(a)
        else:
            a = z
    return a, {"acts": acts, "pre": pre, "bf16": bf16}


def mse_loss(out, target):
    d = out - target
    return float((d * d).sum(axis=1).mean())


def mse_grad(out, target):
    return 2.0 * (out - target) / out.shape[0]


def backward(weights, cache, dout):
    """Gradients of sum(dout * out) with respect to weights and biases."""
    rnd = round_bf16 if cache["bf16"] else (lambda v: v)
    acts, pre = cache["acts"], cache["pre"]
    nl = len(weights)
    gW = [None] * nl
    gb = [None] * nl
    g = np.asarray(dout, np.float64)
    for k in range(nl - 1, -1, -1):
        if k < nl - 1:
            g = g * (pre[k] > 0.0)
        gb[k] = g.sum(axis=0)
        gq = rnd(g)
        gW[k] = gq.T @ acts[k]
        if k > 0:
            W = rnd(np.asarray(weights[k], np.float64))
            g = gq @ W
    return gW, gb


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; in-place lists."""
    for i in range(len(params)):
        m[i] = b1 * m[i] + (1.0 - b1) * grads[i]
        v[i] = b2 * v[i] + (1.0 - b2) * grads[i] * grads[i]
        mh = m[i] / (1.0 - b1 ** t)
        vh = v[i] / (1.0 - b2 ** t)
        params[i] = params[i] - lr * mh / (np.sqrt(vh) + eps)
    return params, m, v


NF_WIDTH = 128
NF_NPARAM = 4 * (NF_WIDTH * NF_WIDTH + NF_WIDTH) + 3 * NF_WIDTH + 3


def flatten(weights, biases):
    """Flat parameter vector in the order W1, b1, ..., W4, b4, W5, b5."""
    parts = []
    for W, b in zip(weights, biases):
        parts.append(np.asarray(W, np.float64).ravel())
        parts.append(np.asarray(b, np.float64).ravel())
    return np.concatenate(parts)


def unflatten(params, width=NF_WIDTH, depth=4, nout=3):
    """Inverse of flatten: lists of W [out][in] and b [out]."""
    p = np.asarray(params, np.float64)
    ws, bs = [], []
    off = 0
    fan = width
    for _ in range(depth):
        ws.append(p[off:off + width * fan].reshape(width, fan))
        off += width * fan
        bs.append(p[off:off + width])
        off += width
    ws.append(p[off:off + nout * width].reshape(nout, width))
    off += nout * width
    bs.append(p[off:off + nout])
    return ws, bs
