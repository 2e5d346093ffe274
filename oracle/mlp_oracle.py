"""FP64 CPU reference of the warm-start network (test infrastructure).

TEST INFRASTRUCTURE: only the tests may import this module.  It restates the
network the library trains -- Fourier features of the frequency, two tanh
layers and a linear output layer, mean squared error -- with a hand-written
backward pass, in float64.  With round_bf16=True every matrix-product operand
is first rounded to bfloat16 (round to nearest even), which is what the GPU
kernels do before their FP32-accumulating matrix-core products, so the two
can be compared tightly; the unrounded form is pinned by finite differences.
"""
from __future__ import annotations

import numpy as np

__all__ = ["features", "unpack", "bf16", "forward", "loss_grad"]


def features(omega, n_freq, scale):
    """phi[i, 2k] = sin((k+1) pi w_i / scale), phi[i, 2k+1] = cos(...), k < n_freq."""
    w = np.asarray(omega, float)[:, None]
    k = np.arange(1, n_freq + 1)[None, :]
    a = k * np.pi * w / scale
    phi = np.empty((w.shape[0], 2 * n_freq))
    phi[:, 0::2] = np.sin(a)
    phi[:, 1::2] = np.cos(a)
    return phi


def unpack(p, F, W, O):
    p = np.asarray(p, float)
    o = 0
    W1 = p[o:o + W * F].reshape(W, F); o += W * F
    b1 = p[o:o + W]; o += W
    W2 = p[o:o + W * W].reshape(W, W); o += W * W
    b2 = p[o:o + W]; o += W
    W3 = p[o:o + O * W].reshape(O, W); o += O * W
    b3 = p[o:o + O]; o += O
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def bf16(x):
    """Round float64 values to the nearest bfloat16 (via float32, ties to even)."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, phi, F, W, O, round_bf16=False):
    r = bf16 if round_bf16 else (lambda x: x)
    W1, b1, W2, b2, W3, b3 = unpack(p, F, W, O)
    H1 = np.tanh(r(phi) @ r(W1).T + b1)
    H2 = np.tanh(r(H1) @ r(W2).T + b2)
    out = r(H2) @ r(W3).T + b3
    return H1, H2, out


def loss_grad(p, phi, target, n_cols, F, W, O, round_bf16=False):
    """Mean squared error over the first n_cols outputs and its gradient (flat)."""
    r = bf16 if round_bf16 else (lambda x: x)
    W1, b1, W2, b2, W3, b3 = unpack(p, F, W, O)
    H1, H2, out = forward(p, phi, F, W, O, round_bf16)
    n = phi.shape[0]
    diff = np.zeros_like(out)
    diff[:, :n_cols] = out[:, :n_cols] - np.asarray(target, float)[:, :n_cols]
    loss = float((diff ** 2).sum() / (n * n_cols))
    dout = 2.0 * diff / (n * n_cols)
    dW3 = r(dout).T @ r(H2)
    db3 = dout.sum(0)
    dH2 = r(dout) @ r(W3)
    dZ2 = dH2 * (1.0 - H2 ** 2)
    dW2 = r(dZ2).T @ r(H1)
    db2 = dZ2.sum(0)
    dH1 = r(dZ2) @ r(W2)
    dZ1 = dH1 * (1.0 - H1 ** 2)
    dW1 = r(dZ1).T @ r(phi)
    db1 = dZ1.sum(0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])
    return loss, g
