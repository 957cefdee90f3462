"""FP64 reference of the residual surrogate network (forward, backward, Adam).

TEST INFRASTRUCTURE ONLY: the GPU library's BF16-MFMA training and inference
kernels are checked against this plain numpy implementation.  It shares no
code with the HIP library.

Network: x (n, D_IN) -> [Linear -> GELU] x 4 (width 256) -> Linear -> y (n,)
GELU(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3)))   (tanh form)
Loss: mean squared error, L = mean((y - t)^2).
Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
      w -= lr * (m / (1 - b1^s)) / (sqrt(v / (1 - b2^s)) + eps).
Weights: list of (W_l, b_l) with W_l of shape (in, out).
"""
from __future__ import annotations

import numpy as np

C_GELU = np.sqrt(2.0 / np.pi)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(C_GELU * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    u = C_GELU * (z + 0.044715 * z ** 3)
    th = np.tanh(u)
    du = C_GELU * (1.0 + 3.0 * 0.044715 * z ** 2)
    return 0.5 * (1.0 + th) + 0.5 * z * (1.0 - th ** 2) * du


def init(rng, d_in, width=256, depth=4):
    """He-style uniform init (the GPU library receives these weights)."""
    dims = [d_in] + [width] * depth + [1]
    params = []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = np.sqrt(6.0 / a) if b != 1 else np.sqrt(3.0 / a)
        params.append((rng.uniform(-lim, lim, (a, b)), np.zeros(b)))
    return params


def forward(params, x):
    """Returns the output (n,) and the cache of pre-activations/activations."""
    acts = [np.asarray(x, np.float64)]
    pres = []
    h = acts[0]
    for i, (W, b) in enumerate(params):
        z = h @ W + b
        if i + 1 < len(params):
            pres.append(z)
            h = gelu(z)
            acts.append(h)
        else:
            h = z
    return h[:, 0], (acts, pres)


def loss_and_grads(params, x, t):
    y, (acts, pres) = forward(params, x)
    n = x.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = (2.0 / n) * r[:, None]
    grads = [None] * len(params)
    d = dy
    for i in range(len(params) - 1, -1, -1):
        W, b = params[i]
        grads[i] = (acts[i].T @ d, d.sum(axis=0))
        if i > 0:
            d = (d @ W.T) * gelu_grad(pres[i - 1])
    return loss, grads


def adam_step(params, grads, state, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update; state is a list of (mW, vW, mb, vb)."""
    out = []
    for (W, b), (gW, gb), (mW, vW, mb, vb) in zip(params, grads, state):
        mW[:] = b1 * mW + (1 - b1) * gW
        vW[:] = b2 * vW + (1 - b2) * gW * gW
        mb[:] = b1 * mb + (1 - b1) * gb
        vb[:] = b2 * vb + (1 - b2) * gb * gb
        c1, c2 = 1 - b1 ** step, 1 - b2 ** step
        W = W - lr * (mW / c1) / (np.sqrt(vW / c2) + eps)
        b = b - lr * (mb / c1) / (np.sqrt(vb / c2) + eps)
        out.append((W, b))
    return out


def adam_state(params):
    return [(np.zeros_like(W), np.zeros_like(W), np.zeros_like(b), np.zeros_like(b))
            for W, b in params]


def n_params(params):
    return sum(W.size + b.size for W, b in params)
