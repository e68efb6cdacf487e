"""Reference forward pass, loss gradient and Adam step of the initial-guess network (a project
addition: the paper's initial data are the analytic guesses of Sec. 3 and the coarse-grid
solutions of Algorithm 2; this network is a learned third source of initial data).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network, all matrices [out][in]:  h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  y = W3 h2 + b3;
loss = mean over batch x d_out of (y - target)^2.

Everything is computed in FP64. With `bf16=True` the values that the library feeds to its BF16
matrix cores are rounded to BF16 (round to nearest, ties to even) at the same places:
the weights W1, W2, W3; the activations h1 and h2 as inputs of the next layer; the output
gradient dL/dy and the layer-2 pre-activation gradient as inputs of the weight-gradient and
back-propagation products. Biases, x, y, tanh values (used in the derivative 1 - t^2), the
bias gradients and the layer-1 gradient are not rounded. With `bf16=False` the functions are
the exact FP64 network and its exact gradient.

Adam follows Kingma and Ba, "Adam: a method for stochastic optimization", Algorithm 1.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x):
    """Nearest BF16 value (8 significant bits, FP32 exponent range), ties to even, as float64.

    Written with frexp: x = m 2^e, m in [0.5, 1); the BF16 spacing at x is 2^(e-8), floored
    at the subnormal spacing 2^-133. np.rint rounds halves to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    e = np.maximum(e, -125)
    step = np.ldexp(1.0, e - 8)
    return np.rint(x / step) * step


def unpack(params, d_in, d_h, d_out):
    p = np.asarray(params, dtype=np.float64)
    k = 0
    out = {}
    for name, shape in (("W1", (d_h, d_in)), ("b1", (d_h,)), ("W2", (d_h, d_h)), ("b2", (d_h,)),
                        ("W3", (d_out, d_h)), ("b3", (d_out,))):
        size = int(np.prod(shape))
        out[name] = p[k:k + size].reshape(shape)
        k += size
    assert k == p.size
    return out


def pack(d):
    return np.concatenate([d[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def forward(params, x, dims, bf16=True):
    """Returns y and the intermediate values (dict) of the forward pass."""
    r = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    P = unpack(params, *dims)
    x = np.asarray(x, dtype=np.float64)
    W1, W2, W3 = r(P["W1"]), r(P["W2"]), r(P["W3"])
    t1 = np.tanh(x @ W1.T + P["b1"])
    h1 = r(t1)
    t2 = np.tanh(h1 @ W2.T + P["b2"])
    h2 = r(t2)
    y = h2 @ W3.T + P["b3"]
    return y, dict(t1=t1, h1=h1, t2=t2, h2=h2, W1=W1, W2=W2, W3=W3)


def loss_grad(params, x, target, dims, bf16=True):
    """Loss (mean squared error) and its gradient, packed like params."""
    r = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    y, c = forward(params, x, dims, bf16)
    B, D = y.shape
    d = y - np.asarray(target, dtype=np.float64)
    loss = float(np.mean(d * d))
    dY = (2.0 / (B * D)) * d
    dYr = r(dY)
    g = {}
    g["W3"] = dYr.T @ c["h2"]
    g["b3"] = dY.sum(axis=0)
    dA2 = (dYr @ c["W3"]) * (1.0 - c["t2"] ** 2)
    g["b2"] = dA2.sum(axis=0)
    dA2r = r(dA2)
    g["W2"] = dA2r.T @ c["h1"]
    dA1 = (dA2r @ c["W2"]) * (1.0 - c["t1"] ** 2)
    g["b1"] = dA1.sum(axis=0)
    g["W1"] = dA1.T @ x
    return loss, pack(g), y


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step; returns new (params, m, v)."""
    g = np.asarray(grads, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    p = np.asarray(params, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v
