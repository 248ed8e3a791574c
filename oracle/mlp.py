"""Fit-initialisation MLP, FP64 forward/backward and Adam (oracle; test only).

Network (not in the paper; it maps a normalised D(q, .) curve to a start for
the least-squares fit): x (64) -> 3 x [Linear(256), GELU] -> Linear(3).
GELU is the exact form gelu(z) = z Phi(z) = 0.5 z (1 + erf(z / sqrt 2)).
Loss: mean squared error over the batch and the 3 outputs.

Parameter vector layout (flat, float): W1 [256, 64], b1 [256], W2 [256, 256],
b2 [256], W3 [256, 256], b3 [256], W4 [3, 256], b4 [3]; row-major, W[o, i]
multiplies input i into output o.  148,995 numbers.

The GPU keeps BF16 copies of the weights and of the activations that feed the
next layer; ``bf16_round`` reproduces that rounding (round to nearest even)
so that the oracle can be run on the same rounded operands.
"""

import math

import numpy as np
from scipy.special import erf

SIZES = [(256, 64), (256, 256), (256, 256), (3, 256)]


def n_params():
    return sum(o * i + o for o, i in SIZES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, off = [], 0
    for o, i in SIZES:
        W = theta[off:off + o * i].reshape(o, i)
        off += o * i
        b = theta[off:off + o]
        off += o
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def bf16_round(x):
    """Round float64/float32 values to the nearest bfloat16 (ties to even), as float64."""
    a = np.asarray(x, dtype=np.float32).copy()
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta, X, round_hidden=False):
    """Returns (Y [B, 3], cache).  round_hidden: round GELU outputs to BF16."""
    layers = unpack(theta)
    h = np.asarray(X, dtype=np.float64)
    cache = {"h": [h], "z": []}
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        cache["z"].append(z)
        if li < len(layers) - 1:
            h = gelu(z)
            if round_hidden:
                h = bf16_round(h)
            cache["h"].append(h)
        else:
            h = z
    return h, cache


def loss(theta, X, T):
    Y, _ = forward(theta, X)
    return float(np.mean((Y - T) ** 2))


def backward(theta, X, T, round_hidden=False):
    """Gradient of the mean squared error w.r.t. theta (flat), and the loss."""
    layers = unpack(theta)
    Y, cache = forward(theta, X, round_hidden)
    B = X.shape[0]
    dz = 2.0 * (Y - T) / (B * Y.shape[1])
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        h_in = cache["h"][li]
        grads[li] = (dz.T @ h_in, dz.sum(axis=0))
        if li > 0:
            dh = dz @ W
            dz = dh * gelu_grad(cache["z"][li - 1])
    return pack(grads), float(np.mean((Y - T) ** 2))


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    r = np.random.default_rng(seed)
    layers = []
    for o, i in SIZES:
        s = 1.0 / math.sqrt(i)
        layers.append((r.uniform(-s, s, (o, i)), r.uniform(-s, s, o)))
    return pack(layers)
