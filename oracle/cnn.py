"""FP64 reference of the learned Newton initial-guess network.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  This part is not in the
paper; it is the reference the device kernels' forward and backward passes
are checked against.

Network: four 3x3x3 convolutions with zero ("same") padding on the node grid,
channels 4 -> 16 -> 16 -> 16 -> 2, GELU (exact, with erf) after the first
three.  Correlation convention:
    out[o, z, y, x] = b[o] + sum_{c, dz, dy, dx} W[o, c, dz, dy, dx] in[c, z+dz-1, y+dy-1, x+dx-1].
Parameters are one flat vector, layer by layer: W (Cout, Cin, 3, 3, 3) then b.
Loss: mean squared error over every output entry.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

CHANNELS = (4, 16, 16, 16, 2)


def param_shapes():
    shapes = []
    for cin, cout in zip(CHANNELS[:-1], CHANNELS[1:]):
        shapes.append((cout, cin, 3, 3, 3))
        shapes.append((cout,))
    return shapes


def n_params():
    return sum(int(np.prod(s)) for s in param_shapes())


def unflatten(theta):
    out, k = [], 0
    for s in param_shapes():
        n = int(np.prod(s))
        out.append(np.asarray(theta[k:k + n], dtype=np.float64).reshape(s))
        k += n
    return out


def flatten(tensors):
    return np.concatenate([t.ravel() for t in tensors])


def conv3d(x, W, b):
    """Zero-padded 3x3x3 correlation, x: (Cin, Z, Y, X)."""
    cin, Z, Y, X = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))
    out = np.broadcast_to(b[:, None, None, None], (W.shape[0], Z, Y, X)).copy()
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                out += np.einsum("oc,czyx->ozyx", W[:, :, dz, dy, dx],
                                 xp[:, dz:dz + Z, dy:dy + Y, dx:dx + X])
    return out


def conv3d_grad(x, W, gout):
    """Gradients of conv3d w.r.t. its input, weights and bias."""
    cin, Z, Y, X = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))
    gxp = np.zeros_like(xp)
    gW = np.zeros_like(W)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                sl = (slice(None), slice(dz, dz + Z), slice(dy, dy + Y), slice(dx, dx + X))
                gW[:, :, dz, dy, dx] = np.einsum("ozyx,czyx->oc", gout, xp[sl])
                gxp[sl] += np.einsum("oc,ozyx->czyx", W[:, :, dz, dy, dx], gout)
    gb = gout.sum(axis=(1, 2, 3))
    return gxp[:, 1:-1, 1:-1, 1:-1], gW, gb


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(theta, x):
    """Returns the output and the pre-activations of every layer."""
    P = unflatten(theta)
    pre, h = [], x
    for L in range(4):
        z = conv3d(h, P[2 * L], P[2 * L + 1])
        pre.append((h, z))
        h = gelu(z) if L < 3 else z
    return h, pre


def loss_and_grad(theta, x, target):
    """Mean squared error and its gradient w.r.t. the flat parameters."""
    y, pre = forward(theta, x)
    diff = y - target
    loss = float(np.mean(diff * diff))
    g = 2.0 * diff / diff.size
    P = unflatten(theta)
    grads = [None] * len(P)
    for L in range(3, -1, -1):
        h, z = pre[L]
        if L < 3:
            g = g * gelu_grad(z)
        gh, gW, gb = conv3d_grad(h, P[2 * L], g)
        grads[2 * L], grads[2 * L + 1] = gW, gb
        g = gh
    return loss, flatten(grads)


def adam_step(theta, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments) of the flat parameters."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
