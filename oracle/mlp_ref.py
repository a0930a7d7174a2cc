"""Plain FP64 CPU oracle of the surface-flux surrogate network.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The network and its loss
are not part of the paper; they are defined by the surrogate ABI: layers
n_in -> width (GELU, erf form) x depth -> n_out = 2F outputs (means mu_f,
then log variances s_f, f < F), targets y[B, F], loss
L = mean_b sum_f [ r^2 + sg(r^2) exp(-s_f) + s_f ],  r = y_f - mu_f.
The log-variance outputs learn through the output layer only: their part of
the gradient is not propagated into the hidden layers, which the mean
outputs alone train.

With ``bf=True`` the values the GPU stores in BF16 are rounded to BF16
(round to nearest even) at the same points -- the input, the weights, each
hidden activation (GELU of the unrounded pre-activation), the pre-activation
kept for the backward pass, the output-layer gradient and each
backpropagated gradient -- while every sum is exact FP64.  Parameters use the
logical order of the ABI: per layer W[n_out][n_in] row-major, then b.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def bf16(x):
    """Round FP64/FP32 values to BF16 (nearest even), returned as FP64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def shapes(n_in, width, depth, n_out=4):
    dims = [n_in] + [width] * depth + [n_out]
    return [(dims[i + 1], dims[i]) for i in range(depth + 1)]


def unpack(theta, n_in, width, depth, n_out=4):
    out, o = [], 0
    for n, k in shapes(n_in, width, depth, n_out):
        W = theta[o:o + n * k].reshape(n, k)
        o += n * k
        b = theta[o:o + n]
        o += n
        out.append((W, b))
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_d(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def forward(theta, x, dims, bf=False):
    """Returns (output [B, n_out], cache)."""
    r = bf16 if bf else (lambda v: np.asarray(v, np.float64))
    layers = unpack(np.asarray(theta, np.float64), *dims)
    a = r(x)
    acts, pres = [a], []
    for l, (W, b) in enumerate(layers):
        Wq = r(W)
        z = a @ Wq.T + b
        if l < len(layers) - 1:
            pres.append(r(z))
            g = gelu(z)
            a = r(g)
            acts.append(a)
        else:
            out = z
    return out, (acts, pres, layers)


def loss_and_grad(theta, x, y, dims, bf=False):
    """Loss and analytic gradient (logical order)."""
    r = bf16 if bf else (lambda v: np.asarray(v, np.float64))
    out, (acts, pres, layers) = forward(theta, x, dims, bf)
    B, F = x.shape[0], out.shape[1] // 2
    mu, s = out[:, :F], out[:, F:2 * F]
    res = y - mu
    e = np.exp(-s)
    loss = np.sum(res * res + res * res * e + s) / B
    dz = np.zeros_like(out)
    dz[:, :F] = -2.0 * res / B
    dz[:, F:2 * F] = (1.0 - res * res * e) / B
    dz = r(dz)
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        gW = dz.T @ acts[l]
        gb = dz.sum(axis=0)
        grads.append((gW, gb))
        if l == len(layers) - 1:
            dz = dz.copy()
            dz[:, F:2 * F] = 0.0          # log variances: output layer only
        if l > 0:
            da = dz @ r(W)
            dz = r(da * gelu_d(pres[l - 1]))
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def init(n_in, width, depth, seed, n_out=4):
    rng = np.random.default_rng(seed)
    parts = []
    for l, (n, k) in enumerate(shapes(n_in, width, depth, n_out)):
        std = math.sqrt((2.0 if l < depth else 1.0) / k)
        parts += [rng.normal(0.0, std, n * k), np.zeros(n)]
    return np.concatenate(parts)
