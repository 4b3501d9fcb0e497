"""FP64 reference of the learned warm start's network (test infrastructure).

The warm start maps Hamiltonian parameters to a converged dual/primal state of
Algorithm 6 (Section 4's method has no learned part; this is the learned
initialisation for parameter sweeps).  The network is a plain multilayer
perceptron:

    a_0 = x;  z_l = a_{l-1} W_l^T + b_l;  a_l = silu(z_l) (hidden layers);  y = z_last
    silu(z) = z * sigmoid(z)

trained on normalised targets t_hat = (t - mean) / std with the mean squared error
L = mean over (batch, outputs) of (y - t_hat)^2, by Adam (Kingma & Ba, 2015):
    m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
    theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Weights are held in FP32 (master copy) and used in the forward and backward
passes after rounding to bfloat16 (round to nearest, ties to even); biases stay
FP32.  Everything here is FP64 arithmetic on those values.

Pins (tests/test_oracle_mlp.py): central finite differences of the loss for every
parameter of a small network; Adam's step under a constant gradient equals
lr g / (|g| + eps) at every step (bias correction); silu closed-form values;
bfloat16 rounding of values whose nearest neighbours and ties are known.
"""
from __future__ import annotations

import numpy as np

ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8
STD_FLOOR = 1e-6


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def flatten(params) -> np.ndarray:
    """Parameters in the library's layout: W_0, b_0, W_1, b_1, ... (row-major W)."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def unflatten(flat, dims):
    out, o = [], 0
    for l in range(len(dims) - 1):
        nW = dims[l + 1] * dims[l]
        W = np.asarray(flat[o:o + nW]).reshape(dims[l + 1], dims[l])
        o += nW
        b = np.asarray(flat[o:o + dims[l + 1]])
        o += dims[l + 1]
        out.append((W, b))
    return out


def used_weights(params, rounding=True):
    """The values the passes use: bfloat16-rounded W, FP32 b (as float64)."""
    return [((bf16_round(W) if rounding else np.asarray(W, np.float64)), np.asarray(b, np.float64))
            for W, b in params]


def forward(params, x, rounding=True):
    """Returns (y, cache); y are the normalised outputs."""
    P = used_weights(params, rounding)
    a = np.asarray(x, np.float64)
    zs, acts = [], [a]
    for l, (W, b) in enumerate(P):
        z = a @ W.T + b
        zs.append(z)
        a = silu(z) if l < len(P) - 1 else z
        acts.append(a)
    return a, (P, zs, acts)


def normalisation(targets, rel_floor=0.0):
    """Per-output mean and standard deviation of a training set, the deviation floored at
    max(STD_FLOOR, rel_floor * largest deviation): outputs that barely vary are not blown up
    into noise the network would have to fit."""
    t = np.asarray(targets, np.float64)
    mean = t.mean(axis=0)
    std = np.sqrt(((t - mean) ** 2).mean(axis=0))
    return mean, np.maximum(std, max(STD_FLOOR, rel_floor * std.max()))


def loss_and_grads(params, x, t, mean, std, rounding=True):
    """MSE on normalised targets and its gradient w.r.t. the used parameters."""
    y, (P, zs, acts) = forward(params, x, rounding)
    th = (np.asarray(t, np.float64) - mean) / std
    B, O = y.shape
    r = y - th
    loss = float(np.sum(r * r) / (B * O))
    dz = 2.0 * r / (B * O)
    grads = [None] * len(P)
    for l in range(len(P) - 1, -1, -1):
        W, _ = P[l]
        grads[l] = (dz.T @ acts[l], dz.sum(axis=0))
        if l > 0:
            dz = (dz @ W) * silu_grad(zs[l - 1])
    return loss, grads


def predict(params, x, mean, std):
    """Denormalised network outputs."""
    y, _ = forward(params, x)
    return y * std + mean


class Adam:
    """Adam over a flat FP32 parameter vector, moments in FP64."""

    def __init__(self, n):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0

    def step(self, theta, g, lr):
        self.t += 1
        g = np.asarray(g, np.float64)
        self.m = ADAM_B1 * self.m + (1 - ADAM_B1) * g
        self.v = ADAM_B2 * self.v + (1 - ADAM_B2) * g * g
        mh = self.m / (1 - ADAM_B1 ** self.t)
        vh = self.v / (1 - ADAM_B2 ** self.t)
        return np.asarray(theta, np.float64) - lr * mh / (np.sqrt(vh) + ADAM_EPS)


def flat_grads(grads) -> np.ndarray:
    return np.concatenate([np.concatenate([gW.ravel(), gb.ravel()]) for gW, gb in grads])
