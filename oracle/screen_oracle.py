"""CPU oracle for the learned pair screen.

TEST INFRASTRUCTURE ONLY (imported by tests, never by the library).  Plain
NumPy FP64 statements of the pair features, the rigorous pair-energy bound
and the 4 -> 64 -> 64 -> 1 SiLU network with its mean-squared-error loss,
analytic gradient and Adam update (Kingma and Ba, 2015).

Parameter vector layout: W1[64][4], b1[64], W2[64][64], b2[64], W3[64], b3.
All functions accept complex inputs (for complex-step derivative checks).
"""
from __future__ import annotations

import numpy as np

H, NIN = 64, 4
NP = H * NIN + H + H * H + H + H + 1


def unpack(p):
    o = 0
    W1 = p[o:o + H * NIN].reshape(H, NIN); o += H * NIN
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(x, p):
    """y = W3 silu(W2 silu(W1 x + b1) + b2) + b3 for each row of x."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    z1 = x @ W1.T + b1
    a1 = silu(z1)
    z2 = a1 @ W2.T + b2
    a2 = silu(z2)
    return a2 @ W3 + b3


def loss(x, t, p):
    r = forward(x, p) - t
    return np.sum(r * r) / len(t)


def loss_grad(x, t, p):
    """Analytic gradient of the mean squared error (backpropagation)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    n = len(t)
    z1 = x @ W1.T + b1
    a1 = silu(z1)
    z2 = a1 @ W2.T + b2
    a2 = silu(z2)
    y = a2 @ W3 + b3
    dy = 2.0 * (y - t) / n
    gW3 = a2.T @ dy
    gb3 = np.sum(dy)
    dz2 = np.outer(dy, W3) * dsilu(z2)
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * dsilu(z1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(axis=0)
    return np.sum((y - t) ** 2) / n, np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def pair_features(B, eps_occ, centroids):
    """[nocc*nocc][4]: (|r_i - r_j| / 10, log ||B_i||_F, log ||B_j||_F, (eps_i + eps_j) / 10)."""
    nocc = B.shape[0]
    nb = np.sqrt(np.einsum("iap,iap->i", B, B))
    out = np.empty((nocc, nocc, 4))
    d = np.sqrt(((centroids[:, None, :] - centroids[None, :, :]) ** 2).sum(-1))
    out[:, :, 0] = d / 10.0
    out[:, :, 1] = np.log(nb)[:, None]
    out[:, :, 2] = np.log(nb)[None, :]
    out[:, :, 3] = (eps_occ[:, None] + eps_occ[None, :]) / 10.0
    return out.reshape(nocc * nocc, 4)


def pair_bound(B, eps_occ, eps_vir):
    """3 (N N^T)_ij^2 / (2 min eps_vir - eps_i - eps_j), N[i][P] = ||B_i[:, P]||_2."""
    N = np.sqrt(np.einsum("iap,iap->ip", B, B))
    S = N @ N.T
    return 3.0 * S * S / (2.0 * eps_vir.min() - eps_occ[:, None] - eps_occ[None, :])
