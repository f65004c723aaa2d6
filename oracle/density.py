"""Spectral-density MLP in float64 (TEST INFRASTRUCTURE ONLY).

Forward and backward of the three-layer network the library trains on BF16
matrix cores (the learned spectral predictor of Sec. 4.1, trained with a
mean squared error):

    H1 = GELU(X W1 + b1), H2 = GELU(H1 W2 + b2), Y = H2 W3 + b3,
    loss = mean((Y - T)^2),

with the exact GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2 and its
derivative Phi(z) + z phi(z).  Written with plain matrix products so each
gradient can be checked against finite differences.
"""
from __future__ import annotations

import math

import numpy as np

_erf = np.vectorize(math.erf)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    Z1 = X @ W1 + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2 + b2
    H2 = gelu(Z2)
    Y = H2 @ W3 + b3
    return Y, (X, Z1, H1, Z2, H2)


def loss_and_grads(params, X, T):
    W1, b1, W2, b2, W3, b3 = params
    Y, (X, Z1, H1, Z2, H2) = forward(params, X)
    D = Y - T
    loss = float(np.mean(D * D))
    dY = 2.0 * D / D.size
    gW3 = H2.T @ dY
    gb3 = dY.sum(axis=0)
    dZ2 = (dY @ W3.T) * gelu_grad(Z2)
    gW2 = H1.T @ dZ2
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2.T) * gelu_grad(Z1)
    gW1 = X.T @ dZ1
    gb1 = dZ1.sum(axis=0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]
