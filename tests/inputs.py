"""Seeded synthetic inputs shared by the oracle pins and the GPU tests.

Symmetric positive semi-definite matrices with a prescribed spectrum,
T = Q diag(w) Q^T with Q the orthogonal factor of a Gaussian matrix,
right-hand sides, and random parameter vectors of the linear recurrent test
model.  This module only draws inputs; it computes nothing of the minSR
method."""
import numpy as np


def orthogonal(n, rng):
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))


def spectrum_loguniform(n, cond, rng, zeros=0):
    """n eigenvalues log-uniform in [1/cond, 1] (the largest exactly 1), the
    last `zeros` of them exactly 0."""
    w = np.exp(rng.uniform(np.log(1.0 / cond), 0.0, n))
    w[0] = 1.0
    if zeros:
        w[n - zeros:] = 0.0
    return w


def psd_matrix(w, seed):
    """Q diag(w) Q^T for a seeded orthogonal Q, symmetrised exactly."""
    rng = np.random.default_rng(seed)
    n = len(w)
    Q = orthogonal(n, rng)
    T = (Q * w) @ Q.T
    return 0.5 * (T + T.T), Q


def rhs(n, seed):
    return np.random.default_rng(seed + 7919).standard_normal(n)


def linear_theta(H, seed, scale=0.6, diag=None):
    """Parameters (W, V, b, U, c) of the linear recurrent test model, flat in
    that order: Gaussian W of spectral scale about `scale` (or diag(diag)),
    Gaussian V, U / sqrt(H), small Gaussian biases."""
    rng = np.random.default_rng(seed)
    W = scale * rng.standard_normal((H, H)) / np.sqrt(H)
    if diag is not None:
        W = np.diag(np.asarray(diag, dtype=float))
    V = rng.standard_normal((H, 2))
    b = 0.3 * rng.standard_normal(H)
    U = rng.standard_normal((2, H)) / np.sqrt(H)
    c = 0.2 * rng.standard_normal(2)
    return np.concatenate([W.ravel(), V.ravel(), b, U.ravel(), c])
