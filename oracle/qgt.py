"""The subsampled quantum geometric tensor of Prop. 3 (Sec. 5; App. H), in
float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

  population   by enumeration of all configurations (small N): the Born
               weights P, mu_i = E[O_i], X = O - mu, the population QGT
               Q_ij = E[X_i X_j^*] and the average single-sample variance
               V_avg = (1 / N_p^2) sum_ij Var(X_i X_j^*),
               Var(Z) = E|Z - E Z|^2 = E|Z|^2 - |E Z|^2
  estimate     Q~ = (1 / N_s) sum_s X(sigma_s) X(sigma_s)^dagger with the
               population mean (Eq. Qtilde_est)
  bound        ||Q - Q~||_F <= (N_p / sqrt(N_s)) sqrt(V_avg / epsilon) with
               probability at least 1 - epsilon; for S = Re Q the right-hand
               side is alpha^-1 sqrt(V_avg / epsilon), alpha = sqrt(N_s) / N_p
               (Eq. UB)
  subsampled_S S~ = O' O'^T with O' the empirically centred real form of
               Eq. real-valued (the metric the minSR step works with)
"""
import math

import numpy as np

from . import jacobian, minsr, model


def all_configs(N):
    idx = np.arange(2 ** N)
    return ((idx[:, None] >> (N - 1 - np.arange(N))[None, :]) & 1).astype(np.int64)


def population(spec, theta):
    s = all_configs(spec.N)
    lp = model.log_psi(spec, theta, s)
    P = np.exp(2.0 * lp.real)
    D = jacobian.log_derivatives(spec, theta, s)            # (2^N, N_p), complex or real
    mu = P @ D
    X = D - mu
    Q = (X.T * P) @ np.conj(X)                               # E[X_i X_j^*]
    A = np.abs(X) ** 2
    M = (A.T * P) @ A                                        # E|X_i|^2 |X_j|^2 = E|X_i X_j^*|^2
    v_avg = float(np.mean(M - np.abs(Q) ** 2))
    return dict(configs=s, P=P, mu=mu, X=X, Q=Q, V_avg=v_avg)


def estimate(Xs):
    """Q~ from population-centred rows Xs (N_s, N_p)."""
    return (Xs.T @ np.conj(Xs)) / Xs.shape[0]


def bound(Np, Ns, v_avg, epsilon):
    return Np / math.sqrt(Ns) * math.sqrt(v_avg / epsilon)


def subsampled_S(D, eps_dummy=None):
    """S~ = O' O'^T from raw log-derivatives D (N_s, N_p)."""
    eps = np.zeros(D.shape[0]) if eps_dummy is None else eps_dummy
    Op, _, _ = minsr.real_form(D, eps)
    return Op @ Op.T
