"""Conditioning of the regularised minSR solve, in float64 (App. E).

TEST INFRASTRUCTURE ONLY (see the package docstring).

  spectrum      eigenvalues of the symmetric T, ascending (library eigvalsh)
  kappa2        kappa_2(T + lambda I) = (w_max + lambda) / (w_min + lambda),
                T positive semidefinite, so its computed smallest eigenvalue
                is taken as max(w_min, 0) (App. E: kappa_2(S_lambda) for the
                positive semidefinite S; T shares its non-zero spectrum)
  digits        d = -log10(kappa_2 * eps), the rule-of-thumb number of
                reliable decimal digits for machine epsilon eps (App. E,
                Eq. errors); eps = 2^-52 for FP64, 2^-23 for FP32
"""
import math

import numpy as np


def spectrum(T):
    return np.linalg.eigvalsh(T)


def kappa2(w, lam):
    """(w_max + lambda) / (max(w_min, 0) + lambda) for ascending w."""
    lo = max(float(w[0]), 0.0)
    den = lo + lam
    return math.inf if den <= 0.0 else (float(w[-1]) + lam) / den


def digits(kappa, eps):
    return -math.log10(kappa * eps) if math.isfinite(kappa) else -math.inf


def condition(T, lam, eps):
    """(w_min, w_max, kappa_2, d) of T + lambda I."""
    w = spectrum(T)
    k = kappa2(w, lam)
    return float(w[0]), float(w[-1]), k, digits(k, eps)
