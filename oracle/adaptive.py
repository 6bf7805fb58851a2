"""Adaptive regularisation around the minSR solve, in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

  ||T||      Frobenius norm of T.  The paper writes ||T|| without naming
             the norm; the Frobenius norm is the default matrix norm of the
             array libraries such code is written with, it is exact and
             cheap, and it bounds the spectral norm from above by at most
             sqrt(rank T).
  lambda     c ||T||^{2/3} with c = 3e-4 in the paper's 2D Heisenberg runs
             (Sec. 3.3; App. D, Table 1)
  tau        (I - lambda (T + lambda I)^{-1}) e' = e' - lambda x, with
             x = (T + lambda I)^{-1} e'                (App. F, Eq. trust-region-lr)
             For the pseudo-inverse solve (lambda = 0) tau = T x = T T^+ e',
             the part of e' in the range of T: the lambda -> 0 limit of the
             same expression and the quantity g^T S^+ g of App. F's
             pseudo-inverse derivation.
  eta_*      eta / ||tau||_2                           (App. F)
  rho        (E(theta) - E(theta - dtheta)) / (g^T dtheta - dtheta^T S dtheta / 2)
             with g = O' e' (the energy gradient), S = O' O'^T; for
             dtheta = eta_used O' x this is
             (E(theta) - E(theta - dtheta)) / (eta_used e'^T tau - eta_used^2 ||tau||^2 / 2),
             which under the trust-region rate (eta_used ||tau|| = eta) is
             App. G's (E - E') / (eta_* e'^T tau - eta^2 / 2).  The update
             of this project is theta <- theta - dtheta, so App. G's
             E_{theta + dtheta} is the energy at theta - dtheta.
  lambda'    omega lambda if rho < 1/4, lambda / omega if rho > 3/4,
             lambda otherwise (App. G; omega = 3/2 there).  A ratio that is
             not a number (a failed trial) counts as rho < 1/4.
  E(theta - dtheta) is estimated from fresh samples of the trial
  parameters (App. G's extra forward pass): Philox key `key`, counter
  (counter XOR 2^63) -- a stream no step's own samples use -- then local
  energies and their sample mean.
"""
import numpy as np

from . import hamiltonian, jacobian, minsr, model, philox

TRIAL_COUNTER_BIT = 1 << 63


def tnorm(T):
    """Frobenius norm of T: sqrt(sum_ij T_ij^2)."""
    return float(np.sqrt(np.sum(T * T)))


def lambda_pow23(T, coef):
    """Sec. 3.3 schedule lambda = coef * ||T||^{2/3}."""
    return coef * tnorm(T) ** (2.0 / 3.0)


def tau_vector(T, ep, x, lam, pinv):
    """App. F: tau = e' - lambda x (Cholesky), T x (pseudo-inverse)."""
    if pinv:
        return T @ x
    return ep - lam * x


def predicted_decrease(eta_used, ep, tau):
    """App. G's quadratic-model decrease for dtheta = eta_used O' x."""
    return eta_used * float(ep @ tau) - 0.5 * eta_used ** 2 * float(tau @ tau)


def lm_ratio(E0, E1, eta_used, ep, tau):
    """App. G: measured over predicted energy decrease."""
    return (E0 - E1) / predicted_decrease(eta_used, ep, tau)


def lm_next(lam, rho, omega):
    """App. G's update of the damping from the ratio."""
    if not (rho >= 0.25):          # includes a ratio that is not a number
        return omega * lam
    if rho > 0.75:
        return lam / omega
    return lam


def step(spec, theta, m, ham, Ns, eta, lam, mu, key, counter, pinv_cutoff=0.0,
         lam_mode="const", trust_region=False, omega=1.5):
    """Alg. 1's loop body with the adaptive pieces.

    lam_mode  "const": lambda = lam; "pow23": lambda = lam ||T||^{2/3};
              "lm": lambda = lam (the carried damping), and the step
              returns lam_next from App. G's ratio.
    trust_region  use eta_* = eta / ||tau|| (App. F) in place of eta."""
    u = philox.uniforms(key, counter, Ns, spec.N)
    sigma, lp = model.sample(spec, theta, u)
    eps = hamiltonian.local_energy(spec, theta, ham, sigma, lp)
    D = jacobian.log_derivatives(spec, theta, sigma)
    Op, ep, E = minsr.real_form(D, eps)
    T = Op.T @ Op
    tn = tnorm(T)
    pinv = pinv_cutoff > 0.0
    if lam_mode == "pow23":
        lam_used = lam * tn ** (2.0 / 3.0)
    else:
        lam_used = lam
    x = minsr.solve(T, ep, lam_used, pinv_cutoff)
    tau = tau_vector(T, ep, x, lam_used, pinv)
    tnorm_tau = float(np.sqrt(tau @ tau))
    eta_used = eta / tnorm_tau if trust_region else eta
    dtheta = eta_used * (Op @ x)
    res = dict(sigma=sigma, logpsi=lp, eps=eps, E=E, Op=Op, ep=ep, T=T, x=x, dtheta=dtheta,
               tnorm=tn, lam_used=lam_used, tau=tau, tau_norm=tnorm_tau, eta_used=eta_used,
               ep_tau=float(ep @ tau))
    if lam_mode == "lm":
        trial = theta - dtheta
        u1 = philox.uniforms(key, counter ^ TRIAL_COUNTER_BIT, Ns, spec.N)
        s1, lp1 = model.sample(spec, trial, u1)
        e1 = hamiltonian.local_energy(spec, trial, ham, s1, lp1)
        E1 = float(np.mean(e1).real)
        rho = lm_ratio(float(E.real), E1, eta_used, ep, tau)
        res.update(E_trial=E1, rho=rho, lam_next=lm_next(lam, rho, omega), sigma_trial=s1)
    theta_new, m_new = minsr.momentum(theta, m, dtheta, mu)
    res.update(theta=theta_new, m=m_new)
    return res
