"""One minSR iteration (Alg. 1) in float64.

  E        = mean_s eps_s                                   (Eq. energy)
  O_ks     = d_k log Psi(sigma^(s)) / sqrt(N_s)              (Sec. 2.3)
  Obar     = O - row means;  ebar_s = (eps_s - E)^* / sqrt(N_s)
  O', e'   = (Re Obar, Im Obar),  2 (Re ebar; -Im ebar)      (Eq. real-valued)
             (a positive ansatz keeps only the real block)
  T        = O'^T O'                                         (Eq. minsrR)
  x        = (T + lambda I)^{-1} e'   (Cholesky), or the Moore-Penrose
             pseudo-inverse of T at lambda = 0 (App. F) with eigenvalues at
             or below cutoff * lambda_max(T) dropped
  dtheta   = eta O' x                                        (Eq. minsrR)
  m        = mu m + (1 - mu) dtheta;  theta = theta - m      (App. B)

Orientation: O' is N_p x n (n = N_s, or 2 N_s for a complex ansatz), as in
the paper.  Library steps: matmul, scipy Cholesky, numpy eigh.
"""
import numpy as np
import scipy.linalg

from . import hamiltonian, jacobian, model, philox


def real_form(D, eps):
    """O' (N_p x n), e' (n,), E (complex) from raw log-derivatives D
    (N_s x N_p) and local energies eps (N_s,)."""
    Ns = D.shape[0]
    O = D.T / np.sqrt(Ns)
    Obar = O - O.mean(axis=1, keepdims=True)
    E = np.mean(eps)
    ebar = np.conj(eps - E) / np.sqrt(Ns)
    if np.iscomplexobj(D):
        Op = np.concatenate([Obar.real, Obar.imag], axis=1)
        ep = 2.0 * np.concatenate([ebar.real, -ebar.imag])
    else:
        Op = Obar
        ep = 2.0 * ebar.real
    return Op, ep, E


def solve(T, ep, lam, pinv_cutoff=0.0):
    """x = (T + lam I)^{-1} e' (pinv_cutoff == 0), else the pseudo-inverse
    solution of T x = e' with relative eigenvalue cutoff."""
    n = T.shape[0]
    if pinv_cutoff > 0.0:
        w, V = np.linalg.eigh(T)
        keep = w > pinv_cutoff * w[-1]
        return V[:, keep] @ ((V[:, keep].T @ ep) / w[keep])
    c = scipy.linalg.cho_factor(T + lam * np.eye(n), lower=True)
    return scipy.linalg.cho_solve(c, ep)


def update(D, eps, eta, lam, pinv_cutoff=0.0):
    """The minSR direction dtheta and its intermediates."""
    Op, ep, E = real_form(D, eps)
    T = Op.T @ Op
    x = solve(T, ep, lam, pinv_cutoff)
    dtheta = eta * (Op @ x)
    return dict(E=E, Op=Op, ep=ep, T=T, x=x, dtheta=dtheta)


def momentum(theta, m, dtheta, mu):
    """App. B: m <- mu m + (1 - mu) dtheta; theta <- theta - m."""
    m_new = mu * m + (1.0 - mu) * dtheta
    return theta - m_new, m_new


def step(spec, theta, m, ham, Ns, eta, lam, mu, key, counter, pinv_cutoff=0.0):
    """Alg. 1, one pass of its loop body, with uniforms from Philox."""
    u = philox.uniforms(key, counter, Ns, spec.N)
    sigma, lp = model.sample(spec, theta, u)
    eps = hamiltonian.local_energy(spec, theta, ham, sigma, lp)
    D = jacobian.log_derivatives(spec, theta, sigma)
    res = update(D, eps, eta, lam, pinv_cutoff)
    theta_new, m_new = momentum(theta, m, res["dtheta"], mu)
    res.update(sigma=sigma, logpsi=lp, eps=eps, theta=theta_new, m=m_new)
    return res
