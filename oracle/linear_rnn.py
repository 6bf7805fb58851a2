"""The linear recurrent test model of App. C (Sec. 2.5, Props. 1 and 2), in
float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The model (App. C.1, Eq. linear_rnn and Eq. softmax_def): a real, positive
autoregressive wave function over N sites with local dimension q = 2,

    h_0 = 0,   z_i = U h_{i-1} + c,   p_i = softmax(z_i),
    h_i = W h_{i-1} + V onehot(sigma_i) + b,
    log Psi(sigma) = (1/2) sum_i log p_i[sigma_i]      (Eq. logpsi_sum)

Parameters theta = (W [H x H], V [H x q], b [H], U [q x H], c [q]), each
block row-major, in that order (the order of Prop. 1).

  log_psi / sample     the forward recursion (sampling draws sigma_i = 0
                       when u < p_i[0], else 1, from caller uniforms)
  log_derivatives      O = d log Psi / d theta per configuration, by
                       reverse accumulation through the recursion with the
                       softmax score (Eq. softmax_score)
  gauge_direction      the generator d theta_X = ([X, W], X V, X b, -U X, 0)
                       of Prop. 1 (Eq. prop_gauge_direction)
  gauge_transform      the finite map (A W A^-1, A V, A b, U A^-1, c) of
                       Eq. gauge_map
  population_S         the population SR matrix by enumeration: Born
                       weights P, O-bar = O - E[O], S = E[O-bar O-bar^T]
  chi                  chi_{a,i} = E[u_a^T C_i u_a], C_i = diag(p_i) - p_i
                       p_i^T, u_a = U e_a (Eq. prop_chi_def), by enumeration
  geometric_factor     m_{i-1}(r) = sum_{k=0}^{i-2} r^k (Eq. geometric_factor)
  closed_form_Sbb      S_{b_a b_a} = (1/4) sum_i m_{i-1}(r_a)^2 chi_{a,i} for
                       a diagonal W = diag(r) (Eq. Sbaba)
"""
import numpy as np

Q = 2   # local dimension (spin 1/2)


def num_params(H, q=Q):
    return H * H + H * q + H + q * H + q


def offsets(H, q=Q):
    """Start of each block in the flat theta: W, V, b, U, c."""
    o = {}
    k = 0
    for name, n in (("W", H * H), ("V", H * q), ("b", H), ("U", q * H), ("c", q)):
        o[name] = k
        k += n
    return o


def unpack(theta, H, q=Q):
    o = offsets(H, q)
    W = theta[o["W"]:o["W"] + H * H].reshape(H, H)
    V = theta[o["V"]:o["V"] + H * q].reshape(H, q)
    b = theta[o["b"]:o["b"] + H]
    U = theta[o["U"]:o["U"] + q * H].reshape(q, H)
    c = theta[o["c"]:o["c"] + q]
    return W, V, b, U, c


def pack(W, V, b, U, c):
    return np.concatenate([np.ravel(W), np.ravel(V), np.ravel(b), np.ravel(U), np.ravel(c)])


def _softmax(z):
    e = np.exp(z - np.max(z))
    return e / np.sum(e)


def _run(theta, H, sig):
    """Conditionals p_i [N, q] and the states h_{i-1} [N, H] feeding site i
    for one configuration."""
    W, V, b, U, c = unpack(theta, H)
    N = len(sig)
    h = np.zeros(H)
    ps = np.zeros((N, Q))
    hs = np.zeros((N, H))
    for i in range(N):
        hs[i] = h
        ps[i] = _softmax(U @ h + c)
        h = W @ h + V[:, sig[i]] + b
    return ps, hs


def log_psi(theta, H, sigma):
    sigma = np.atleast_2d(sigma)
    out = np.zeros(sigma.shape[0])
    for s, sig in enumerate(sigma):
        ps, _ = _run(theta, H, sig)
        out[s] = 0.5 * sum(np.log(ps[i, sig[i]]) for i in range(len(sig)))
    return out


def sample(theta, H, N, u):
    """Exact autoregressive draws: sigma_i = 0 if u[s, i] < p_i[0] else 1."""
    W, V, b, U, c = unpack(theta, H)
    Ns = u.shape[0]
    sigma = np.zeros((Ns, N), dtype=np.int64)
    lp = np.zeros(Ns)
    for s in range(Ns):
        h = np.zeros(H)
        acc = 0.0
        for i in range(N):
            p = _softmax(U @ h + c)
            k = 0 if u[s, i] < p[0] else 1
            sigma[s, i] = k
            acc += np.log(p[k])
            h = W @ h + V[:, k] + b
        lp[s] = 0.5 * acc
    return sigma, lp


def log_derivatives(theta, H, sigma):
    """O[s] = d log Psi(sigma_s) / d theta, shape (Ns, N_p).

    The site score is d log p_i[sigma_i] = (e_sigma_i - p_i)^T dz_i
    (Eq. softmax_score); with the factor 1/2 of log Psi, g_i = (e - p_i)/2
    is the adjoint of z_i.  z_i = U h_{i-1} + c gives dU += g_i h_{i-1}^T,
    dc += g_i and adds U^T g_i to the adjoint of h_{i-1}; h_i = W h_{i-1} +
    V e_sigma_i + b gives, for the adjoint a_i of h_i, dW += a_i h_{i-1}^T,
    dV[:, sigma_i] += a_i, db += a_i and adds W^T a_i to the adjoint of
    h_{i-1}.  h_N feeds nothing, so a_N = 0."""
    sigma = np.atleast_2d(sigma)
    W, V, b, U, c = unpack(theta, H)
    O = np.zeros((sigma.shape[0], num_params(H)))
    for s, sig in enumerate(sigma):
        ps, hs = _run(theta, H, sig)
        N = len(sig)
        dW = np.zeros((H, H)); dV = np.zeros((H, Q)); db = np.zeros(H)
        dU = np.zeros((Q, H)); dc = np.zeros(Q)
        a = np.zeros(H)                       # adjoint of h_i, i = N first
        for i in range(N - 1, -1, -1):        # site i + 1 of the paper
            hprev = hs[i]
            # h_i = W h_{i-1} + V e + b
            dW += np.outer(a, hprev)
            dV[:, sig[i]] += a
            db += a
            # z_i = U h_{i-1} + c
            e = np.zeros(Q); e[sig[i]] = 1.0
            g = 0.5 * (e - ps[i])
            dU += np.outer(g, hprev)
            dc += g
            a = W.T @ a + U.T @ g             # adjoint of h_{i-1}
        O[s] = pack(dW, dV, db, dU, dc)
    return O


def gauge_direction(theta, H, X):
    """d theta_X = ([X, W], X V, X b, -U X, 0) (Prop. 1)."""
    W, V, b, U, c = unpack(theta, H)
    return pack(X @ W - W @ X, X @ V, X @ b, -U @ X, np.zeros(Q))


def gauge_transform(theta, H, A):
    """theta mapped by A in GL(H) (Eq. gauge_map)."""
    W, V, b, U, c = unpack(theta, H)
    Ai = np.linalg.inv(A)
    return pack(A @ W @ Ai, A @ V, A @ b, U @ Ai, c)


def all_configs(N):
    idx = np.arange(2 ** N)
    return ((idx[:, None] >> (N - 1 - np.arange(N))[None, :]) & 1).astype(np.int64)


def population_S(theta, H, N):
    """(S, P, O) with S = E[(O - E O)(O - E O)^T] under P = Psi^2 (real
    model: S = Re Q = Q), by enumeration of the 2^N configurations."""
    s = all_configs(N)
    P = np.exp(2.0 * log_psi(theta, H, s))
    O = log_derivatives(theta, H, s)
    X = O - P @ O
    return (X.T * P) @ X, P, O


def chi(theta, H, N, a):
    """chi_{a,i}, i = 1..N: the softmax covariance at site i along the
    readout u_a = U e_a, averaged over histories drawn from P
    (Eq. prop_chi_def)."""
    W, V, b, U, c = unpack(theta, H)
    ua = U[:, a]
    s = all_configs(N)
    P = np.exp(2.0 * log_psi(theta, H, s))
    out = np.zeros(N)
    for w, sig in zip(P, s):
        ps, _ = _run(theta, H, sig)
        for i in range(N):
            C = np.diag(ps[i]) - np.outer(ps[i], ps[i])
            out[i] += w * (ua @ C @ ua)
    return out


def geometric_factor(r, i):
    """m_{i-1}(r) = sum_{k=0}^{i-2} r^k (zero for i = 1)."""
    return sum(r ** k for k in range(i - 1))


def closed_form_Sbb(theta, H, N, a):
    """(1/4) sum_{i=1}^{N} m_{i-1}(r_a)^2 chi_{a,i} with r_a = W[a, a]; the
    derivation assumes W diagonal (App. C.5)."""
    W, _, _, _, _ = unpack(theta, H)
    r = W[a, a]
    x = chi(theta, H, N, a)
    return 0.25 * sum(geometric_factor(r, i) ** 2 * x[i - 1] for i in range(1, N + 1))


def bias_index(H, a):
    return offsets(H)["b"] + a
