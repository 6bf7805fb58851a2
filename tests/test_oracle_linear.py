"""Pins of the linear recurrent test model of App. C (oracle/linear_rnn.py)
against what the paper and the mathematics fix, independently of the
oracle's own derivative code where possible:

  - Born normalisation by enumeration (the logits of site i must not see
    sigma_i: a model that read h_i instead of h_{i-1} fails);
  - O against central finite differences of log Psi;
  - the finite gauge map of Eq. gauge_map leaves log Psi unchanged for every
    configuration (App. C.1), and its generator of Prop. 1 is annihilated
    by every row of O and by the finite-sample and population S;
  - the population Fisher form equals the per-site sum (1/4) E[dz_i^T C_i
    dz_i] of App. C.3-C.4, with dz_i taken by finite differences of the
    logits;
  - Prop. 2: S_{b_a b_a} equals the closed form (1/4) sum_i m_{i-1}(r_a)^2
    chi_{a,i} of Eq. Sbaba (chi by enumeration of the softmax covariance),
    the marginal and expanding lower bounds of Eqs. prop_marginal_bound and
    prop_expanding_bound hold for lambda_max(S), and m_{i-1} has the closed
    forms of Eqs. marginal_m and expanding_m.
"""
import numpy as np
import pytest

from oracle import linear_rnn as lr
from tests.inputs import linear_theta as _theta


def test_layout_order_and_size():
    H = 5
    th = np.arange(lr.num_params(H), dtype=float)
    W, V, b, U, c = lr.unpack(th, H)
    assert lr.num_params(H) == H * H + 5 * H + 2
    assert W[1, 2] == H + 2 and V[0, 1] == H * H + 1 and b[0] == H * H + 2 * H
    assert U[1, 0] == H * H + 3 * H + H and c[1] == lr.num_params(H) - 1
    assert np.array_equal(lr.pack(W, V, b, U, c), th)


@pytest.mark.parametrize("N,H", [(1, 3), (6, 3), (8, 4)])
def test_born_normalisation(N, H):
    th = _theta(H, 10 + N)
    P = np.exp(2.0 * lr.log_psi(th, H, lr.all_configs(N)))
    assert abs(P.sum() - 1.0) < 1e-13


def test_first_site_is_softmax_of_c():
    # h_0 = 0, so p_1 = softmax(c) whatever W, V, b, U
    H = 4
    th = _theta(H, 3)
    c = lr.unpack(th, H)[4]
    for s0 in (0, 1):
        lp = lr.log_psi(th, H, np.array([[s0]]))[0]
        ref = 0.5 * (c[s0] - np.log(np.exp(c[0]) + np.exp(c[1])))
        assert abs(lp - ref) < 1e-15


def test_sampling_draws_the_conditionals():
    H, N = 3, 5
    th = _theta(H, 4)
    rng = np.random.default_rng(5)
    u = rng.random((40, N))
    sig, lp = lr.sample(th, H, N, u)
    assert np.allclose(lp, lr.log_psi(th, H, sig), rtol=0, atol=1e-14)
    # u below p_i[0] draws 0: evaluate the conditionals independently
    for s in range(40):
        W, V, b, U, c = lr.unpack(th, H)
        h = np.zeros(H)
        for i in range(N):
            z = U @ h + c
            p0 = 1.0 / (1.0 + np.exp(z[1] - z[0]))
            assert sig[s, i] == (0 if u[s, i] < p0 else 1)
            h = W @ h + V[:, sig[s, i]] + b


def test_log_derivatives_match_finite_differences():
    H, N = 3, 6
    th = _theta(H, 6)
    sig = lr.all_configs(N)[[0, 5, 17, 42, 63]]
    O = lr.log_derivatives(th, H, sig)
    h = 1e-6
    for k in range(lr.num_params(H)):
        e = np.zeros_like(th); e[k] = h
        fd = (lr.log_psi(th + e, H, sig) - lr.log_psi(th - e, H, sig)) / (2 * h)
        assert np.max(np.abs(fd - O[:, k])) < 1e-8, k


def test_finite_gauge_map_leaves_psi_unchanged():
    H, N = 4, 7
    th = _theta(H, 7)
    rng = np.random.default_rng(8)
    A = np.eye(H) + 0.5 * rng.standard_normal((H, H))
    assert np.linalg.cond(A) < 50
    s = lr.all_configs(N)
    lp0 = lr.log_psi(th, H, s)
    lp1 = lr.log_psi(lr.gauge_transform(th, H, A), H, s)
    assert np.max(np.abs(lp1 - lp0)) < 1e-12
    # the parameters themselves did move
    assert np.max(np.abs(lr.gauge_transform(th, H, A) - th)) > 0.1


def test_gauge_generator_is_tangent_to_the_orbit():
    # d/dt of the map at A = I + t X is the generator of Prop. 1
    H = 4
    th = _theta(H, 9)
    X = np.random.default_rng(10).standard_normal((H, H))
    t = 1e-6
    fd = (lr.gauge_transform(th, H, np.eye(H) + t * X)
          - lr.gauge_transform(th, H, np.eye(H) - t * X)) / (2 * t)
    assert np.max(np.abs(fd - lr.gauge_direction(th, H, X))) < 1e-8


@pytest.mark.parametrize("seed", [11, 12])
def test_gauge_directions_are_zero_modes_per_sample(seed):
    # Prop. 1 (i): O(sigma) . d theta_X = 0 for every configuration
    H, N = 5, 8
    th = _theta(H, seed)
    rng = np.random.default_rng(seed + 100)
    s = lr.all_configs(N)[rng.choice(2 ** N, 60, replace=False)]
    O = lr.log_derivatives(th, H, s)
    for _ in range(3):
        d = lr.gauge_direction(th, H, rng.standard_normal((H, H)))
        v = O @ d
        scale = np.abs(O) @ np.abs(d)
        assert np.all(np.abs(v) <= 1e-13 * scale)
    # a generic direction is not
    r = rng.standard_normal(lr.num_params(H))
    assert np.max(np.abs(O @ r)) > 1e-2


def test_gauge_directions_lie_in_ker_S():
    # Prop. 1 (ii): finite-sample O'O'^T and the population S both
    # annihilate d theta_X
    H, N = 3, 7
    th = _theta(H, 13)
    S, P, O = lr.population_S(th, H, N)
    rng = np.random.default_rng(14)
    d = lr.gauge_direction(th, H, rng.standard_normal((H, H)))
    nS = np.linalg.norm(S, 2)
    assert np.linalg.norm(S @ d) < 1e-13 * nS * np.linalg.norm(d)
    idx = rng.choice(2 ** N, 30, replace=False)
    Oc = O[idx] - O[idx].mean(axis=0)
    Sf = Oc.T @ Oc / 30
    assert np.linalg.norm(Sf @ d) < 1e-13 * np.linalg.norm(Sf, 2) * np.linalg.norm(d)
    # the number of zero modes is at least the gauge dimension H^2 (minus the
    # generators that leave theta fixed, none for a generic theta)
    G = np.stack([lr.gauge_direction(th, H, np.eye(H)[:, [i]] @ np.eye(H)[[j], :])
                  for i in range(H) for j in range(H)], axis=1)
    assert np.linalg.matrix_rank(G, tol=1e-10) == H * H
    w = np.linalg.eigvalsh(S)
    assert np.sum(np.abs(w) < 1e-12 * w.max()) >= H * H


def test_population_fisher_form_is_the_per_site_sum():
    # App. C.3-C.4: d theta^T S d theta = (1/4) sum_i E[dz_i^T C_i dz_i],
    # dz_i the change of the logits along d theta (central differences here)
    H, N = 3, 6
    th = _theta(H, 15)
    S, P, _ = lr.population_S(th, H, N)
    d = np.random.default_rng(16).standard_normal(lr.num_params(H))
    s = lr.all_configs(N)
    t = 1e-6

    def logits(theta, sig):
        W, V, b, U, c = lr.unpack(theta, H)
        h = np.zeros(H)
        zs = []
        for i in range(N):
            zs.append(U @ h + c)
            h = W @ h + V[:, sig[i]] + b
        return np.array(zs)

    rhs = 0.0
    for w, sig in zip(P, s):
        dz = (logits(th + t * d, sig) - logits(th - t * d, sig)) / (2 * t)
        ps, _ = lr._run(th, H, sig)
        for i in range(N):
            C = np.diag(ps[i]) - np.outer(ps[i], ps[i])
            rhs += w * (dz[i] @ C @ dz[i])
    rhs *= 0.25
    lhs = d @ S @ d
    assert abs(lhs - rhs) < 1e-7 * abs(lhs)


def test_geometric_factor_closed_forms():
    for i in range(1, 12):
        assert lr.geometric_factor(1.0, i) == i - 1            # Eq. marginal_m
        r = 1.7
        assert abs(lr.geometric_factor(r, i) - (1 - r ** (i - 1)) / (1 - r)) < 1e-12 * max(1, r ** i)
    N = 9
    assert sum((i - 1) ** 2 for i in range(1, N + 1)) == (N - 1) * N * (2 * N - 1) // 6


@pytest.mark.parametrize("r", [1.0, 1.3, 0.5, -1.2])
def test_prop2_closed_form_of_the_bias_element(r):
    # Eq. Sbaba: the diagonal element of the population S along b_a
    H, N, a = 3, 7, 1
    th = _theta(H, 17, diag=[0.4, r, -0.7])
    S, _, _ = lr.population_S(th, H, N)
    k = lr.bias_index(H, a)
    cf = lr.closed_form_Sbb(th, H, N, a)
    assert abs(S[k, k] - cf) < 1e-12 * cf


def test_prop2_lower_bounds():
    H, N, a = 3, 8, 0
    # marginal mode r_a = 1 (Eq. prop_marginal_bound)
    th = _theta(H, 18, diag=[1.0, 0.3, -0.5])
    S, _, _ = lr.population_S(th, H, N)
    x = lr.chi(th, H, N, a)
    chi0 = x.min()
    assert chi0 > 0
    lmax = np.linalg.eigvalsh(S).max()
    k = lr.bias_index(H, a)
    assert lmax >= S[k, k] * (1 - 1e-12)
    assert S[k, k] >= chi0 / 4 * (N - 1) * N * (2 * N - 1) / 6 * (1 - 1e-12)
    # expanding mode |r_a| > 1 (Eq. prop_expanding_bound)
    r = 1.4
    th = _theta(H, 19, diag=[r, 0.3, -0.5])
    S, _, _ = lr.population_S(th, H, N)
    x = lr.chi(th, H, N, a)
    m = (1 - r ** (N - 1)) / (1 - r)
    assert np.linalg.eigvalsh(S).max() >= 0.25 * m * m * x[N - 1] * (1 - 1e-12)


def test_planted_mistakes_fail_the_pins():
    # a sign error in the -U X block, or [W, X] for [X, W], breaks Prop. 1
    H, N = 4, 6
    th = _theta(H, 20)
    X = np.random.default_rng(21).standard_normal((H, H))
    O = lr.log_derivatives(th, H, lr.all_configs(N)[:20])
    W, V, b, U, c = lr.unpack(th, H)
    good = lr.gauge_direction(th, H, X)
    bad1 = lr.pack(X @ W - W @ X, X @ V, X @ b, U @ X, np.zeros(2))
    bad2 = lr.pack(W @ X - X @ W, X @ V, X @ b, -U @ X, np.zeros(2))
    assert np.max(np.abs(O @ good)) < 1e-12
    assert np.max(np.abs(O @ bad1)) > 1e-3
    assert np.max(np.abs(O @ bad2)) > 1e-3
