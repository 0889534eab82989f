"""Pins of the oracle's covariance adaptation and full-covariance sampling
(Alg. 1 sampling step; Eqs. mean_update, cov_update, s_formula): NumPy's
weighted covariance, the parallel-axis identity for a scatter about a point
other than the weighted mean, rank and definiteness, the diagonal case
against the C oracle's sampler, the weights against the C oracle's update,
and the covariance of drawn samples against Sigma (a transposed factor
fails it)."""
import numpy as np
import pytest

from oracle import cov
import workloads as W


def _data(K=40, H=3, seed=0):
    rng = np.random.default_rng(seed)
    U = rng.normal(0, 0.4, (K, H, 14)) + rng.normal(0, 0.2, (1, H, 14))
    return U


def test_equal_weights_full_step_is_the_sample_covariance():
    U = _data()
    K, n = U.shape[0], U[0].size
    w = np.full(K, 1.0 / K)
    nu_new = cov.mean_update(U, w, np.zeros(n), 1.0)
    S = cov.cov_update(U, w, nu_new, np.eye(n), 1.0)
    np.testing.assert_allclose(S, np.cov(U.reshape(K, n), rowvar=False, bias=True), rtol=0, atol=1e-14)


def test_weighted_full_step_matches_numpy_aweights():
    U = _data(seed=1)
    K, n = U.shape[0], U[0].size
    rng = np.random.default_rng(2)
    s = rng.exponential(1.0, K)
    w = s / s.sum()
    nu_new = cov.mean_update(U, w, np.zeros(n), 1.0)
    S = cov.cov_update(U, w, nu_new, np.zeros((n, n)), 1.0)
    ref = np.cov(U.reshape(K, n), rowvar=False, aweights=s, bias=True)
    np.testing.assert_allclose(S, ref, rtol=0, atol=1e-14)


def test_scatter_about_the_updated_mean_obeys_the_parallel_axis_identity():
    """With eta < 1 the scatter is about nu_{m+1}, not about the weighted
    mean mu: Delta Sigma = Cov_w + (mu - nu_{m+1})(mu - nu_{m+1})^T."""
    U = _data(seed=3)
    K, n = U.shape[0], U[0].size
    rng = np.random.default_rng(4)
    s = rng.exponential(1.0, K)
    w = s / s.sum()
    nu = rng.normal(0, 0.5, n)
    eta = 0.3
    nu_new = cov.mean_update(U, w, nu, eta)
    mu = w @ U.reshape(K, n)
    np.testing.assert_allclose(nu_new, 0.7 * nu + 0.3 * mu, rtol=0, atol=1e-15)
    S0 = np.diag(rng.uniform(0.1, 0.2, n))
    S = cov.cov_update(U, w, nu_new, S0, eta, eps=1e-3)
    d = mu - nu_new
    ref = 0.7 * S0 + 0.3 * (np.cov(U.reshape(K, n), rowvar=False, aweights=s, bias=True) + np.outer(d, d)) \
        + 1e-3 * np.eye(n)
    np.testing.assert_allclose(S, ref, rtol=0, atol=1e-14)


def test_eta_zero_keeps_sigma_and_eps_adds_to_the_diagonal():
    U = _data(seed=5)
    K, n = U.shape[0], U[0].size
    A = np.random.default_rng(6).normal(size=(n, n))
    S0 = A @ A.T
    w = np.full(K, 1.0 / K)
    np.testing.assert_array_equal(cov.cov_update(U, w, np.zeros(n), S0, 0.0), S0)
    np.testing.assert_allclose(cov.cov_update(U, w, np.zeros(n), S0, 0.0, eps=0.25) - S0, 0.25 * np.eye(n),
                               rtol=0, atol=1e-13)


def test_no_weight_keeps_sigma():
    U = _data(seed=14)
    K, n = U.shape[0], U[0].size
    S0 = np.diag(np.linspace(0.1, 0.2, n))
    np.testing.assert_array_equal(cov.cov_update(U, np.zeros(K), np.zeros(n), S0, 0.5, eps=1e-3), S0)


def test_update_is_symmetric_psd_with_rank_at_most_the_weighted_samples():
    U = _data(K=30, H=4, seed=7)
    K, n = U.shape[0], U[0].size
    w = np.zeros(K)
    w[[2, 11, 29]] = [0.5, 0.3, 0.2]
    nu_new = cov.mean_update(U, w, np.zeros(n), 1.0)
    S = cov.cov_update(U, w, nu_new, np.eye(n), 1.0)
    np.testing.assert_allclose(S, S.T, rtol=0, atol=1e-15)
    ev = np.linalg.eigvalsh(S)
    assert ev.min() > -1e-13
    # three points about their own weighted mean span at most two directions
    assert np.sum(ev > 1e-10 * ev.max()) == 2


def test_weights_shift_invariance_elites_and_nonfinite():
    rng = np.random.default_rng(8)
    c = rng.uniform(10, 20, 50)
    w = cov.weights(c, 0.7)
    np.testing.assert_allclose(w.sum(), 1.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(cov.weights(c + 1e3, 0.7), w, rtol=1e-12, atol=0)
    # the ratio of two weights is exp(-(c_a - c_b) / beta)
    np.testing.assert_allclose(w[3] / w[7], np.exp(-(c[3] - c[7]) / 0.7), rtol=1e-12)
    we = cov.weights(c, 0.7, n_elite=5)
    assert np.count_nonzero(we) == 5
    assert set(np.nonzero(we)[0]) == set(np.argsort(c)[:5])
    c2 = c.copy()
    c2[[0, 4]] = [np.inf, np.nan]
    w2 = cov.weights(c2, 0.7)
    assert w2[0] == 0 and w2[4] == 0 and abs(w2.sum() - 1) < 1e-15
    assert not cov.weights(np.full(4, np.inf), 1.0).any()


def test_mean_update_matches_the_c_oracle_update():
    import oracle
    U = _data(K=32, H=5, seed=9)
    rng = np.random.default_rng(10)
    c = rng.uniform(5, 9, 32)
    nu = rng.normal(0, 0.1, (5, 14))
    for eta, ne in ((1.0, None), (0.4, 6)):
        ref, nf, ess = oracle.Oracle.update(U, c, 0.5, nu, eta=eta, n_elite=ne)
        got = cov.mean_update(U, cov.weights(c, 0.5, ne), nu, eta).reshape(5, 14)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


def test_diagonal_sigma_reduces_to_the_diagonal_sampler():
    import oracle
    sc = W.make_scene(1)
    o = oracle.Oracle(sc)
    K, H, seed, m = 16, 6, 1234, 2
    rng = np.random.default_rng(11)
    nu = rng.normal(0, 0.2, (H, 14))
    sigma = rng.uniform(0.1, 0.6, 14)
    u_max = float(sc["u_max"])
    L = cov.factor(cov.diagonal_sigma(sigma, H))
    np.testing.assert_array_equal(np.diag(L), np.tile(sigma, H))  # sqrt(sigma^2) is exact in FP64
    got = cov.sample(nu, L, o.noise(seed, K, H, m), u_max)
    np.testing.assert_allclose(got, o.sample(nu, sigma, seed, K, m).reshape(K, -1), rtol=0, atol=1e-15)


def test_factor_is_lower_with_positive_diagonal():
    A = np.random.default_rng(12).normal(size=(9, 9))
    S = A @ A.T + 0.1 * np.eye(9)
    L = cov.factor(S)
    assert np.all(np.triu(L, 1) == 0) and np.all(np.diag(L) > 0)
    np.testing.assert_allclose(L @ L.T, S, rtol=0, atol=1e-12)


def test_drawn_samples_have_covariance_sigma():
    """Monte Carlo: the empirical covariance of L z over many standard
    normal z matches Sigma within five standard errors per entry; with L^T
    in place of L it would be L^T L, far off for this Sigma."""
    rng = np.random.default_rng(13)
    n, N = 6, 400_000
    A = rng.normal(size=(n, n))
    S = A @ A.T + 0.2 * np.eye(n)
    L = cov.factor(S)
    Z = rng.standard_normal((N, n))
    X = cov.sample(np.zeros(n), L, Z, np.inf)
    C = X.T @ X / N
    se = np.sqrt((np.outer(np.diag(S), np.diag(S)) + S * S) / N)
    assert np.all(np.abs(C - S) < 5 * se)
    LtL = L.T @ L
    assert np.max(np.abs(LtL - S) / se) > 50


@pytest.mark.parametrize("eta", [1.0, 0.5])
def test_plan_with_diagonal_sigma_and_eta_one_matches_the_c_oracle_plan_mean(eta):
    """First iteration of the full-covariance plan from a diagonal Sigma_0
    draws the diagonal sampler's samples, so its mean update equals the C
    oracle's one-iteration plan."""
    import oracle
    sc = W.make_scene(1)
    o = oracle.Oracle(sc)
    pp = W.plan_params(1)
    K, H = 16, 8
    x0 = W.initial_state(sc)
    sig = np.asarray(pp["sigma"], dtype=np.float64)
    r = cov.plan(o, x0, np.zeros((H, 14)), K, H, pp["lam"], cov.diagonal_sigma(sig, H), 1, 77, eta, 0.0,
                 float(sc["u_max"]))
    ref = o.plan(x0, np.zeros((H, 14)), K, H, pp["lam"], sig, 1, 77, eta=eta, nthreads=4)
    np.testing.assert_allclose(r["costs"], ref["costs"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(r["nu"], ref["nu"], rtol=0, atol=1e-13)
    ev = np.linalg.eigvalsh(r["Sigma"])
    assert ev.min() > -1e-12
