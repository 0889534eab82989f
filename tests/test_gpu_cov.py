"""GPU parity of the covariance adaptation and full-covariance sampling
(Alg. 1 sampling step; Eqs. mean_update, cov_update, s_formula) through the
C ABI against the FP64 oracle on the same inputs.

Tolerances, from the arithmetic:
* covariance update: FP64 products and sums (MFMA FP64) in another order
  than NumPy's: 1e-12 of the largest entry;
* Cholesky: FP64, blocked: 1e-10 of the largest entry of L (the test
  matrices have condition numbers below 1e4);
* samples: the product L z runs in FP32 over n <= 1400 terms of size
  |L| |z| <= 1: 5e-5 absolute;
* plans: FP32 rollouts against FP64 ones through a chaotic contact model,
  compared as the other plan tests do (median cost error, mean within a
  fraction of sigma), and Sigma within 2e-3 of its largest entry (measured
  3e-5 at the small workload).
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def mp():
    import paper_2511_21264_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(mp):
    c = mp.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def cov():
    from oracle import cov as c
    return c


def Td(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


def _spd(n, seed, scale=0.09):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n)) / np.sqrt(n)
    return scale * (A @ A.T + 0.1 * np.eye(n))


@pytest.mark.parametrize("K,H,eta", [(64, 20, 1.0), (1024, 64, 0.5), (37, 3, 0.3), (5, 1, 1.0), (32, 256, 0.7)])
def test_cov_update_matches_oracle(mp, ctx, cov, K, H, eta):
    n = 14 * H
    rng = np.random.default_rng(K + H)
    U = rng.normal(0, 0.3, (K, n)).astype(np.float32)
    s = rng.exponential(1.0, K)
    s[rng.random(K) < 0.3] = 0.0  # non-elite samples carry no weight
    s[0] = 1.0
    w = s / s.sum()
    nu = rng.normal(0, 0.1, n)
    S0 = _spd(n, K)
    ref = cov.cov_update(U.astype(np.float64), w, nu, S0, eta, 1e-4)
    out = torch.zeros((n, n), dtype=torch.float64, device=DEV)
    mp.mppi_cov_update(ctx, Td(U, torch.float32), Td(w), Td(nu), Td(S0), out, eta, 1e-4)
    got = out.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"cov update K={K} n={n} eta={eta}: max rel err {err:.2e}")
    assert err < 1e-12
    assert np.array_equal(got, got.T)


def test_cov_update_in_place_host_arrays_and_unnormalised_weights(mp, ctx, cov):
    K, n = 50, 70
    rng = np.random.default_rng(3)
    U = rng.normal(0, 0.3, (K, n)).astype(np.float32)
    s = rng.exponential(2.0, K)
    nu = rng.normal(0, 0.1, n)
    S0 = _spd(n, 4)
    ref = cov.cov_update(U.astype(np.float64), s / s.sum(), nu, S0, 0.6, 0.0)
    Sd = Td(S0)
    mp.mppi_cov_update(ctx, Td(U, torch.float32), Td(s), Td(nu), Sd, Sd, 0.6)
    assert np.abs(Sd.cpu().numpy() - ref).max() < 1e-12 * np.abs(ref).max()
    out = np.zeros((n, n))
    mp.mppi_cov_update(ctx, U, s, nu, S0, out, 0.6)
    assert np.abs(out - ref).max() < 1e-12 * np.abs(ref).max()
    # no weight at all: Sigma is kept (and eps is not added)
    mp.mppi_cov_update(ctx, U, np.zeros(K), nu, S0, out, 0.6, 1e-3)
    assert np.array_equal(out, np.tril(S0) + np.tril(S0, -1).T)


def test_cov_update_rejects_bad_arguments(mp, ctx):
    U = np.zeros((4, 14), np.float32)
    S = np.eye(14)
    for kw in (dict(eta=1.5), dict(eta=-0.1), dict(eps=-1.0)):
        args = dict(eta=0.5, eps=0.0)
        args.update(kw)
        with pytest.raises(mp.MppiError):
            mp.mppi_cov_update(ctx, U, np.ones(4), np.zeros(14), S, np.zeros_like(S), args["eta"], args["eps"])
    with pytest.raises(mp.MppiError):
        mp.mppi_cov_update(ctx, U, np.array([1.0, -1.0, 0.0, 0.0]), np.zeros(14), S, np.zeros_like(S), 0.5)


@pytest.mark.parametrize("n", [14, 33, 280, 896, 1400, 3584])
def test_cholesky_matches_oracle(mp, ctx, cov, n):
    S = _spd(n, n)
    ref = cov.factor(S)
    L = torch.zeros((n, n), dtype=torch.float64, device=DEV)
    mp.mppi_cholesky(ctx, Td(S), L)
    got = L.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"cholesky n={n}: max rel err {err:.2e}")
    assert err < 1e-10
    assert np.all(np.triu(got, 1) == 0)


def test_cholesky_in_place_host_and_not_positive_definite(mp, ctx, cov):
    n = 100
    S = _spd(n, 5)
    Sd = Td(S)
    mp.mppi_cholesky(ctx, Sd, Sd)
    assert np.abs(Sd.cpu().numpy() - cov.factor(S)).max() < 1e-10
    L = np.zeros((n, n))
    mp.mppi_cholesky(ctx, S, L)
    assert np.abs(L - cov.factor(S)).max() < 1e-10
    bad = np.diag(np.linspace(1.0, 2.0, n))
    bad[40, 40] = -0.5
    with pytest.raises(mp.MppiError) as e:
        mp.mppi_cholesky(ctx, bad, L)
    assert e.value.code == mp.E_NOTPD and "column 40" in str(e.value)


@pytest.mark.parametrize("K,H", [(64, 20), (1024, 64), (70, 3), (1, 100), (8, 256)])
def test_sample_full_matches_oracle(mp, ctx, cov, K, H):
    import oracle
    sc = W.make_scene(1)
    n = 14 * H
    rng = np.random.default_rng(7 + H)
    nu = rng.normal(0, 0.2, (H, 14)).astype(np.float32)
    L = cov.factor(_spd(n, 11 + H))
    seed, m, u_max = 99, 3, float(sc["u_max"])
    U = torch.zeros((K, H, 14), device=DEV)
    mp.mppi_sample_full(ctx, Td(nu, torch.float32), Td(L), seed, m, K, U, u_max)
    ref = cov.sample(nu.astype(np.float64), L, oracle.Oracle.noise(seed, K, H, m), u_max)
    err = np.abs(U.cpu().numpy().reshape(K, n) - ref).max()
    print(f"sample_full K={K} n={n}: max err {err:.2e}")
    assert err < 5e-5


def test_sample_full_with_diagonal_factor_is_the_diagonal_sampler(mp, ctx, cov):
    sc = W.make_scene(1)
    scene = mp.Scene(ctx, sc)
    K, H, seed, m = 256, 16, 5, 1
    rng = np.random.default_rng(8)
    nu = rng.normal(0, 0.2, (H, 14)).astype(np.float32)
    sigma = rng.uniform(0.1, 0.5, 14).astype(np.float32)
    L = np.diag(np.tile(sigma.astype(np.float64), H))
    U = np.zeros((K, H, 14), np.float32)
    mp.mppi_sample_full(ctx, nu, L, seed, m, K, U, float(sc["u_max"]))
    ref = np.zeros((K, H, 14), np.float32)
    mp.mppi_sample(ctx, scene, nu, sigma, seed, m, K, ref)
    # one rounding of sigma * z + nu (fma) against two (product, then sum)
    assert np.abs(U - ref).max() <= 2 * np.finfo(np.float32).eps * float(sc["u_max"])
    scene.close()


def _plan_case(mp, ctx, cov, qp_params=None, n_elite=None):
    import oracle
    sc = W.make_scene(1)
    scene = mp.Scene(ctx, sc)
    o = oracle.Oracle(sc)
    pp = W.plan_params(1)
    cp = W.cov_params(1)
    K, H, M = pp["K"], pp["H"], pp["M"]
    n = 14 * H
    x0 = W.initial_state(sc).astype(np.float32)
    sig = pp["sigma"].astype(np.float32)
    Unew = torch.zeros((H, 14), device=DEV)
    costs = torch.zeros(K, device=DEV)
    Sout = torch.zeros((n, n), dtype=torch.float64, device=DEV)
    st = mp.mppi_plan_cov(ctx, scene, Td(x0, torch.float32), torch.zeros((H, 14), device=DEV), K, H, pp["lam"],
                          Td(sig, torch.float32), Unew, costs, eps=cp["eps"], Sigma_out=Sout, qp=qp_params, M=M,
                          seed=pp["seed"], eta=cp["eta"], n_elite=n_elite or 0)
    project = None
    if qp_params is not None:
        from oracle import qp as qpo
        dt = sc["h"] * sc["n_sub"]
        X0 = np.repeat(x0[None, 28:42].astype(np.float64), K, axis=0)

        def project(U):
            return qpo.project_sequences(U, X0, dt, float(sc["u_max"]),
                                         np.asarray(qp_params["pos_lo"], np.float32).astype(np.float64),
                                         np.asarray(qp_params["pos_hi"], np.float32).astype(np.float64),
                                         qp_params["acc_max"], qp_params["jerk_max"], qp_params["rho"],
                                         qp_params["iters"], qp_params["alpha"])
    r = cov.plan(o, x0.astype(np.float64), np.zeros((H, 14)), K, H, pp["lam"],
                 cov.diagonal_sigma(sig.astype(np.float64), H), M, pp["seed"], cp["eta"], cp["eps"],
                 float(sc["u_max"]), n_elite=n_elite, project=project)
    cg = costs.cpu().numpy()
    rel = np.abs(cg - r["costs"]) / np.abs(r["costs"])
    dU = np.abs(Unew.cpu().numpy() - r["nu"]).max()
    Sg = Sout.cpu().numpy()
    dS = np.abs(Sg - r["Sigma"]).max() / np.abs(r["Sigma"]).max()
    print(f"plan cov{' + qp' if qp_params else ''}: cost rel err median {np.median(rel):.2e} max {rel.max():.2e}; "
          f"|dU|max {dU:.2e}; |dSigma|/max {dS:.2e}; ess {st['ess']:.2f}")
    scene.close()
    return st, rel, dU, dS, pp, Sg


def test_plan_cov_against_oracle(mp, ctx, cov):
    """Alg. 1 with the full covariance at the small workload (K=64, H=20,
    5 iterations, eta 0.5): the oracle composes noise, Cholesky, sampling,
    FP64 rollouts, weights and both updates in the same order."""
    st, rel, dU, dS, pp, Sg = _plan_case(mp, ctx, cov)
    assert st["rc"] == 0
    assert np.median(rel) < 1e-3
    assert dU < 0.05 * pp["sigma"][0]
    assert dS < 2e-3
    assert np.linalg.eigvalsh(Sg).min() > 0


def test_plan_cov_with_elite_set_against_oracle(mp, ctx, cov):
    """Alg. 1's elite set: only the 8 lowest costs carry weight in both
    updates (the covariance update skips the groups of samples without
    weight)."""
    st, rel, dU, dS, pp, Sg = _plan_case(mp, ctx, cov, n_elite=8)
    assert st["rc"] == 0
    assert np.median(rel) < 1e-3
    assert dU < 0.05 * pp["sigma"][0]
    assert dS < 2e-3


def test_plan_cov_with_qp_against_oracle(mp, ctx, cov):
    st, rel, dU, dS, pp, Sg = _plan_case(mp, ctx, cov, W.qp_params(1))
    assert st["rc"] == 0
    assert np.median(rel) < 1e-3
    assert dU < 0.05 * pp["sigma"][0]
    assert dS < 2e-3


def test_plan_cov_full_size_first_iteration_and_sigma(mp, ctx):
    """The workload the bench times (K = 1024, H = 64): from Sigma_0 =
    diag(sigma^2) the first iteration draws the diagonal sampler's samples
    (up to one rounding), so its mean equals the plain plan's to FP32
    rounding propagated through the rollouts; Sigma_1 is symmetric and
    positive definite, with the eps floor under its spectrum."""
    sc = W.make_scene(2)
    scene = mp.Scene(ctx, sc)
    pp = W.plan_params(2)
    cp = W.cov_params(2)
    K, H = pp["K"], pp["H"]
    n = 14 * H
    x0 = Td(W.initial_state(sc), torch.float32)
    sig = Td(pp["sigma"], torch.float32)
    nom = torch.zeros((H, 14), device=DEV)
    U1, U2 = torch.zeros((H, 14), device=DEV), torch.zeros((H, 14), device=DEV)
    S1 = torch.zeros((n, n), dtype=torch.float64, device=DEV)
    st = mp.mppi_plan_cov(ctx, scene, x0, nom, K, H, pp["lam"], sig, U1, eps=cp["eps"], Sigma_out=S1, M=1,
                          seed=pp["seed"], eta=cp["eta"])
    mp.mppi_plan(ctx, scene, x0, nom, K, H, pp["lam"], sig, U2, M=1, seed=pp["seed"], eta=cp["eta"], sync=True)
    torch.cuda.synchronize()
    d = np.abs(U1.cpu().numpy() - U2.cpu().numpy()).max()
    S = S1.cpu().numpy()
    ev = np.linalg.eigvalsh(S)
    print(f"plan cov K={K} H={H} M=1: |nu - nu_plain| {d:.2e}, Sigma eigenvalues [{ev.min():.2e}, {ev.max():.2e}]")
    assert st["rc"] == 0
    assert d < 1e-3 * pp["sigma"][0]
    assert np.array_equal(S, S.T)
    assert ev.min() > 0.5 * cp["eps"]
    scene.close()


def test_cov_entry_points_reject_bad_arguments(mp, ctx):
    sc = W.make_scene(1)
    scene = mp.Scene(ctx, sc)
    pp = W.plan_params(1)
    H = pp["H"]
    n = 14 * H
    x0 = W.initial_state(sc).astype(np.float32)
    sig = pp["sigma"].astype(np.float32)
    U = np.zeros((H, 14), np.float32)
    for kw in (dict(eps=-1.0), dict(eps=np.inf), dict(eta=0.0), dict(eta=1.5)):
        args = dict(eps=1e-4, eta=0.5)
        args.update(kw)
        with pytest.raises(mp.MppiError):
            mp.mppi_plan_cov(ctx, scene, x0, U, 8, H, pp["lam"], sig, U, eps=args["eps"], eta=args["eta"])
    with pytest.raises(mp.MppiError):  # n = 14 H above the covariance limit
        Hb = mp.COV_MAX_N // 14 + 1
        mp.mppi_plan_cov(ctx, scene, x0, np.zeros((Hb, 14), np.float32), 8, Hb, pp["lam"], sig,
                         np.zeros((Hb, 14), np.float32), eps=1e-4, eta=0.5)
    with pytest.raises(mp.MppiError):  # a host Sigma_0 with a non-finite entry
        S0 = np.eye(n)
        S0[3, 3] = np.nan
        mp.mppi_plan_cov(ctx, scene, x0, U, 8, H, pp["lam"], sig, U, eps=1e-4, eta=0.5, Sigma0=S0)
    L = np.eye(14)
    with pytest.raises(mp.MppiError):  # u_max must be positive
        mp.mppi_sample_full(ctx, np.zeros((1, 14), np.float32), L, 1, 0, 4, np.zeros((4, 1, 14), np.float32), 0.0)
    with pytest.raises(mp.MppiError):  # n above the limit
        m = mp.COV_MAX_N + 1
        mp.mppi_cholesky(ctx, np.eye(m), np.zeros((m, m)))
    scene.close()
