"""Covariance adaptation and full-covariance sampling -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and `bench.py`'s `cpu_baseline` leg
may import this module; the product library never loads it.

Alg. 1 draws the samples from N(nu_m, Sigma_m) and, after scoring them,
updates both moments (Eqs. mean_update and cov_update with the weights of
Eq. s_formula).  Everything here is plain FP64 NumPy.  The readings (also
listed with the design notes):

* A sampled sequence is the vector of its H x 14 joint velocities in
  step-major order: index i = 14 k + d, n = 14 H; Sigma is n x n.
* Weights s_j = exp(-(c_j - c_min) / beta) over the n_e lowest finite
  costs (zero for the others and for non-finite costs); the shift by the
  lowest cost cancels in every normalised quantity.  beta is the
  temperature of Eq. s_formula (lambda elsewhere in this code).
* Delta Sigma is the weighted scatter about nu_{m+1}, the updated mean (as
  Eq. cov_update writes it), divided by sum_j s_j (the denominator of the
  printed equation indexes s but sums s_j).
* Sigma_{m+1} = (1 - eta) Sigma_m + eta Delta Sigma + eps I.  The paper adds
  no regulariser; eps >= 0 keeps Sigma positive definite when eta = 1 and
  only a few samples carry weight (Delta Sigma has rank <= n_e).  With no
  positive weight (no finite cost) Sigma is kept, as the mean is.
* Samples: u_j = clip(nu_m + L_m z_j, -u_max, u_max) with L_m the lower
  Cholesky factor of Sigma_m and z_j the Philox normals of the diagonal
  sampler (z_j[14 k + d]); for a diagonal Sigma this is the diagonal sampler.
"""
from __future__ import annotations

import numpy as np


def weights(costs, beta, n_elite=None):
    """Normalised weights w_j = s_j / sum s (Eq. s_formula) over the n_elite
    lowest finite costs (ties: the lower index first); zeros elsewhere."""
    c = np.asarray(costs, dtype=np.float64)
    K = c.size
    fin = np.isfinite(c)
    w = np.zeros(K)
    if not fin.any():
        return w
    idx = np.nonzero(fin)[0]
    order = idx[np.lexsort((idx, c[idx]))]
    ne = K if not n_elite or n_elite >= K else int(n_elite)
    elite = order[:ne]
    cmin = c[elite].min()
    s = np.exp(-(c[elite] - cmin) / beta)
    w[elite] = s / s.sum()
    return w


def flat(U):
    """[K, H, 14] -> [K, 14 H] in step-major order."""
    U = np.asarray(U, dtype=np.float64)
    return U.reshape(U.shape[0], -1)


def mean_update(U, w, nu, eta):
    """Eq. mean_update: (1 - eta) nu + eta sum_j w_j u_j (w normalised)."""
    X = flat(U)
    nu = np.asarray(nu, dtype=np.float64).reshape(-1)
    return (1.0 - eta) * nu + eta * (np.asarray(w, dtype=np.float64) @ X)


def cov_update(U, w, nu_new, Sigma, eta, eps=0.0):
    """Eq. cov_update: (1 - eta) Sigma + eta Delta Sigma + eps I with
    Delta Sigma = sum_j w_j (u_j - nu_new)(u_j - nu_new)^T / sum_j w_j."""
    X = flat(U)
    w = np.asarray(w, dtype=np.float64)
    if not w.sum() > 0:
        return np.asarray(Sigma, dtype=np.float64).copy()  # no sample carries weight: Sigma is kept
    D = X - np.asarray(nu_new, dtype=np.float64).reshape(-1)[None, :]
    dS = (D * w[:, None]).T @ D / w.sum()
    n = X.shape[1]
    return (1.0 - eta) * np.asarray(Sigma, dtype=np.float64) + eta * dS + eps * np.eye(n)


def factor(Sigma):
    """Lower Cholesky factor L with L L^T = Sigma."""
    return np.linalg.cholesky(np.asarray(Sigma, dtype=np.float64))


def sample(nu, L, z, u_max):
    """u_j = clip(nu + L z_j, +-u_max) for z[K, n] (or [K, H, 14]); returns [K, n]."""
    Z = flat(z)
    nu = np.asarray(nu, dtype=np.float64).reshape(-1)
    return np.clip(nu[None, :] + Z @ np.asarray(L, dtype=np.float64).T, -u_max, u_max)


def diagonal_sigma(sigma, H):
    """Sigma_0 = diag(sigma^2) for sigma[14] (every step) or sigma[H, 14]."""
    s = np.asarray(sigma, dtype=np.float64)
    s = np.broadcast_to(s.reshape(-1, 14), (H, 14)).reshape(-1)
    return np.diag(s * s)


def plan(o, x0, nominal, K, H, beta, Sigma0, M, seed, eta, eps, u_max, n_elite=None, project=None):
    """Alg. 1 with the full covariance: per iteration m, draw z (the Philox
    normals of iteration m), u_j = clip(nu + L z_j), optionally smooth them
    (`project(U[K,H,14]) -> U`), roll them out, weight them, update nu then
    Sigma (nu and Sigma stay FP64 between iterations, Eqs. mean_update and
    cov_update).  Returns nu[H,14], Sigma, the last costs, weights and
    samples."""
    nu = np.asarray(nominal, dtype=np.float64).reshape(-1).copy()
    S = np.asarray(Sigma0, dtype=np.float64).copy()
    x0 = np.asarray(x0, dtype=np.float64)
    c = w = U = None
    for m in range(M):
        z = o.noise(seed, K, H, m)
        U = sample(nu, factor(S), z, u_max).reshape(K, H, 14)
        if project is not None:
            U = project(U)
        c = o.rollout_batch(x0, U)
        c = c[0] if isinstance(c, tuple) else c
        w = weights(c, beta, n_elite)
        nu = mean_update(U, w, nu, eta)
        S = cov_update(U, w, nu, S, eta, eps)
    return dict(nu=nu.reshape(H, 14), Sigma=S, costs=c, weights=w, U=U)
