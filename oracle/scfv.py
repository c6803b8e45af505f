"""SCFV global aggregation oracle -- TEST INFRASTRUCTURE ONLY (numpy, float64).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this module; the GPU path shares nothing with it.

What it computes (Sec. III-D, Eqs. (6)-(8); Sec. IV-C, Eqs. (9)-(14)): the
Scalable Compressed Fisher Vector of one image's local descriptors.

  1. PCA: every 128-D descriptor d_t becomes x_t = A (d_t - m), 32-D
     (A: 32 x 128, m: 128).
  2. A GMM of N components with weights w_i, means mu_i and diagonal
     variances var_i = sigma_i^2 (32-D each).  The posterior of component i
     for x_t is gamma_t(i) = w_i p_i(x_t) / sum_j w_j p_j(x_t) (Eq. (6); its
     printed normaliser runs over "N ... local features", which must be the
     components), p_i the diagonal Gaussian density.
  3. Gradient with respect to the means (Eq. (7)), over the K descriptors:
       g_mu_i = 1 / (K sqrt(w_i)) sum_t gamma_t(i) (x_t - mu_i) / sigma_i.
  4. Gradient with respect to the variances (the quantity of Eq. (13), with
     the normalisation of the Fisher information, sqrt(2 w_i), that Eq. (7)
     uses for the means):
       g_var_i = 1 / (K sqrt(2 w_i)) sum_t gamma_t(i) [((x_t - mu_i) / sigma_i)^2 - 1].
  5. delta(i) = the population standard deviation of the 32 entries of
     g_mu_i (Eq. (8)); components ranked by delta, descending (ties: lower
     index first); the first n are kept by a bit budget.
  6. The compressed vector: one sign bit per entry of g_mu_i (and g_var_i)
     of the kept components, bit k set when the entry is positive.

Two formulations are given, and the tests hold them to each other and to
the mathematics: `aggregate_plain` loops over descriptors and components as
Eqs. (6)-(8) read; `aggregate_matrix` is the matrix form of Sec. IV-C:
  P  = (D.*D)(1./V)^T - 2 D (M./V)^T + O ((M.*M)./V)^T       (Eq. (10), V the variances)
  Q  = the posteriors, P turned into normalised probabilities with the
       weights and the Gaussians' normalising constants
  GM = (Q^T D - (Q^T O) .* M) ./ S                             (Eq. (12), S = sqrt(V))
  GV = (Q^T (D.*D) - (Q^T D) .* 2M + (Q^T O) .* (M.*M - V)) ./ V   (Eq. (14))
(Eqs. (12) and (14) print the same letter V for the standard deviation
where Eq. (10) uses it for the variance; the reading above is the one under
which they equal Eqs. (7) and (13).)
"""
from __future__ import annotations

import numpy as np

DIM = 128
PDIM = 32


def project(desc, pca_mean, pca_matrix):
    """x_t = A (d_t - m) for every row of desc (K x 128) -> K x 32."""
    d = np.asarray(desc, dtype=np.float64)
    return (d - np.asarray(pca_mean, dtype=np.float64)[None, :]) @ np.asarray(pca_matrix, dtype=np.float64).T


def log_gauss(x, mu, var):
    """log of the diagonal Gaussian density N(x; mu, diag(var))."""
    return -0.5 * (np.sum((x - mu) ** 2 / var) + np.sum(np.log(var)) + x.size * np.log(2 * np.pi))


def posteriors_plain(X, w, mu, var):
    """gamma_t(i) (Eq. (6)), one descriptor and one component at a time
    (log-sum-exp over components for a finite ratio)."""
    K, N = X.shape[0], len(w)
    G = np.zeros((K, N))
    for t in range(K):
        lp = np.array([np.log(w[i]) + log_gauss(X[t], mu[i], var[i]) for i in range(N)])
        m = lp.max()
        e = np.exp(lp - m)
        G[t] = e / e.sum()
    return G


def aggregate_plain(X, w, mu, var):
    """(g_mu, g_var, gamma) from Eqs. (6)-(7) and the variance gradient, by
    loops over components and descriptors.  X: K x 32 projected
    descriptors; w: N; mu, var: N x 32.  K = 0 gives zeros."""
    X = np.asarray(X, dtype=np.float64)
    w, mu, var = (np.asarray(a, dtype=np.float64) for a in (w, mu, var))
    K, N = X.shape[0], len(w)
    gm = np.zeros((N, X.shape[1]))
    gv = np.zeros((N, X.shape[1]))
    if K == 0:
        return gm, gv, np.zeros((0, N))
    gamma = posteriors_plain(X, w, mu, var)
    sig = np.sqrt(var)
    for i in range(N):
        for t in range(K):
            u = (X[t] - mu[i]) / sig[i]
            gm[i] += gamma[t, i] * u
            gv[i] += gamma[t, i] * (u * u - 1.0)
        gm[i] /= K * np.sqrt(w[i])
        gv[i] /= K * np.sqrt(2.0 * w[i])
    return gm, gv, gamma


def aggregate_matrix(X, w, mu, var):
    """The same quantities by the matrix form of Sec. IV-C (Eqs. (10),
    (12), (14)) with library matrix products."""
    D = np.asarray(X, dtype=np.float64)
    w, M, V = (np.asarray(a, dtype=np.float64) for a in (w, mu, var))
    K, N = D.shape[0], len(w)
    if K == 0:
        return np.zeros((N, D.shape[1])), np.zeros((N, D.shape[1])), np.zeros((0, N))
    O = np.ones_like(D)
    P = (D * D) @ (1.0 / V).T - 2.0 * D @ (M / V).T + O @ ((M * M) / V).T      # Eq. (10)
    # normalised probability: log(w_j p_j(x_t)) = log w_j - P/2 - sum log V / 2 - const
    L = np.log(w)[None, :] - 0.5 * P - 0.5 * np.sum(np.log(V), axis=1)[None, :]
    L -= L.max(axis=1, keepdims=True)
    Q = np.exp(L)
    Q /= Q.sum(axis=1, keepdims=True)
    S = np.sqrt(V)
    QtD, QtO = Q.T @ D, Q.T @ O
    GM = (QtD - QtO * M) / S                                                     # Eq. (12)
    GV = (Q.T @ (D * D) - QtD * 2.0 * M + QtO * (M * M - V)) / V                 # Eq. (14)
    GM /= (K * np.sqrt(w))[:, None]
    GV /= (K * np.sqrt(2.0 * w))[:, None]
    return GM, GV, Q


def delta(gm):
    """Eq. (8): population standard deviation of each component's 32-D
    mean gradient."""
    g = np.asarray(gm, dtype=np.float64)
    c = g - g.mean(axis=1, keepdims=True)
    return np.sqrt((c * c).mean(axis=1))


def rank(dl):
    """Components by delta descending, ties by lower index."""
    dl = np.asarray(dl)
    return np.lexsort((np.arange(len(dl)), -dl))


def sign_bits(g):
    """One uint32 per component: bit k set when entry k is positive."""
    g = np.asarray(g)
    return ((g > 0).astype(np.uint64) << np.arange(g.shape[1], dtype=np.uint64)[None, :]).sum(axis=1).astype(
        np.uint32)


def scfv(desc, params, matrix_form=True):
    """Whole aggregation of one image's descriptors (K x 128) with stand-in
    parameters (dict: pca_mean, pca_matrix, weights, means, variances) ->
    dict(gm, gv, delta, order, bits_mu, bits_var, x)."""
    X = project(desc, params["pca_mean"], params["pca_matrix"])
    f = aggregate_matrix if matrix_form else aggregate_plain
    gm, gv, _ = f(X, params["weights"], params["means"], params["variances"])
    dl = delta(gm)
    return dict(gm=gm, gv=gv, delta=dl, order=rank(dl), bits_mu=sign_bits(gm), bits_var=sign_bits(gv), x=X)
