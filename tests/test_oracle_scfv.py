"""Pins for the SCFV aggregation oracle (Sec. III-D, Eqs. (6)-(8); Sec. IV-C,
Eqs. (9)-(14)), against what the mathematics fixes: the posteriors against a
library Gaussian density, both gradients against central finite differences
of the mean log-likelihood (the Fisher vector is its gradient, scaled by the
inverse square root of the Fisher information), the one-component closed
form, delta against a library standard deviation, and the plain and matrix
formulations against each other."""
import numpy as np
import pytest
from scipy import stats

from oracle import scfv


def _gmm(rng, N=7, d=32):
    w = rng.uniform(0.5, 2.0, N)
    w /= w.sum()
    mu = rng.normal(0, 0.3, (N, d))
    var = rng.uniform(0.02, 0.2, (N, d))
    return w, mu, var


def _loglik(X, w, mu, var):
    """Mean over descriptors of log sum_j w_j p_j(x_t), with scipy's density."""
    tot = 0.0
    for x in X:
        tot += np.log(sum(w[j] * stats.multivariate_normal.pdf(x, mu[j], np.diag(var[j])) for j in range(len(w))))
    return tot / len(X)


def test_posteriors_against_library_density():
    rng = np.random.default_rng(0)
    w, mu, var = _gmm(rng)
    X = mu[rng.integers(0, len(w), 12)] + rng.normal(0, 0.2, (12, 32))
    G = scfv.posteriors_plain(X, w, mu, var)
    for t, x in enumerate(X):
        p = np.array([w[j] * stats.multivariate_normal.pdf(x, mu[j], np.diag(var[j])) for j in range(len(w))])
        np.testing.assert_allclose(G[t], p / p.sum(), rtol=1e-9, atol=1e-300)
    np.testing.assert_allclose(G.sum(axis=1), 1.0, atol=1e-12)
    assert G.min() >= 0


@pytest.mark.parametrize("seed", [1, 2])
def test_mean_gradient_is_scaled_loglik_gradient(seed):
    """g_mu_ik = sigma_ik / sqrt(w_i) * d/d mu_ik of the mean log-likelihood."""
    rng = np.random.default_rng(seed)
    w, mu, var = _gmm(rng, N=4, d=32)
    X = mu[rng.integers(0, 4, 9)] + rng.normal(0, 0.25, (9, 32))
    gm, _, _ = scfv.aggregate_plain(X, w, mu, var)
    h = 1e-6
    for i, k in [(0, 0), (1, 5), (3, 31), (2, 17)]:
        a, b = mu.copy(), mu.copy()
        a[i, k] += h
        b[i, k] -= h
        fd = (_loglik(X, w, a, var) - _loglik(X, w, b, var)) / (2 * h)
        np.testing.assert_allclose(gm[i, k], fd * np.sqrt(var[i, k]) / np.sqrt(w[i]), rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("seed", [3, 4])
def test_variance_gradient_is_scaled_loglik_gradient(seed):
    """g_var_ik = sigma_ik / sqrt(2 w_i) * d/d sigma_ik of the mean
    log-likelihood."""
    rng = np.random.default_rng(seed)
    w, mu, var = _gmm(rng, N=4, d=32)
    X = mu[rng.integers(0, 4, 9)] + rng.normal(0, 0.25, (9, 32))
    _, gv, _ = scfv.aggregate_plain(X, w, mu, var)
    h = 1e-6
    for i, k in [(0, 3), (1, 0), (3, 30), (2, 12)]:
        s = np.sqrt(var[i, k])
        a, b = var.copy(), var.copy()
        a[i, k] = (s + h) ** 2
        b[i, k] = (s - h) ** 2
        fd = (_loglik(X, w, mu, a) - _loglik(X, w, mu, b)) / (2 * h)
        np.testing.assert_allclose(gv[i, k], fd * s / np.sqrt(2 * w[i]), rtol=1e-6, atol=1e-9)


def test_one_component_closed_form():
    """One component (w = 1): every posterior is 1, so g_mu is the mean
    standardised offset and g_var the standardised second moment less one,
    over sqrt(2)."""
    rng = np.random.default_rng(5)
    mu = rng.normal(0, 0.3, (1, 32))
    var = rng.uniform(0.05, 0.2, (1, 32))
    X = rng.normal(0, 0.4, (20, 32))
    for f in (scfv.aggregate_plain, scfv.aggregate_matrix):
        gm, gv, G = f(X, np.ones(1), mu, var)
        np.testing.assert_allclose(G, 1.0)
        u = (X - mu) / np.sqrt(var)
        np.testing.assert_allclose(gm[0], u.mean(axis=0), rtol=1e-12)
        np.testing.assert_allclose(gv[0], ((u * u).mean(axis=0) - 1) / np.sqrt(2), rtol=1e-10, atol=1e-14)


def test_matrix_form_equals_plain_form():
    rng = np.random.default_rng(6)
    w, mu, var = _gmm(rng, N=16)
    X = mu[rng.integers(0, 16, 40)] + rng.normal(0, 0.3, (40, 32))
    a = scfv.aggregate_plain(X, w, mu, var)
    b = scfv.aggregate_matrix(X, w, mu, var)
    for u, v in zip(a, b):
        np.testing.assert_allclose(u, v, rtol=1e-9, atol=1e-12)


def test_empty_image_gives_zeros():
    rng = np.random.default_rng(7)
    w, mu, var = _gmm(rng)
    for f in (scfv.aggregate_plain, scfv.aggregate_matrix):
        gm, gv, _ = f(np.zeros((0, 32)), w, mu, var)
        assert not gm.any() and not gv.any()


def test_delta_rank_and_bits():
    rng = np.random.default_rng(8)
    g = rng.normal(size=(10, 32))
    np.testing.assert_allclose(scfv.delta(g), np.std(g, axis=1), rtol=1e-12)
    dl = np.array([0.5, 0.7, 0.5, 0.1, 0.7])
    np.testing.assert_array_equal(scfv.rank(dl), [1, 4, 0, 2, 3])
    v = np.zeros((2, 32))
    v[0, [0, 3, 31]] = 1.0
    v[1, 1] = -1.0
    v[1, 2] = 0.0
    np.testing.assert_array_equal(scfv.sign_bits(v), [(1 | 8 | (1 << 31)), 0])


def test_projection():
    rng = np.random.default_rng(9)
    m = rng.uniform(0, 0.2, 128)
    A = np.linalg.qr(rng.normal(size=(128, 32)))[0].T
    d = rng.uniform(0, 0.2, (5, 128))
    np.testing.assert_allclose(scfv.project(m[None, :], m, A), 0.0, atol=1e-15)
    np.testing.assert_allclose(scfv.project(d, m, A), (d - m) @ A.T, rtol=1e-12)
