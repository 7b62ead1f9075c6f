"""Pins of the oracle's Matern kernels (named by Section 6 as further kernel functions).

Each pin comes from outside the oracle's own formulas:
* Matern 1/2 on sorted 1-D inputs is the covariance of a stationary Ornstein-Uhlenbeck
  (Gauss-Markov) process, so its inverse is tridiagonal with closed-form entries;
* every half-integer Matern covariance is the Fourier cosine transform of its spectral
  density, proportional to (2 nu_m / l^2 + w^2)^-(nu_m + 1/2) in one dimension, here
  integrated numerically;
* the NLML gradient against central differences of the NLML itself.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import Hyper

SMOOTHNESS = {"matern12": 0.5, "matern32": 1.5, "matern52": 2.5}


def test_matern12_inverse_is_the_markov_precision():
    rng = np.random.default_rng(41)
    x = np.sort(rng.uniform(0.0, 5.0, size=9))[:, None]
    ell, nu = 0.7, 1.3
    K = oracle.cov(x, x, Hyper(ell, nu, 0.0, "matern12"))
    rho = np.exp(-np.diff(x[:, 0]) / ell)
    n = x.shape[0]
    Q = np.zeros((n, n))
    c = 1.0 / (1.0 - rho ** 2)
    for i in range(n):
        Q[i, i] = (c[i - 1] if i > 0 else 1.0) + (c[i] - 1.0 if i < n - 1 else 0.0)
    for i in range(n - 1):
        Q[i, i + 1] = Q[i + 1, i] = -rho[i] * c[i]
    Q /= nu
    np.testing.assert_allclose(np.linalg.inv(K), Q, rtol=1e-9, atol=1e-9 * np.max(np.abs(Q)))


@pytest.mark.parametrize("kernel", ["matern12", "matern32", "matern52"])
def test_matern_is_the_cosine_transform_of_its_spectral_density(kernel):
    ell, nu = 0.8, 1.7
    p = SMOOTHNESS[kernel] + 0.5
    a2 = 2.0 * SMOOTHNESS[kernel] / ell ** 2

    def spec(w):
        return (a2 + w * w) ** (-p)

    norm = integrate.quad(spec, 0.0, np.inf, epsabs=0, epsrel=1e-12, limit=400)[0]
    # (the slowly decaying nu_m = 1/2 spectrum defeats the oscillatory quadrature at short
    # distances; the Markov-precision pin covers them)
    r = np.array([0.0, 0.8, 1.7, 3.1] if kernel == "matern12" else [0.0, 0.05, 0.3, 0.8, 1.7, 3.1])
    x = np.stack([r, np.zeros_like(r)], axis=1)
    got = oracle.cov(x[:1], x, Hyper(ell, nu, 0.0, kernel))[0]
    for k, rk in enumerate(r):
        if rk == 0.0:
            want = nu
        else:
            want = nu * integrate.quad(spec, 0.0, np.inf, weight="cos", wvar=rk, epsabs=1e-13,
                                       limlst=200)[0] / norm
        assert abs(got[k] - want) <= 1e-8 * nu, (kernel, rk, got[k], want)


@pytest.mark.parametrize("kernel", ["matern12", "matern32", "matern52"])
def test_matern_special_values(kernel):
    """k(0) = nu, and at sqrt(2 nu_m) r / l = 1: exp(-1), 2 exp(-1), (7/3) exp(-1)."""
    ell, nu = 1.9, 0.6
    q1 = {"matern12": 1.0, "matern32": math.sqrt(3.0), "matern52": math.sqrt(5.0)}[kernel]
    r = ell / q1
    x = np.array([[0.0, 0.0], [r * 0.6, r * 0.8]])
    k = oracle.cov(x, x, Hyper(ell, nu, 0.0, kernel))
    want = {"matern12": 1.0, "matern32": 2.0, "matern52": 7.0 / 3.0}[kernel] * math.exp(-1.0) * nu
    assert k[0, 0] == pytest.approx(nu, rel=1e-15) and k[1, 1] == pytest.approx(nu, rel=1e-15)
    assert k[0, 1] == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("kernel", ["matern12", "matern32", "matern52"])
def test_matern_gradient_vs_central_differences(kernel):
    rng = np.random.default_rng(43)
    Z = rng.normal(size=(40, 3))
    y = np.sin(Z[:, 0]) + 0.1 * rng.normal(size=40)
    theta = np.array([0.2, -0.1, math.log(0.05)])
    h = Hyper.from_log(theta, kernel)
    L, a, _ = oracle.fit(Z, y, h)
    g = oracle.nlml_grad(Z, h, L, a)
    fd = np.zeros(3)
    step = 1e-5
    for k in range(3):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += step
        tm[k] -= step
        fd[k] = (oracle.fit(Z, y, Hyper.from_log(tp, kernel))[2] - oracle.fit(Z, y, Hyper.from_log(tm, kernel))[2]) / (2 * step)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-7)


def test_squared_exponential_unchanged_by_the_kernel_tag():
    rng = np.random.default_rng(44)
    Z = rng.normal(size=(7, 2))
    h = Hyper(0.9, 1.2, 0.1)
    np.testing.assert_array_equal(oracle.cov(Z, Z, h), oracle.se_cov(Z, Z, 0.9, 1.2))
    assert h.kernel == "se" and Hyper.from_log(h.log()).kernel == "se"
