"""Pins of the FP64 oracle against closed forms, brute force and independent library routines.

Each test fixes one part of the oracle with something other than the oracle
itself: a closed-form posterior, a textbook loop, LAPACK/numpy eigen-solvers,
finite differences, or torch's own Adam.  A dropped term, a wrong sign, a
transposed operand or a missing factor 1/2 in the oracle fails at least one.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import Hyper

U = np.finfo(np.float64).eps


def _rand_pts(n, D, seed, scale=1.0):
    return np.random.default_rng(seed).normal(0.0, scale, size=(n, D))


# ---------------------------------------------------------------- P1: one training point
@pytest.mark.parametrize("ell,nu,s2", [(1.0, 1.0, 0.01), (0.7, 2.5, 0.3), (3.0, 0.2, 1.5)])
def test_one_point_posterior_closed_form(ell, nu, s2):
    h = Hyper(ell, nu, s2)
    z1 = np.array([[0.3, -1.2, 0.5]])
    y1 = np.array([0.8])
    zs = np.array([[0.3, -1.2, 0.5], [1.0, 0.0, -0.4], [-2.0, 1.0, 1.0]])
    a = nu + s2
    r2 = np.sum((zs - z1) ** 2, axis=1)
    L, alpha, f = oracle.fit(z1, y1, h)
    assert alpha[0] == pytest.approx(y1[0] / a, rel=1e-15)
    mean = oracle.predict_mean(z1, zs, h, alpha)
    np.testing.assert_allclose(mean, nu * np.exp(-r2 / (2 * ell ** 2)) * y1[0] / a, rtol=1e-14)
    var = oracle.predict_var(z1, zs, h, L)
    np.testing.assert_allclose(var, nu - nu ** 2 * np.exp(-r2 / ell ** 2) / a, rtol=1e-13)
    assert var[0] == pytest.approx(nu * s2 / a, rel=1e-13)
    nl = 0.5 * math.log(a) + y1[0] ** 2 / (2 * a) + 0.5 * math.log(2 * math.pi)
    assert f == pytest.approx(nl, rel=1e-15)
    g = oracle.nlml_grad(z1, h, L, alpha)
    assert g[0] == pytest.approx(0.0, abs=1e-15)
    assert g[1] == pytest.approx(nu / (2 * a) - y1[0] ** 2 * nu / (2 * a * a), rel=1e-13)
    assert g[2] == pytest.approx(s2 / (2 * a) - y1[0] ** 2 * s2 / (2 * a * a), rel=1e-13)


# ---------------------------------------------------------------- P2: two training points
def test_two_point_closed_form():
    ell, nu, s2 = 1.3, 1.7, 0.2
    h = Hyper(ell, nu, s2)
    Z = np.array([[0.0, 1.0], [0.5, -0.25]])
    y = np.array([1.1, -0.4])
    r2 = 0.5 ** 2 + 1.25 ** 2
    a, b = nu + s2, nu * math.exp(-r2 / (2 * ell ** 2))
    L, alpha, f = oracle.fit(Z, y, h)
    Lx = np.array([[math.sqrt(a), 0.0], [b / math.sqrt(a), math.sqrt(a - b * b / a)]])
    np.testing.assert_allclose(L, Lx, rtol=1e-15, atol=1e-16)
    det = a * a - b * b
    Kinv = np.array([[a, -b], [-b, a]]) / det
    np.testing.assert_allclose(alpha, Kinv @ y, rtol=1e-14)
    nl = 0.5 * math.log(det) + 0.5 * y @ Kinv @ y + math.log(2 * math.pi)
    assert f == pytest.approx(nl, rel=1e-15)
    # gradient from the 2x2 closed form: dK/dlog l = [[0, b r2/l^2],[., 0]], dK/dlog nu = [[nu, b],[b, nu]]
    W = Kinv - np.outer(Kinv @ y, Kinv @ y)
    g = oracle.nlml_grad(Z, h, L, alpha)
    assert g[0] == pytest.approx(W[0, 1] * b * r2 / ell ** 2, rel=1e-13)
    assert g[1] == pytest.approx(0.5 * (W[0, 0] * nu + W[1, 1] * nu + 2 * W[0, 1] * b), rel=1e-13)
    assert g[2] == pytest.approx(0.5 * s2 * (W[0, 0] + W[1, 1]), rel=1e-13)


# ---------------------------------------------------------------- P3: factor
def _textbook_cholesky(A):
    n = len(A)
    L = [[0.0] * n for _ in range(n)]
    for j in range(n):
        s = A[j][j] - sum(L[j][k] ** 2 for k in range(j))
        if not s > 0:   # a non-positive or NaN pivot
            return None, j + 1
        L[j][j] = math.sqrt(s)
        for i in range(j + 1, n):
            L[i][j] = (A[i][j] - sum(L[i][k] * L[j][k] for k in range(j))) / L[j][j]
    return np.array(L), 0


def test_cholesky_vs_textbook_and_reconstruction():
    Z = _rand_pts(7, 3, 1)
    K = oracle.train_cov(Z, Hyper(0.9, 1.2, 0.05))
    L = oracle.cholesky(K)
    Lb, info = _textbook_cholesky(K.tolist())
    assert info == 0
    np.testing.assert_allclose(L, Lb, rtol=1e-13, atol=1e-15)
    assert np.all(np.triu(L, 1) == 0) and np.all(np.diag(L) > 0)
    Z = _rand_pts(300, 8, 2)
    K = oracle.train_cov(Z, Hyper(1.0, 1.0, 0.01))
    L = oracle.cholesky(K)
    assert np.linalg.norm(K - L @ L.T) / np.linalg.norm(K) <= 4 * 300 * U


def test_potrf_info_matches_textbook_first_bad_pivot():
    Z = _rand_pts(9, 2, 3)
    K = oracle.train_cov(Z, Hyper(1.0, 1.0, 0.1))
    for col in (1, 4, 9):
        Kb = K.copy()
        Kb[col - 1, col - 1] = -3.0
        _, info_tb = _textbook_cholesky(Kb.tolist())
        assert info_tb == col
        assert oracle.potrf_info(Kb) == col
    assert oracle.potrf_info(K) == 0


def test_potrf_info_nan_input_is_its_column():
    """A NaN training input makes its row and column of K NaN: the pivots before it stay
    finite and its own pivot fails the positivity test, as in the textbook loop."""
    for row in (0, 3, 8):
        Z = _rand_pts(9, 2, 4)
        Z[row, 0] = float("nan")
        K = oracle.train_cov(Z, Hyper(1.0, 1.0, 0.1))
        _, info_tb = _textbook_cholesky(K.tolist())
        assert info_tb == row + 1
        assert oracle.potrf_info(K) == row + 1


# ---------------------------------------------------------------- P4, P5: log-det and alpha
def test_logdet_vs_eigen_and_det():
    for n in (3, 8):
        Z = _rand_pts(n, 4, 10 + n)
        h = Hyper(1.1, 0.8, 0.05)
        K = oracle.train_cov(Z, h)
        y = np.random.default_rng(n).normal(size=n)
        L, a, f = oracle.fit(Z, y, h)
        logdet = 2 * (f - 0.5 * y @ a - 0.5 * n * math.log(2 * math.pi))
        assert logdet == pytest.approx(np.sum(np.log(np.linalg.eigvalsh(K))), rel=1e-12, abs=1e-12)
        assert logdet == pytest.approx(math.log(np.linalg.det(K)), rel=1e-12, abs=1e-12)


def test_alpha_vs_inverse():
    n = 64
    Z = _rand_pts(n, 3, 5)
    h = Hyper(0.8, 1.5, 0.02)
    K = oracle.train_cov(Z, h)
    y = np.random.default_rng(6).normal(size=n)
    L, a, _ = oracle.fit(Z, y, h)
    np.testing.assert_allclose(a, np.linalg.inv(K) @ y, rtol=1e-9, atol=1e-11)
    assert np.linalg.norm(K @ a - y) / (np.linalg.norm(K, 2) * np.linalg.norm(a)) <= 10 * n * U


# ---------------------------------------------------------------- mean and covariance by brute force
def test_mean_and_cov_vs_brute_force():
    Z = _rand_pts(40, 3, 7)
    Zs = _rand_pts(25, 3, 8)
    h = Hyper(1.2, 0.9, 0.04)
    y = np.random.default_rng(9).normal(size=40)
    K = oracle.train_cov(Z, h)
    Kinv = np.linalg.inv(K)
    r2 = ((Zs[:, None, :] - Z[None, :, :]) ** 2).sum(-1)
    Ksz = h.signal_var * np.exp(-r2 / (2 * h.lengthscale ** 2))
    r2ss = ((Zs[:, None, :] - Zs[None, :, :]) ** 2).sum(-1)
    Kss = h.signal_var * np.exp(-r2ss / (2 * h.lengthscale ** 2))
    L, a, _ = oracle.fit(Z, y, h)
    np.testing.assert_allclose(oracle.predict_mean(Z, Zs, h, a), Ksz @ Kinv @ y, rtol=1e-9, atol=1e-12)
    S = oracle.predict_var(Z, Zs, h, L, full_cov=True)
    np.testing.assert_allclose(S, Kss - Ksz @ Kinv @ Ksz.T, rtol=1e-8, atol=1e-12)
    v = oracle.predict_var(Z, Zs, h, L)
    np.testing.assert_allclose(v, np.diag(S), rtol=1e-12, atol=1e-14)
    vn = oracle.predict_var(Z, Zs, h, L, add_noise=True)
    np.testing.assert_allclose(vn - v, h.noise_var, rtol=1e-12)
    Sn = oracle.predict_var(Z, Zs, h, L, full_cov=True, add_noise=True)
    np.testing.assert_allclose(np.diag(Sn) - np.diag(S), h.noise_var, rtol=1e-12)


# ---------------------------------------------------------------- P6: nearly diagonal K
def test_nearly_diagonal_closed_form():
    # D = 128 standardised features with l = 1: off-diagonal entries ~ exp(-128) ~ 1e-56
    rng = np.random.default_rng(11)
    n, D = 256, 128
    Z = rng.normal(size=(n, D))
    y = rng.normal(size=n)
    h = Hyper(1.0, 1.0, 0.01)
    L, a, f = oracle.fit(Z, y, h)
    c = h.signal_var + h.noise_var
    np.testing.assert_allclose(a, y / c, rtol=1e-14)
    assert f == pytest.approx(0.5 * n * math.log(c) + y @ y / (2 * c) + 0.5 * n * math.log(2 * math.pi), rel=1e-14)
    Zs = rng.normal(size=(32, D))
    np.testing.assert_allclose(oracle.predict_var(Z, Zs, h, L), h.signal_var, rtol=1e-14)
    np.testing.assert_allclose(oracle.predict_mean(Z, Zs, h, a), 0.0, atol=1e-14)


# ---------------------------------------------------------------- P7: rank-one limit (Sherman-Morrison)
def test_rank_one_limit_sherman_morrison():
    rng = np.random.default_rng(12)
    n = 200
    Z = rng.normal(size=(n, 4))
    y = rng.normal(size=n)
    nu, s2 = 1.3, 0.05
    h = Hyper(1e9, nu, s2)
    L, a, f = oracle.fit(Z, y, h)
    c = s2 + n * nu
    a_x = (y - nu * y.sum() / c) / s2
    np.testing.assert_allclose(a, a_x, rtol=1e-10 * (1 + n * nu / s2) / 100)
    logdet = (n - 1) * math.log(s2) + math.log(c)
    assert f == pytest.approx(0.5 * y @ a_x + 0.5 * logdet + 0.5 * n * math.log(2 * math.pi), rel=1e-12)
    Zs = rng.normal(size=(5, 4))
    np.testing.assert_allclose(oracle.predict_mean(Z, Zs, h, a), nu * y.sum() / c, rtol=1e-10)
    g = oracle.nlml_grad(Z, h, L, a)
    trKinv = (n - n * nu / c) / s2
    assert g[1] == pytest.approx(0.5 * (nu * n / c) - 0.5 * nu * (y.sum() / c) ** 2, rel=1e-8)
    assert g[2] == pytest.approx(0.5 * s2 * (trKinv - a_x @ a_x), rel=1e-8)
    assert abs(g[0]) < 1e-9


# ---------------------------------------------------------------- P10: finite differences
@pytest.mark.parametrize("theta", [(0.0, 0.0, math.log(0.1)), (0.4, -0.3, math.log(0.02))])
def test_gradient_vs_central_differences(theta):
    rng = np.random.default_rng(13)
    Z = rng.normal(size=(120, 3))
    y = np.sin(Z[:, 0]) + 0.1 * rng.normal(size=120)
    hstep = 1e-5

    def f(t):
        return oracle.fit(Z, y, Hyper.from_log(t))[2]

    h = Hyper.from_log(theta)
    L, a, _ = oracle.fit(Z, y, h)
    g = oracle.nlml_grad(Z, h, L, a)
    for k in range(3):
        tp = np.array(theta, dtype=float); tp[k] += hstep
        tm = np.array(theta, dtype=float); tm[k] -= hstep
        fd = (f(tp) - f(tm)) / (2 * hstep)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-6)
    gm = oracle.nlml_grad(Z, h, L, a, trainable=(1, 0, 1))
    assert gm[1] == 0.0 and gm[0] == g[0] and gm[2] == g[2]


# ---------------------------------------------------------------- P11: Adam
def test_adam_first_step_and_torch():
    torch = pytest.importorskip("torch")
    g = np.array([3.0, -0.02, 1e3])
    th, m, v = oracle.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    np.testing.assert_allclose(th, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-15)
    rng = np.random.default_rng(14)
    grads = rng.normal(size=(10, 3))
    p = torch.zeros(3, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.05, betas=(0.9, 0.999), eps=1e-8)
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 11):
        opt.zero_grad()
        p.grad = torch.tensor(grads[t - 1], dtype=torch.float64)
        opt.step()
        th, m, v = oracle.adam_step(th, grads[t - 1], m, v, t, lr=0.05)
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-12, atol=1e-15)
    th2, _, _ = oracle.adam_step(np.ones(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1, trainable=(1, 0, 1))
    assert th2[1] == 1.0


def test_optimize_trace_semantics():
    rng = np.random.default_rng(15)
    Z = rng.normal(size=(60, 2))
    y = np.cos(Z[:, 1]) + 0.1 * rng.normal(size=60)
    theta, tr = oracle.optimize(Z, y, (0.0, 0.0, math.log(0.1)), steps=5, lr=0.1)
    assert tr.shape == (6,)
    assert tr[0] == pytest.approx(oracle.fit(Z, y, Hyper(1.0, 1.0, 0.1))[2], rel=1e-15)
    assert tr[-1] == pytest.approx(oracle.fit(Z, y, Hyper.from_log(theta))[2], rel=1e-15)
    assert tr[-1] < tr[0]


def test_optimize_trajectory_vs_torch_adam():
    """oracle.optimize takes each gradient at the current theta: its trajectory equals
    torch.optim.Adam on the log-hyperparameters driven by the oracle's gradient at the
    parameters torch holds at each step (a gradient at a stale theta, or an update
    applied before the NLML is recorded, would depart from it after the first step)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(16)
    Z = rng.normal(size=(80, 3))
    y = np.sin(Z[:, 0]) - 0.5 * Z[:, 2] + 0.1 * rng.normal(size=80)
    theta0 = (0.3, -0.2, math.log(0.05))
    steps, lr = 3, 0.2
    theta, tr = oracle.optimize(Z, y, theta0, steps=steps, lr=lr)
    p = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    want = []
    for _ in range(steps):
        h = Hyper.from_log(p.detach().numpy())
        L, a, f = oracle.fit(Z, y, h)
        want.append(f)
        opt.zero_grad()
        p.grad = torch.tensor(oracle.nlml_grad(Z, h, L, a), dtype=torch.float64)
        opt.step()
    want.append(oracle.fit(Z, y, Hyper.from_log(p.detach().numpy()))[2])
    np.testing.assert_allclose(theta, p.detach().numpy(), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(tr, want, rtol=1e-13)
    # the steps really move theta (so a stale gradient would be seen)
    assert np.all(np.abs(theta - np.array(theta0)) > 0.1)


# ---------------------------------------------------------------- P15, P16: variance bounds, interpolation
def test_variance_bounds_and_interpolation():
    rng = np.random.default_rng(16)
    Z = rng.normal(size=(80, 3))
    y = rng.normal(size=80)
    h = Hyper(0.9, 1.4, 0.03)
    L, a, _ = oracle.fit(Z, y, h)
    v = oracle.predict_var(Z, rng.normal(size=(50, 3)), h, L)
    assert np.all(v >= -1e-12) and np.all(v <= h.signal_var * (1 + 1e-15))
    vt = oracle.predict_var(Z, Z[:10], h, L)
    assert np.all(vt <= h.signal_var * h.noise_var / (h.signal_var + h.noise_var) * (1 + 1e-9))
    # at training inputs K_f alpha = (K - s2 I) alpha = y - s2 alpha exactly, so mu -> y as s2 -> 0
    prev = None
    for s2 in (1e-2, 1e-4, 1e-6):
        hh = Hyper(0.9, 1.4, s2)
        L, a, _ = oracle.fit(Z, y, hh)
        mu = oracle.predict_mean(Z, Z, hh, a)
        np.testing.assert_allclose(mu + s2 * a, y, rtol=0, atol=1e-9)
        err = np.max(np.abs(mu - y))
        if prev is not None:
            assert err < prev
        prev = err


# ---------------------------------------------------------------- Fig. 1 task census
def test_tile_task_census_fig1():
    assert oracle.tile_task_census(1, 0) == dict(potrf=1, trsm=0, syrk=0, gemm=0)
    assert oracle.tile_task_census(4, 0) == dict(potrf=1, trsm=3, syrk=3, gemm=3)
    assert oracle.tile_task_census(16, 0) == dict(potrf=1, trsm=15, syrk=15, gemm=105)
    for T in (1, 4, 16, 32):
        tot = oracle.tile_task_census(T)
        assert tot == dict(potrf=T, trsm=math.comb(T, 2), syrk=math.comb(T, 2), gemm=math.comb(T, 3))
    assert sum(oracle.tile_task_census(32).values()) == 5984
