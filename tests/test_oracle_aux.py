"""Pins of the data generator, the warm-start network oracle, the summary statistics and the BF16 split."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.spatial.distance import pdist

import datagen
import oracle


# ---------------------------------------------------------------- generator: RK4 vs exact ZOH discretisation
def test_rk4_step_vs_exact_zoh():
    m, c, k, dt = 1.0, 0.4, 1.0, 0.1
    A = np.array([[0.0, 1.0], [-k / m, -c / m]])
    B = np.array([0.0, 1.0 / m])
    # exact zero-order-hold discretisation via the augmented matrix exponential
    M = np.zeros((3, 3)); M[:2, :2] = A * dt; M[:2, 2] = B * dt
    E = sla.expm(M)
    Phi, Gam = E[:2, :2], E[:2, 2]
    rng = np.random.default_rng(0)
    u = rng.uniform(-1, 1, size=400)
    x_rk = datagen.simulate_msd(u, m, c, k, dt)
    s = np.zeros(2)
    xs = [0.0]
    for t in range(400):
        s = Phi @ s + Gam * u[t]
        xs.append(s[0])
    # local RK4 error is O(dt^5) ~ 1e-7 per step; over 400 damped steps it stays ~1e-6
    assert np.max(np.abs(x_rk - np.array(xs))) < 5e-6
    # one step agrees with the exact step to the local error
    assert abs(x_rk[1] - xs[1]) < 1e-7 and abs(x_rk[2] - xs[2]) < 1e-7
    # for a linear ODE one RK4 step is exactly the 4th-order Taylor polynomial of exp(A dt)
    Ad = A * dt
    I2 = np.eye(2)
    Phi4 = I2 + Ad + Ad @ Ad / 2 + Ad @ Ad @ Ad / 6 + Ad @ Ad @ Ad @ Ad / 24
    Gam4 = dt * (I2 + Ad / 2 + Ad @ Ad / 6 + Ad @ Ad @ Ad / 24) @ B
    s = np.zeros(2)
    for t in range(400):
        s = Phi4 @ s + Gam4 * u[t]
        assert abs(s[0] - x_rk[t + 1]) <= 1e-13
    # static gain: constant u = 1 drives x to 1/k
    x_const = datagen.simulate_msd(np.ones(3000), 1.0, 0.4, 2.0, 0.1)
    assert x_const[-1] == pytest.approx(0.5, abs=1e-6)


def test_dataset_layout_and_standardisation():
    cfg = datagen.MSDConfig(n_train=300, n_test=50, D=5, seed=3)
    ds = datagen.make_dataset(cfg)
    assert ds.Z.shape == (300, 5) and ds.Zs.shape == (50, 5) and ds.y.shape == (300,)
    np.testing.assert_allclose(ds.Z.mean(0), 0, atol=1e-12)
    np.testing.assert_allclose(ds.Z.std(0), 1, rtol=1e-12)
    assert ds.y.mean() == pytest.approx(0, abs=1e-12) and ds.y.std() == pytest.approx(1, rel=1e-12)
    # lag structure: column j of row t is u_{t-1-j}, so column j+1 of row t+1 equals column j of row t
    np.testing.assert_array_equal(ds.Z_raw[1:, 1:], ds.Z_raw[:-1, :-1])
    rng = np.random.default_rng(3)
    u = rng.uniform(-1, 1, size=cfg.burn_in + cfg.D + 350)
    t0 = cfg.burn_in + cfg.D
    np.testing.assert_array_equal(ds.Z_raw[0], u[t0 - 1 - np.arange(5)])
    ds2 = datagen.make_dataset(cfg)
    np.testing.assert_array_equal(ds.Z, ds2.Z)


# ---------------------------------------------------------------- MLP oracle: central differences and torch autograd
def test_mlp_gradient_vs_fd_and_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    p = oracle.mlp_init(5)
    p[4096:4096 + 128] = rng.normal(0, 0.1, 128)          # non-zero biases
    X = rng.normal(size=(16, 32))
    Y = rng.normal(size=(16, 3))
    loss, g = oracle.mlp_loss_and_grad(p, X, Y)
    assert g.shape == (oracle.N_PARAMS,) == (21123,)
    h = 1e-6
    for idx in rng.choice(oracle.N_PARAMS, size=25, replace=False):
        pp = p.copy(); pp[idx] += h
        pm = p.copy(); pm[idx] -= h
        fd = (oracle.mlp_loss_and_grad(pp, X, Y)[0] - oracle.mlp_loss_and_grad(pm, X, Y)[0]) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)
    # torch autograd on the same network (float64, CPU)
    tp = torch.tensor(p, requires_grad=True)
    W1, b1, W2, b2, W3, b3 = torch.split(tp, [4096, 128, 16384, 128, 384, 3])
    gelu = torch.nn.GELU(approximate="none")
    tX = torch.tensor(X)
    out = gelu(gelu(tX @ W1.view(128, 32).T + b1) @ W2.view(128, 128).T + b2) @ W3.view(3, 128).T + b3
    tl = torch.mean((out - torch.tensor(Y)) ** 2)
    tl.backward()
    assert loss == pytest.approx(tl.item(), rel=1e-13)
    np.testing.assert_allclose(g, tp.grad.numpy(), rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(oracle.mlp_forward(p, X), out.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_mlp_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    p0 = rng.normal(size=50)
    grads = rng.normal(size=(5, 50))
    tp = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t in range(5):
        tp.grad = torch.tensor(grads[t]); opt.step()
        p, m, v = oracle.mlp_adam_step(p, grads[t], m, v, t + 1)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12)


# ---------------------------------------------------------------- summary statistics vs library routines
def test_summary_stats_vs_numpy_quantile_and_pdist():
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=600, n_test=10, D=16, seed=7))
    idx = datagen.subsample_indices(600, 256, 14)
    assert len(np.unique(idx)) == 256
    s = oracle.summary_stats(ds.Z_raw, ds.Z, ds.y_raw, idx)
    assert s.shape == (oracle.N_STATS,)
    np.testing.assert_allclose(s[:8], np.quantile(ds.Z_raw.var(0), np.arange(8) / 7), rtol=1e-14)
    d = pdist(ds.Z[idx])
    assert d.size == 256 * 255 // 2
    np.testing.assert_allclose(s[8:31], np.quantile(np.log(d), np.arange(1, 24) / 24), rtol=1e-12, atol=1e-13)
    assert s[31] == pytest.approx(math.log(np.var(ds.y_raw)), rel=1e-14)


# ---------------------------------------------------------------- BF16 split (P14)
def test_bf16_rne_vs_torch_and_split_exact():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = (rng.normal(size=20000) * 10.0 ** rng.uniform(-5, 5, size=20000)).astype(np.float32)
    x[:4] = [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 0.0]   # exact ties: round to even
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(oracle.bf16_rne(x), ref)
    hi, mid, lo = oracle.split_bf16x3(x)
    for part in (hi, mid, lo):
        np.testing.assert_array_equal(oracle.bf16_rne(part), part)
    recon = (hi.astype(np.float64) + mid.astype(np.float64) + lo.astype(np.float64))
    np.testing.assert_array_equal(recon, x.astype(np.float64))
    assert np.all(np.abs(mid) <= np.abs(hi) * 2.0 ** -8 * (1 + 1e-7))
