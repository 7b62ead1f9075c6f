"""GPU parity of the Matern kernels (1/2, 3/2, 5/2) against the FP64 oracle.

The whole path runs with the selected covariance function: assembly, factorisation,
alpha, NLML, mean, variance and full covariance, the gradient (whose fused reduction
weights K^{-1} with the Matern value and its length-scale derivative), Adam, and the
float32 path with refinement.  Tolerances as for the squared exponential: 1e-10
relative in float64, 1e-9 on the gradient.
"""
import math

import numpy as np
import pytest

import datagen
import oracle
from oracle import Hyper

from tests.checks import assert_close, assert_elementwise  # noqa: E402,F401

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from tests.test_gpu_parity import _gpu_fit, _gpu_predict, _rel, lib  # noqa: E402,F401

MATERN = ["matern12", "matern32", "matern52"]


@pytest.mark.parametrize("kernel", MATERN)
@pytest.mark.parametrize("n,tile,D", [(300, 100, 3), (512, 128, 8)])
def test_matern_fit_predict_gradient(lib, kernel, n, tile, D):
    rng = np.random.default_rng(n + len(kernel))
    Z = rng.normal(size=(n, D))
    y = np.sin(Z[:, 0]) + 0.1 * rng.normal(size=n)
    Zs = rng.normal(size=(33, D))
    h = Hyper(1.3, 0.9, 0.05, kernel)
    L, a, f = oracle.fit(Z, y, h)
    g = _gpu_fit(lib, Z, y, h, tile, m=33)
    assert abs(g["nlml"] - f) / abs(f) < 1e-10
    assert_close(g["alpha"].cpu().numpy(), a, 1e-10)
    mean, var = _gpu_predict(lib, g, Zs, h)
    assert_close(mean, oracle.predict_mean(Z, Zs, h, a), 1e-10)
    assert_close(var, oracle.predict_var(Z, Zs, h, L), 1e-10)
    _, S = _gpu_predict(lib, g, Zs, h, full_cov=True)
    So = oracle.predict_var(Z, Zs, h, L, full_cov=True)
    assert np.max(np.abs(S - So)) < 1e-10 * max(1.0, np.max(np.abs(So)))
    grad = torch.empty(3, dtype=torch.float64, device="cuda:0")
    lib.gpr_nlml_grad(g["Z"], n, D, h, g["K"], tile, "fp64", g["alpha"], (1, 1, 1), grad, g["ws"], g["wsb"])
    go = oracle.nlml_grad(Z, h, L, a)
    np.testing.assert_allclose(grad.cpu().numpy(), go, rtol=1e-9, atol=1e-9 * np.max(np.abs(go)))


@pytest.mark.parametrize("kernel", MATERN)
def test_matern_optimize_matches_oracle_adam(lib, kernel):
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=192, n_test=8, D=8, seed=7))
    theta0 = [0.0, 0.0, math.log(0.1)]
    th_o, tr_o = oracle.optimize(ds.Z, ds.y, theta0, steps=4, lr=0.1, kernel=kernel)
    n, d, tile = 192, 8, 64
    dev = "cuda:0"
    Zt, yt = torch.tensor(ds.Z, device=dev), torch.tensor(ds.y, device=dev)
    K = torch.empty(lib.gpr_tiles_bytes(n, tile, "fp64"), dtype=torch.uint8, device=dev)
    wsb = lib.gpr_workspace_size(n, 0, d, tile, "fp64")
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    th, st, tr = lib.gpr_optimize(Zt, yt, n, d, tile, "fp64", theta0, (1, 1, 1), 4, 0.1, 0.9, 0.999, 1e-8, None,
                                  K, ws, wsb, kernel=kernel)
    np.testing.assert_allclose(th, th_o, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(tr, tr_o, rtol=1e-10)


def test_matern_float32_path_with_refinement(lib):
    rng = np.random.default_rng(77)
    n, tile, D = 1024, 256, 6
    Z = rng.normal(size=(n, D))
    y = np.sin(Z[:, 0]) + 0.1 * rng.normal(size=n)
    Zs = rng.normal(size=(64, D))
    h = Hyper(1.5, 1.0, 0.02, "matern52")
    L, a, f = oracle.fit(Z, y, h)
    g = _gpu_fit(lib, Z, y, h, tile, prec="fp32", sweeps=3, m=64)
    assert abs(g["nlml"] - f) / abs(f) < 1e-6
    mean, var = _gpu_predict(lib, g, Zs, h)
    assert_close(mean, oracle.predict_mean(Z, Zs, h, a), 1e-6)
    assert np.max(np.abs(var - oracle.predict_var(Z, Zs, h, L))) < 1e-4


@pytest.mark.parametrize("kernel", ["matern12", "matern32", "matern52"])
@pytest.mark.parametrize("prec", ["bf16x6", "bf16x3"])
def test_matern_split_modes_gradient_and_variance(lib, kernel, prec):
    """Tiles of 256 and 256 test points: the split modes run the inversion, the trace
    products (whose Matern weights walk the accumulators through LDS) and the variance's
    substitution from bfloat16 planes.  Bounds as for the squared exponential: mean and
    NLML 1e-6 after the default sweeps; variance 1e-4 (bf16x3 1e-3); gradient 1e-3
    (bf16x3 1e-2), normwise."""
    rng = np.random.default_rng(91)
    n, tile, D, m = 1024, 256, 6, 256
    Z = rng.normal(size=(n, D))
    y = np.sin(Z[:, 0]) + 0.1 * rng.normal(size=n)
    Zs = rng.normal(size=(m, D))
    h = Hyper(1.5, 1.0, 0.02, kernel)
    L, a, f = oracle.fit(Z, y, h)
    g = _gpu_fit(lib, Z, y, h, tile, prec=prec, sweeps=6 if prec == "bf16x3" else 3, m=m)
    assert abs(g["nlml"] - f) / abs(f) < 1e-6
    mean, var = _gpu_predict(lib, g, Zs, h)
    assert_close(mean, oracle.predict_mean(Z, Zs, h, a), 1e-6)
    v_tol, g_tol = (1e-3, 1e-2) if prec == "bf16x3" else (1e-4, 1e-3)
    assert np.max(np.abs(var - oracle.predict_var(Z, Zs, h, L))) < v_tol
    grad = torch.empty(3, dtype=torch.float64, device="cuda:0")
    lib.gpr_nlml_grad(g["Z"], n, D, h, g["K"], tile, prec, g["alpha"], (1, 1, 1), grad, g["ws"], g["wsb"])
    go = oracle.nlml_grad(Z, h, L, a)
    ge = grad.cpu().numpy()
    err = np.linalg.norm(ge - go) / np.linalg.norm(go)
    print(f"[matern-split] {kernel} {prec}: gradient {err:.2e}", flush=True)
    assert err < g_tol


def test_gp_front_end_with_a_matern_kernel(lib):
    from paper_2505_00136_amd.gp import GP
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=256, n_test=16, D=4, seed=8))
    gp = GP(ds.Z, ds.y, hyper=(1.2, 0.8, 0.05), tile=64, kernel="matern32")
    gp.fit()
    h = Hyper(1.2, 0.8, 0.05, "matern32")
    L, a, f = oracle.fit(ds.Z, ds.y, h)
    assert float(gp.nlml().item()) == pytest.approx(f, rel=1e-10)
    mean = gp.predict(ds.Zs).cpu().numpy()
    assert_close(mean, oracle.predict_mean(ds.Z, ds.Zs, h, a), 1e-10)
