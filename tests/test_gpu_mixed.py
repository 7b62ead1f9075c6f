"""GPU parity of the mixed-precision paths against the FP64 oracle.

Bounds (stated, derived from the arithmetic):
* the float32 / bf16x6 factor has a backward error of order n u32 ||K|| (u32 = 6e-8);
  after three float64 refinement sweeps alpha and the mean are limited by
  (kappa u32)^4 plus float64 rounding, so they must match the oracle to 1e-6 (the
  target for mean and NLML) and in practice reach ~1e-10;
* the NLML takes log|K| from the mixed factor: its relative error is bounded by
  n u32 kappa-weighted terms / |NLML|, required here <= 1e-6;
* the variance uses the mixed factor without refinement (float64 sums and subtraction),
  so its error is of order kappa u32: bound 1e-4 relative (stated bound for the variance);
* bf16x3 keeps about 16 significant bits per product, so its bounds are 1e-4 (NLML)
  and 1e-3 (variance), and alpha converges only while kappa 2^-16 < 1.
"""
import math

import numpy as np
import pytest

import datagen
import oracle
from oracle import Hyper

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from tests.tiles import tiles_to_dense_lower  # noqa: E402
from tests.test_gpu_parity import _gpu_fit, _gpu_predict, _rel, lib  # noqa: E402,F401


def test_split_bf16x3_bit_exact(lib):
    rng = np.random.default_rng(5)
    x = (rng.normal(size=100003) * 10.0 ** rng.uniform(-6, 6, size=100003)).astype(np.float32)
    x[:5] = [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 0.0, -0.0]
    dev = "cuda:0"
    xt = torch.tensor(x, device=dev)
    parts = [torch.empty(x.size, dtype=torch.int16, device=dev) for _ in range(3)]
    lib.gpr_split_bf16x3(xt, x.size, *parts)
    torch.cuda.synchronize()
    ref = oracle.split_bf16x3(x)
    for got, want in zip(parts, ref):
        bits = (want.view(np.uint32) >> 16).astype(np.uint16)
        np.testing.assert_array_equal(got.cpu().numpy().view(np.uint16), bits)


@pytest.fixture(scope="module")
def dense_case():
    # a dense, moderately conditioned K (lengthscale sqrt(D)), several tiles and a ragged tile edge
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=1000, n_test=300, D=16, seed=11))
    h = Hyper(math.sqrt(16), 1.0, 0.01)
    L, a, f = oracle.fit(ds.Z, ds.y, h)
    return ds, h, L, a, f


@pytest.mark.parametrize("prec,tol_nlml,tol_var", [("fp32", 1e-6, 1e-4), ("bf16x6", 1e-6, 1e-4),
                                                   ("bf16x3", 1e-4, 1e-3)])
def test_mixed_factor_mean_var_nlml(lib, dense_case, prec, tol_nlml, tol_var):
    ds, h, L, a, f = dense_case
    tile = 200
    g = _gpu_fit(lib, ds.Z, ds.y, h, tile, prec=prec, sweeps=3, m=300)
    raw = g["K"].cpu().numpy()
    Lg = tiles_to_dense_lower(raw, 1000, tile, 4)
    ferr = np.max(np.abs(Lg - L)) / np.max(np.abs(L))
    assert ferr < (1e-4 if prec != "bf16x3" else 1e-2)
    assert abs(g["nlml"] - f) / abs(f) < tol_nlml
    mean, var = _gpu_predict(lib, g, ds.Zs, h)
    mo = oracle.predict_mean(ds.Z, ds.Zs, h, a)
    if prec != "bf16x3":
        assert _rel(g["alpha"].cpu().numpy(), a) < 1e-6
        assert _rel(mean, mo) < 1e-6
    vo = oracle.predict_var(ds.Z, ds.Zs, h, L)
    assert _rel(var, vo) < tol_var


def test_refinement_residual_decreases(lib, dense_case):
    ds, h, L, a, f = dense_case
    K = oracle.train_cov(ds.Z, h)
    errs = []
    for sweeps in range(4):
        g = _gpu_fit(lib, ds.Z, ds.y, h, 250, prec="fp32", sweeps=sweeps)
        al = g["alpha"].cpu().numpy()
        errs.append(np.linalg.norm(K @ al - ds.y) / np.linalg.norm(ds.y))
    assert all(e1 <= e0 * 1.0001 for e0, e1 in zip(errs[:-1], errs[1:]))
    assert errs[-1] < 1e-9 < errs[0]


def test_mixed_gradient_and_full_cov(lib, dense_case):
    ds, h, L, a, f = dense_case
    go = oracle.nlml_grad(ds.Z, h, L, a)
    g = _gpu_fit(lib, ds.Z, ds.y, h, 200, prec="fp32", sweeps=3, m=100)
    _, S = _gpu_predict(lib, g, ds.Zs[:100], h, full_cov=True)
    So = oracle.predict_var(ds.Z, ds.Zs[:100], h, L, full_cov=True)
    assert np.linalg.norm(S - So) / np.linalg.norm(So) < 1e-4
    grad = torch.empty(3, dtype=torch.float64, device="cuda:0")
    lib.gpr_nlml_grad(g["Z"], g["n"], g["d"], h, g["K"], 200, "fp32", g["alpha"], (1, 1, 1), grad, g["ws"], g["wsb"])
    np.testing.assert_allclose(grad.cpu().numpy(), go, rtol=1e-3, atol=1e-3 * np.max(np.abs(go)))


@pytest.mark.parametrize("prec", ["fp32", "bf16x6", "bf16x3"])
def test_mixed_optimize_follows_oracle_adam(lib, prec):
    """gpr_optimize in the mixed modes with tiles of 256 (the split modes' gradients from
    bfloat16 planes): five Adam steps stay on the oracle's float64 trajectory to the
    mixed-mode bounds -- NLML trace 1e-6 relative; theta 1e-4 absolute, since each Adam
    step moves theta by about lr in a direction set by the sign pattern of m / sqrt(v),
    which gradient errors of 1e-5 relative do not change."""
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=1024, n_test=8, D=8, seed=13))
    theta0 = [0.0, 0.0, math.log(0.1)]
    th_o, tr_o = oracle.optimize(ds.Z, ds.y, theta0, steps=5, lr=0.1)
    n, d, tile = 1024, 8, 256
    dev = "cuda:0"
    Zt, yt = torch.tensor(ds.Z, device=dev), torch.tensor(ds.y, device=dev)
    K = torch.empty(lib.gpr_tiles_bytes(n, tile, prec), dtype=torch.uint8, device=dev)
    wsb = lib.gpr_workspace_size(n, 0, d, tile, prec)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    th, st, tr = lib.gpr_optimize(Zt, yt, n, d, tile, prec, theta0, (1, 1, 1), 5, 0.1, 0.9, 0.999, 1e-8, None,
                                  K, ws, wsb)
    print(f"[mixed-optimize] {prec}: theta {np.max(np.abs(np.array(th) - th_o)):.2e}, "
          f"trace {np.max(np.abs(np.array(tr) - tr_o) / np.abs(tr_o)):.2e}", flush=True)
    np.testing.assert_allclose(tr, tr_o, rtol=1e-6)
    np.testing.assert_allclose(th, th_o, rtol=0, atol=1e-4)


@pytest.mark.parametrize("prec,m", [("bf16x6", 256), ("bf16x3", 300)])
def test_split_modes_single_tile(lib, prec, m):
    """One tile of 512 (T = 1): the split modes' inversion has no products, the trace one
    job with the alpha subtraction, the variance one block; 300 test points (not a
    multiple of 256) take the float32 substitution beside the split gradient."""
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=512, n_test=m, D=8, seed=17))
    h = Hyper(math.sqrt(8), 1.0, 0.01)
    L, a, f = oracle.fit(ds.Z, ds.y, h)
    g = _gpu_fit(lib, ds.Z, ds.y, h, 512, prec=prec, sweeps=-1, m=m)
    assert abs(g["nlml"] - f) / abs(f) < 1e-6
    assert _rel(g["alpha"].cpu().numpy(), a) < 1e-6
    mean, var = _gpu_predict(lib, g, ds.Zs, h)
    assert _rel(mean, oracle.predict_mean(ds.Z, ds.Zs, h, a)) < 1e-6
    v_tol, g_tol = (1e-3, 1e-2) if prec == "bf16x3" else (1e-4, 1e-3)
    assert _rel(var, oracle.predict_var(ds.Z, ds.Zs, h, L)) < v_tol
    grad = torch.empty(3, dtype=torch.float64, device="cuda:0")
    lib.gpr_nlml_grad(g["Z"], 512, 8, h, g["K"], 512, prec, g["alpha"], (1, 1, 1), grad, g["ws"], g["wsb"])
    go = oracle.nlml_grad(ds.Z, h, L, a)
    assert _rel(grad.cpu().numpy(), go) < g_tol


def test_split_modes_more_tiles_than_one_split_launch(lib):
    """33 tiles of 256 (n = 8448): the plane splits of a block row (up to 33 tiles) take
    two launches of at most 32 tiles each.  Against the float64 path of the same library
    (pinned to the oracle by the parity tests; the oracle itself would take a minute at
    this size) at the bf16x6 bounds: NLML and mean 1e-6, gradient 1e-3; the variance
    within 1e-5 nu absolute -- with 8 features the posterior variances here are small
    (down to 2.6e-4 nu), so relative errors are large for every mixed mode (float32
    products: 2.7e-3 relative, 8.5e-6 absolute; bf16x6 planes: 2.4e-4, 1.7e-6)."""
    n, tile, D, m = 8448, 256, 8, 256
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=n, n_test=m, D=D, seed=23))
    h = Hyper(math.sqrt(D), 1.0, 0.01)
    res = {}
    for prec in ("fp64", "fp32", "bf16x6"):
        g = _gpu_fit(lib, ds.Z, ds.y, h, tile, prec=prec, sweeps=-1, m=m)
        mean, var = _gpu_predict(lib, g, ds.Zs, h)
        grad = torch.empty(3, dtype=torch.float64, device="cuda:0")
        lib.gpr_nlml_grad(g["Z"], n, D, h, g["K"], tile, prec, g["alpha"], (1, 1, 1), grad, g["ws"], g["wsb"])
        res[prec] = dict(nlml=g["nlml"], mean=mean, var=var, grad=grad.cpu().numpy())
    r, f = res["bf16x6"], res["fp64"]
    err = _rel(r["grad"], f["grad"])
    for p in ("fp32", "bf16x6"):
        q = res[p]
        print(f"[split-33-tiles] {p}: var {_rel(q['var'], f['var']):.2e} (max abs {np.max(np.abs(q['var'] - f['var'])):.2e}, "
              f"min var {np.min(f['var']):.2e}), grad {_rel(q['grad'], f['grad']):.2e}, "
              f"mean {_rel(q['mean'], f['mean']):.2e}", flush=True)
    assert abs(r["nlml"] - f["nlml"]) / abs(f["nlml"]) < 1e-6
    assert _rel(r["mean"], f["mean"]) < 1e-6
    assert np.max(np.abs(r["var"] - f["var"])) < 1e-5 * h.signal_var
    assert err < 1e-3
