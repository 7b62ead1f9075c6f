"""GPU parity when the tile edge b does not divide n.

The tiled matrix then has T = ceil(n / b) tiles per dimension and rows n..Tb-1 hold an
identity block with a zero border.  The factor of the padded matrix is the factor of the
n x n covariance bordered by that identity, exactly (every entry that meets the padding is
a sum of exact zeros), so its log-determinant, the solve, the posterior and the gradient
are those of the n x n problem.  Each case is checked against the FP64 oracle on the
n x n problem, with the tolerances of the unpadded tests: 1e-10 relative in float64,
1e-6 on NLML, alpha and mean in the mixed modes (with refinement), and the padding itself
bit-exactly.
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
from tests.tiles import tiles_to_dense_lower, winv_tiles  # noqa: E402

# (n, tile, D): a ragged last tile of 44, 232 and 1 rows, a single tile larger than n,
# a tile that is not a multiple of the 64-wide blocks, and many tiles of 1 padded row
CASES = [(300, 128, 3), (1000, 256, 5), (513, 128, 4), (77, 128, 2), (250, 96, 6), (191, 16, 3)]


def _data(n, D, seed):
    rng = np.random.default_rng(seed)
    Z = rng.normal(size=(n, D))
    y = np.sin(Z[:, 0]) + 0.1 * rng.normal(size=n)
    return Z, y, rng.normal(size=(29, D))


@pytest.mark.parametrize("n,tile,D", CASES)
def test_padded_factor_is_bordered_by_identity(lib, n, tile, D):
    Z, y, _ = _data(n, D, n + tile)
    h = Hyper(1.2, 0.9, 0.05)
    L, a, f = oracle.fit(Z, y, h)
    g = _gpu_fit(lib, Z, y, h, tile)
    raw = g["K"].cpu().numpy()
    Lg = tiles_to_dense_lower(raw, n, tile, 8)
    npad = Lg.shape[0]
    assert npad == -(-n // tile) * tile
    assert np.max(np.abs(Lg[:n, :n] - L)) < 1e-10 * np.max(np.abs(L))
    assert np.all(Lg[n:, :n] == 0.0)
    np.testing.assert_array_equal(Lg[n:, n:], np.eye(npad - n))
    Wl = winv_tiles(raw, n, tile)[-1]
    r = n - (npad - tile)                      # real rows of the last tile
    np.testing.assert_array_equal(Wl[r:, r:], np.eye(tile - r))
    assert np.all(Wl[r:, :r] == 0.0)
    assert abs(g["nlml"] - f) / abs(f) < 1e-10
    assert_close(g["alpha"].cpu().numpy(), a, 1e-10)


@pytest.mark.parametrize("n,tile,D", CASES)
def test_padded_posterior_and_gradient(lib, n, tile, D):
    Z, y, Zs = _data(n, D, 2 * n + tile)
    h = Hyper(1.2, 0.9, 0.05)
    L, a, f = oracle.fit(Z, y, h)
    m = Zs.shape[0]
    g = _gpu_fit(lib, Z, y, h, tile, m=m)
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


@pytest.mark.parametrize("kernel", ["matern12", "matern52"])
def test_padded_matern_gradient(lib, kernel):
    n, tile, D = 300, 128, 3
    Z, y, Zs = _data(n, D, 5)
    h = Hyper(1.3, 0.9, 0.05, kernel)
    L, a, f = oracle.fit(Z, y, h)
    g = _gpu_fit(lib, Z, y, h, tile, m=Zs.shape[0])
    assert abs(g["nlml"] - f) / abs(f) < 1e-10
    mean, var = _gpu_predict(lib, g, Zs, h)
    assert_close(var, oracle.predict_var(Z, Zs, h, L), 1e-10)
    grad = torch.empty(3, dtype=torch.float64, device="cuda:0")
    lib.gpr_nlml_grad(g["Z"], n, D, h, g["K"], tile, "fp64", g["alpha"], (1, 1, 1), grad, g["ws"], g["wsb"])
    go = oracle.nlml_grad(Z, h, L, a)
    np.testing.assert_allclose(grad.cpu().numpy(), go, rtol=1e-9, atol=1e-9 * np.max(np.abs(go)))


# prec: (factor max-abs / max|L|, variance, gradient) bounds of the mixed modes (the
# three-product split carries about 16 significant bits per product)
MIXED_BOUNDS = {"fp32": (1e-4, 1e-4, 1e-3), "bf16x6": (1e-4, 1e-4, 1e-3), "bf16x3": (1e-3, 1e-3, 1e-2)}


@pytest.mark.parametrize("prec,tile", [("fp32", 192), ("bf16x6", 192), ("bf16x6", 256), ("bf16x3", 256)])
def test_padded_mixed_precision(lib, prec, tile):
    """Tile 192 (T = 6, last tile 40 real rows) runs the float32 products of the gradient and
    the variance in every mixed mode; tile 256 (T = 4, last tile 232 real rows) runs the
    split modes' gradient and variance (256 test points) from bfloat16 planes."""
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=1000, n_test=256, D=8, seed=3))
    h = Hyper(math.sqrt(8), 1.0, 0.01)
    L, a, f = oracle.fit(ds.Z, ds.y, h)
    f_tol, v_tol, g_tol = MIXED_BOUNDS[prec]
    T = -(-1000 // tile)
    g = _gpu_fit(lib, ds.Z, ds.y, h, tile, prec=prec, sweeps=6 if prec == "bf16x3" else 3, m=256)
    Lg = tiles_to_dense_lower(g["K"].cpu().numpy(), 1000, tile, 4)
    assert np.max(np.abs(Lg[:1000, :1000] - L)) / np.max(np.abs(L)) < f_tol
    assert np.all(Lg[1000:, :1000] == 0.0) and np.array_equal(Lg[1000:, 1000:], np.eye(T * tile - 1000))
    assert abs(g["nlml"] - f) / abs(f) < 1e-6
    assert_close(g["alpha"].cpu().numpy(), a, 1e-6)
    mean, var = _gpu_predict(lib, g, ds.Zs, h)
    assert_close(mean, oracle.predict_mean(ds.Z, ds.Zs, h, a), 1e-6)
    assert_close(var, oracle.predict_var(ds.Z, ds.Zs, h, L), v_tol)
    go = oracle.nlml_grad(ds.Z, h, L, a)
    grad = torch.empty(3, dtype=torch.float64, device="cuda:0")
    lib.gpr_nlml_grad(g["Z"], 1000, 8, h, g["K"], tile, prec, g["alpha"], (1, 1, 1), grad, g["ws"], g["wsb"])
    ge = grad.cpu().numpy()
    print(f"[padding] {prec} tile {tile}: gradient {ge} oracle {go}", flush=True)
    np.testing.assert_allclose(ge, go, rtol=g_tol, atol=g_tol * np.max(np.abs(go)))


def test_padded_optimize_matches_oracle_adam(lib):
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=200, n_test=8, D=8, seed=11))
    theta0 = [0.0, 0.0, math.log(0.1)]
    th_o, tr_o = oracle.optimize(ds.Z, ds.y, theta0, steps=4, lr=0.1)
    n, d, tile = 200, 8, 64
    dev = "cuda:0"
    Zt, yt = torch.tensor(ds.Z, device=dev), torch.tensor(ds.y, device=dev)
    K = torch.empty(lib.gpr_tiles_bytes(n, tile, "fp64"), dtype=torch.uint8, device=dev)
    wsb = lib.gpr_workspace_size(n, 0, d, tile, "fp64")
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    th, st, tr = lib.gpr_optimize(Zt, yt, n, d, tile, "fp64", theta0, (1, 1, 1), 4, 0.1, 0.9, 0.999, 1e-8, None,
                                  K, ws, wsb)
    np.testing.assert_allclose(th, th_o, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(tr, tr_o, rtol=1e-10)


def test_padded_lookahead_matches_single_stream(lib):
    """The two factorisation schedules give the same bits on a padded matrix."""
    n, tile, D = 1000, 128, 5
    Z, y, _ = _data(n, D, 17)
    h = Hyper(1.0, 1.0, 0.02)
    g1 = _gpu_fit(lib, Z, y, h, tile)
    lib.gpr_set_lookahead(False)
    try:
        g0 = _gpu_fit(lib, Z, y, h, tile)
    finally:
        lib.gpr_set_lookahead(True)
    assert torch.equal(g1["K"], g0["K"]) and torch.equal(g1["alpha"], g0["alpha"])


def test_gp_front_end_with_a_tile_that_does_not_divide_n(lib):
    from paper_2505_00136_amd.gp import GP
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=300, n_test=16, D=4, seed=12))
    gp = GP(ds.Z, ds.y, hyper=(1.2, 0.8, 0.05), tile=128)
    gp.fit()
    h = Hyper(1.2, 0.8, 0.05)
    L, a, f = oracle.fit(ds.Z, ds.y, h)
    assert float(gp.nlml().item()) == pytest.approx(f, rel=1e-10)
    mean = gp.predict(ds.Zs).cpu().numpy()
    assert_close(mean, oracle.predict_mean(ds.Z, ds.Zs, h, a), 1e-10)
