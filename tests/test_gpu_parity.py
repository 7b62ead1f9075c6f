"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Float64 tolerances: the paper's own arithmetic is double precision, so the
factor, alpha, mean, variance and NLML must match the LAPACK-based oracle to
within rounding amplified by the conditioning of K: relative 1e-10 on the
quantities of Eq. 3-5 for the well-conditioned workloads used here (kappa <= 1e3),
normwise (||a - b|| / ||b||), and 1e-9 per entry (tests/checks.py: each entry against
max(|b_i|, 1e-3 max|b|)).
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

from tests.tiles import tiles_to_dense_lower, winv_tiles  # noqa: E402


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_00136_amd import _lib
    _lib.load()
    return _lib


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _gpu_fit(lib, Z, y, h, tile, prec="fp64", sweeps=0, m=0):
    dev = "cuda:0"
    n, d = Z.shape
    Zt = torch.tensor(Z, device=dev)
    yt = torch.tensor(y, device=dev)
    K = torch.empty(lib.gpr_tiles_bytes(n, tile, prec), dtype=torch.uint8, device=dev)
    wsb = lib.gpr_workspace_size(n, m, d, tile, prec)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    lib.gpr_assemble(Zt, n, d, h, tile, prec, K)
    info = lib.gpr_cholesky(K, n, tile, prec, ws, wsb)
    assert info == 0
    alpha = torch.empty(n, dtype=torch.float64, device=dev)
    lib.gpr_solve(K, Zt, n, d, h, tile, prec, yt, alpha, sweeps, ws, wsb)
    nl = torch.empty(1, dtype=torch.float64, device=dev)
    lib.gpr_nlml(K, n, tile, prec, yt, alpha, nl)
    torch.cuda.synchronize()
    return dict(Z=Zt, y=yt, K=K, ws=ws, wsb=wsb, alpha=alpha, nlml=float(nl.item()), n=n, d=d, tile=tile, prec=prec)


def _gpu_predict(lib, f, Zs, h, full_cov=False, add_noise=False):
    dev = "cuda:0"
    m = Zs.shape[0]
    Zst = torch.tensor(Zs, device=dev)
    wsb = lib.gpr_workspace_size(f["n"], m, f["d"], f["tile"], f["prec"])
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    mean = torch.empty(m, dtype=torch.float64, device=dev)
    lib.gpr_predict(f["Z"], f["n"], Zst, m, f["d"], h, f["alpha"], mean, ws, wsb)
    out = torch.empty((m, m) if full_cov else (m,), dtype=torch.float64, device=dev)
    lib.gpr_predict_var(f["Z"], f["n"], Zst, m, f["d"], h, f["K"], f["tile"], f["prec"], full_cov, add_noise, out,
                        ws, wsb)
    torch.cuda.synchronize()
    return mean.cpu().numpy(), out.cpu().numpy()


C1 = dict(n=1024, m=1024, D=8, tile=256, seed=1, h=Hyper(1.0, 1.0, 0.01))


@pytest.fixture(scope="module")
def c1():
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=C1["n"], n_test=C1["m"], D=C1["D"], seed=C1["seed"]))
    h = C1["h"]
    L, a, f = oracle.fit(ds.Z, ds.y, h)
    return ds, h, L, a, f


def test_factor_and_inverse_parity(lib, c1):
    ds, h, L, a, f = c1
    g = _gpu_fit(lib, ds.Z, ds.y, h, C1["tile"])
    raw = g["K"].cpu().numpy()
    Lg = tiles_to_dense_lower(raw, C1["n"], C1["tile"], 8)
    assert np.max(np.abs(Lg - L)) / np.max(np.abs(L)) < 1e-12
    b = C1["tile"]
    for k, Wk in enumerate(winv_tiles(raw, C1["n"], b)):
        Lkk = L[k * b:(k + 1) * b, k * b:(k + 1) * b]
        assert np.all(np.triu(Wk, 1) == 0)
        assert np.max(np.abs(Wk @ Lkk - np.eye(b))) < 1e-11


def test_c1_alpha_mean_var_nlml(lib, c1):
    ds, h, L, a, f = c1
    g = _gpu_fit(lib, ds.Z, ds.y, h, C1["tile"])
    assert_close(g["alpha"].cpu().numpy(), a, 1e-10)
    assert abs(g["nlml"] - f) / abs(f) < 1e-10
    mean, var = _gpu_predict(lib, g, ds.Zs, h)
    assert_close(mean, oracle.predict_mean(ds.Z, ds.Zs, h, a), 1e-10)
    vo = oracle.predict_var(ds.Z, ds.Zs, h, L)
    assert_close(var, vo, 1e-10)
    assert np.all(var >= -1e-12 * h.signal_var) and np.all(var <= h.signal_var * (1 + 1e-12))
    _, varn = _gpu_predict(lib, g, ds.Zs, h, add_noise=True)
    assert_close(varn, vo + h.noise_var, 1e-10)


def test_c1_full_covariance(lib, c1):
    ds, h, L, a, f = c1
    g = _gpu_fit(lib, ds.Z, ds.y, h, C1["tile"])
    Zs = ds.Zs[:300]
    _, S = _gpu_predict(lib, g, Zs, h, full_cov=True)
    So = oracle.predict_var(ds.Z, Zs, h, L, full_cov=True)
    assert_close(S, So, 1e-10)
    _, v = _gpu_predict(lib, g, Zs, h)
    assert_close(np.diag(S), v, 1e-12)
    _, Sn = _gpu_predict(lib, g, Zs, h, full_cov=True, add_noise=True)
    assert_close(Sn - h.noise_var * np.eye(300), So, 1e-10)


@pytest.mark.parametrize("n,tile,D", [(512, 512, 6), (512, 128, 6), (512, 32, 6), (300, 100, 3), (111, 37, 5),
                                      (130, 65, 4), (3, 1, 2), (7, 7, 3)])
def test_tilings_and_ragged_sizes(lib, n, tile, D):
    rng = np.random.default_rng(n * 7 + tile)
    Z = rng.normal(size=(n, D))
    y = np.sin(Z[:, 0]) + 0.1 * rng.normal(size=n)
    Zs = rng.normal(size=(33, D))
    h = Hyper(1.1, 0.9, 0.05)
    L, a, f = oracle.fit(Z, y, h)
    g = _gpu_fit(lib, Z, y, h, tile, m=33)
    assert abs(g["nlml"] - f) / abs(f) < 1e-10
    assert_close(g["alpha"].cpu().numpy(), a, 1e-10)
    mean, var = _gpu_predict(lib, g, Zs, h)
    assert_close(mean, oracle.predict_mean(Z, Zs, h, a), 1e-10)
    assert_close(var, oracle.predict_var(Z, Zs, h, L), 1e-10)


@pytest.mark.parametrize("n,tile", [(2048, 1024), (3072, 1024)])
def test_large_tile_parity(lib, n, tile):
    """Tiles of 1024: every job's 128 x 128 macro-tile grid is a multiple of 8 in both
    directions, so the GEMMs take the 8 x 8 block order of their workgroups."""
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=n, n_test=64, D=16, seed=n))
    h = Hyper(4.0, 1.0, 0.01)
    L, a, f = oracle.fit(ds.Z, ds.y, h)
    g = _gpu_fit(lib, ds.Z, ds.y, h, tile, m=64)
    assert abs(g["nlml"] - f) / abs(f) < 1e-10
    assert_close(g["alpha"].cpu().numpy(), a, 1e-10)
    mean, var = _gpu_predict(lib, g, ds.Zs, h)
    assert_close(mean, oracle.predict_mean(ds.Z, ds.Zs, h, a), 1e-10)
    assert_close(var, oracle.predict_var(ds.Z, ds.Zs, h, L), 1e-10)
    grad = torch.empty(3, dtype=torch.float64, device="cuda:0")
    lib.gpr_nlml_grad(g["Z"], g["n"], g["d"], h, g["K"], tile, "fp64", g["alpha"], (1, 1, 1), grad, g["ws"], g["wsb"])
    go = oracle.nlml_grad(ds.Z, h, L, a)
    np.testing.assert_allclose(grad.cpu().numpy(), go, rtol=1e-9, atol=1e-9 * np.max(np.abs(go)))


def test_tiling_invariance_bitwise_determinism(lib):
    rng = np.random.default_rng(3)
    n, D = 768, 8
    Z = rng.normal(size=(n, D))
    y = rng.normal(size=n)
    h = Hyper(1.0, 1.0, 0.01)
    res = {}
    for tile in (768, 192, 48):
        g1 = _gpu_fit(lib, Z, y, h, tile)
        g2 = _gpu_fit(lib, Z, y, h, tile)
        a1, a2 = g1["alpha"].cpu().numpy(), g2["alpha"].cpu().numpy()
        assert np.array_equal(a1, a2), "run-to-run results must be bitwise identical"
        res[tile] = (a1, g1["nlml"])
    for tile in (192, 48):
        assert_close(res[tile][0], res[768][0], 1e-11)
        assert abs(res[tile][1] - res[768][1]) / abs(res[768][1]) < 1e-12


@pytest.mark.parametrize("n,m", [(1024, 1024), (1000, 333)])
@pytest.mark.parametrize("offset", [0.0, 1e4])
def test_mean_of_points_far_from_the_origin(lib, n, m, offset):
    """The squared-exponential kernel-vector products form distances from Gram products
    when the squared norms of the points are small against the lengthscale, from
    explicit differences otherwise.  Points shifted by 1e4 in every feature would lose
    about 1e-7 of each kernel value to the cancellation of the Gram form; the mean must
    stay within rounding of the oracle's either way (full and ragged 128-point blocks)."""
    rng = np.random.default_rng(int(offset) + n)
    D = 8
    Z = rng.normal(size=(n, D)) + offset
    Zs = np.concatenate([Z[:m // 2], rng.normal(size=(m - m // 2, D)) + offset])   # half of them training points
    alpha = rng.normal(size=n)
    h = Hyper(1.5, 0.8, 0.01)
    dev = "cuda:0"
    Zt, Zst, at = (torch.tensor(x, device=dev) for x in (Z, Zs, alpha))
    wsb = lib.gpr_workspace_size(n, m, D, 256, "fp64")
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    mean = torch.empty(m, dtype=torch.float64, device=dev)
    lib.gpr_predict(Zt, n, Zst, m, D, h, at, mean, ws, wsb)
    torch.cuda.synchronize()
    print(f"[far-points] n={n} m={m} offset={offset:g}", flush=True)
    assert_elementwise(mean.cpu().numpy(), oracle.predict_mean(Z, Zs, h, alpha), 1e-10)


def test_one_point_closed_form(lib):
    z1 = np.array([[0.3, -1.2, 0.5]])
    y1 = np.array([0.8])
    ell, nu, s2 = 0.7, 2.5, 0.3
    h = Hyper(ell, nu, s2)
    g = _gpu_fit(lib, z1, y1, h, 1)
    a = nu + s2
    assert g["alpha"].item() == pytest.approx(y1[0] / a, rel=1e-15)
    assert g["nlml"] == pytest.approx(0.5 * math.log(a) + y1[0] ** 2 / (2 * a) + 0.5 * math.log(2 * math.pi), rel=1e-14)
    zs = np.array([[0.3, -1.2, 0.5], [1.0, 0.0, -0.4]])
    mean, var = _gpu_predict(lib, g, zs, h)
    r2 = np.sum((zs - z1) ** 2, axis=1)
    np.testing.assert_allclose(mean, nu * np.exp(-r2 / (2 * ell ** 2)) * y1[0] / a, rtol=1e-14)
    np.testing.assert_allclose(var, nu - nu ** 2 * np.exp(-r2 / ell ** 2) / a, rtol=1e-13)


def test_not_spd_reports_first_bad_column(lib):
    rng = np.random.default_rng(4)
    n, tile, D = 256, 64, 3
    Z = rng.normal(size=(n, D))
    h = Hyper(1.0, 1.0, 0.1)
    dev = "cuda:0"
    for col in (1, 70, 200, 256):
        Zt = torch.tensor(Z, device=dev)
        K = torch.empty(lib.gpr_tiles_bytes(n, tile, "fp64"), dtype=torch.uint8, device=dev)
        wsb = lib.gpr_workspace_size(n, 0, D, tile, "fp64")
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        lib.gpr_assemble(Zt, n, D, h, tile, "fp64", K)
        # set K[col-1, col-1] = -3 inside its diagonal tile
        k, r = (col - 1) // tile, (col - 1) % tile
        Kd = K.view(torch.float64)
        Kd[k * tile * tile + r * tile + r] = -3.0
        Kh = oracle.train_cov(Z, h)
        Kh[col - 1, col - 1] = -3.0
        assert lib.gpr_cholesky(K, n, tile, "fp64", ws, wsb) == oracle.potrf_info(Kh) == col


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
def test_nan_input_reports_its_column(lib, prec):
    """A NaN in one training input makes its row and column of K NaN; every pivot before it
    stays finite, so the factorisation reports that column as the first bad pivot (1-based),
    as LAPACK's dpotrf does on the oracle's matrix (a NaN pivot fails the positivity test)."""
    rng = np.random.default_rng(5)
    n, tile, D = 512, 128, 3
    h = Hyper(1.0, 1.0, 0.1)
    dev = "cuda:0"
    for row in (0, 130, 511):
        Z = rng.normal(size=(n, D))
        Z[row, 1] = np.nan
        K = torch.empty(lib.gpr_tiles_bytes(n, tile, prec), dtype=torch.uint8, device=dev)
        wsb = lib.gpr_workspace_size(n, 0, D, tile, prec)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        lib.gpr_assemble(torch.tensor(Z, device=dev), n, D, h, tile, prec, K)
        assert lib.gpr_cholesky(K, n, tile, prec, ws, wsb) == oracle.potrf_info(oracle.train_cov(Z, h)) == row + 1


def test_gradient_parity(lib):
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=512, n_test=8, D=8, seed=2))
    h = Hyper(1.3, 0.8, 0.05)
    L, a, f = oracle.fit(ds.Z, ds.y, h)
    go = oracle.nlml_grad(ds.Z, h, L, a)
    for tile in (512, 128, 96 if 512 % 96 == 0 else 64):
        g = _gpu_fit(lib, ds.Z, ds.y, h, tile)
        grad = torch.empty(3, dtype=torch.float64, device="cuda:0")
        lib.gpr_nlml_grad(g["Z"], g["n"], g["d"], h, g["K"], tile, "fp64", g["alpha"], (1, 1, 1), grad, g["ws"],
                          g["wsb"])
        gv = grad.cpu().numpy()
        np.testing.assert_allclose(gv, go, rtol=1e-9, atol=1e-9 * np.max(np.abs(go)))
    g = _gpu_fit(lib, ds.Z, ds.y, h, 128)
    grad = torch.empty(3, dtype=torch.float64, device="cuda:0")
    lib.gpr_nlml_grad(g["Z"], g["n"], g["d"], h, g["K"], 128, "fp64", g["alpha"], (0, 1, 0), grad, g["ws"], g["wsb"])
    gv = grad.cpu().numpy()
    assert gv[0] == 0.0 and gv[2] == 0.0 and gv[1] == pytest.approx(go[1], rel=1e-9)


def test_optimize_matches_oracle_adam(lib):
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=384, n_test=8, D=8, seed=5))
    theta0 = [0.0, 0.0, math.log(0.1)]
    th_o, tr_o = oracle.optimize(ds.Z, ds.y, theta0, steps=6, lr=0.1)
    n, d, tile = 384, 8, 128
    dev = "cuda:0"
    Zt, yt = torch.tensor(ds.Z, device=dev), torch.tensor(ds.y, device=dev)
    K = torch.empty(lib.gpr_tiles_bytes(n, tile, "fp64"), dtype=torch.uint8, device=dev)
    wsb = lib.gpr_workspace_size(n, 0, d, tile, "fp64")
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    th, st, tr = lib.gpr_optimize(Zt, yt, n, d, tile, "fp64", theta0, (1, 1, 1), 6, 0.1, 0.9, 0.999, 1e-8, None,
                                  K, ws, wsb)
    np.testing.assert_allclose(th, th_o, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(tr, tr_o, rtol=1e-10)
    # resuming 3 + 3 steps equals 6 steps bitwise
    th1, st1, tr1 = lib.gpr_optimize(Zt, yt, n, d, tile, "fp64", theta0, (1, 1, 1), 3, 0.1, 0.9, 0.999, 1e-8, None,
                                     K, ws, wsb)
    th2, st2, tr2 = lib.gpr_optimize(Zt, yt, n, d, tile, "fp64", th1, (1, 1, 1), 3, 0.1, 0.9, 0.999, 1e-8, st1,
                                     K, ws, wsb)
    assert th2 == th and st2 == st


def test_autograd_function_backward(lib):
    from paper_2505_00136_amd.gp import GP, nlml
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=256, n_test=8, D=4, seed=6))
    gp = GP(ds.Z, ds.y, hyper=(1.0, 1.0, 0.1), tile=64)
    theta = torch.tensor([0.1, -0.2, math.log(0.05)], dtype=torch.float64, requires_grad=True)
    loss = nlml(theta, gp)
    loss.backward()
    h = Hyper.from_log(theta.detach().numpy())
    L, a, f = oracle.fit(ds.Z, ds.y, h)
    assert loss.item() == pytest.approx(f, rel=1e-10)
    np.testing.assert_allclose(theta.grad.numpy(), oracle.nlml_grad(ds.Z, h, L, a), rtol=1e-9)
    # central differences of the GPU forward (h = 1e-5)
    step = 1e-5
    for k in range(3):
        tp = theta.detach().clone(); tp[k] += step
        tm = theta.detach().clone(); tm[k] -= step
        fd = (nlml(tp, gp).item() - nlml(tm, gp).item()) / (2 * step)
        assert theta.grad[k].item() == pytest.approx(fd, rel=1e-6, abs=1e-6)


@pytest.mark.parametrize("n,tile", [(16, 1), (32, 2), (64, 4), (8, 8), (24, 3), (128, 8)])
def test_small_problems_many_tiles(lib, n, tile):
    """The small end of the problem-size sweep (N = M, up to 16 tiles per dimension, tiles
    down to a single element): gradient, full covariance and two Adam steps against the
    oracle."""
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=n, n_test=n, D=8, seed=n + tile))
    h = Hyper(1.0, 1.0, 0.1)
    L, a, f = oracle.fit(ds.Z, ds.y, h)
    g = _gpu_fit(lib, ds.Z, ds.y, h, tile, m=n)
    assert abs(g["nlml"] - f) / abs(f) < 1e-10
    grad = torch.empty(3, dtype=torch.float64, device="cuda:0")
    lib.gpr_nlml_grad(g["Z"], n, 8, h, g["K"], tile, "fp64", g["alpha"], (1, 1, 1), grad, g["ws"], g["wsb"])
    go = oracle.nlml_grad(ds.Z, h, L, a)
    np.testing.assert_allclose(grad.cpu().numpy(), go, rtol=1e-9, atol=1e-9 * np.max(np.abs(go)))
    g = _gpu_fit(lib, ds.Z, ds.y, h, tile, m=n)
    mean, cov = _gpu_predict(lib, g, ds.Zs, h, full_cov=True)
    assert_close(mean, oracle.predict_mean(ds.Z, ds.Zs, h, a), 1e-10)
    So = oracle.predict_var(ds.Z, ds.Zs, h, L, full_cov=True)
    assert np.max(np.abs(cov - So)) < 1e-10 * max(1.0, np.max(np.abs(So)))
    theta0 = [0.0, 0.0, math.log(0.1)]
    th_o, tr_o = oracle.optimize(ds.Z, ds.y, theta0, steps=2, lr=0.1)
    th, st, tr = lib.gpr_optimize(g["Z"], g["y"], n, 8, tile, "fp64", theta0, (1, 1, 1), 2, 0.1, 0.9, 0.999, 1e-8,
                                  None, g["K"], g["ws"], g["wsb"])
    np.testing.assert_allclose(th, th_o, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(tr, tr_o, rtol=1e-10)


def test_automatic_tile_selection(lib, tmp_path):
    """The selector times every candidate tile on the device and returns the fastest; a
    GP built with tile="auto" uses a valid tile and matches the oracle."""
    from paper_2505_00136_amd.tile_select import candidate_tiles, select_tile
    n, d = 2048, 8
    best, times = select_tile(n, d, "fp64", reps=1, cache_path=str(tmp_path / "tiles.json"))
    assert set(times) == set(candidate_tiles(n)) and best == min(times, key=times.get)
    again, _ = select_tile(n, d, "fp64", cache_path=str(tmp_path / "tiles.json"))
    assert again == best
    from paper_2505_00136_amd.gp import GP
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=512, n_test=16, D=4, seed=9))
    gp = GP(ds.Z, ds.y, hyper=(1.0, 1.0, 0.05), tile="auto")
    assert gp.tile in candidate_tiles(512)
    gp.fit()
    h = Hyper(1.0, 1.0, 0.05)
    _, _, f = oracle.fit(ds.Z, ds.y, h)
    assert float(gp.nlml().item()) == pytest.approx(f, rel=1e-10)


def test_empty_inputs(lib):
    """n = 0: every call is a no-op or returns the prior (mean 0, variance nu, covariance
    K(Zs, Zs)), the NLML and its gradient are 0; m = 0: the predictions touch nothing."""
    dev = "cuda:0"
    rng = np.random.default_rng(5)
    m, d, tile = 17, 3, 64
    h = Hyper(1.1, 0.7, 0.05)
    Zs = rng.normal(size=(m, d))
    Zst = torch.tensor(Zs, device=dev)
    empty = torch.empty((0, d), dtype=torch.float64, device=dev)
    e1 = torch.empty(0, dtype=torch.float64, device=dev)
    assert lib.gpr_tiles_bytes(0, tile, "fp64") == 0
    wsb = lib.gpr_workspace_size(0, m, d, tile, "fp64")
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    K = torch.empty(0, dtype=torch.uint8, device=dev)
    lib.gpr_assemble(empty, 0, d, h, tile, "fp64", K)
    assert lib.gpr_cholesky(K, 0, tile, "fp64", ws, wsb) == 0
    lib.gpr_solve(K, empty, 0, d, h, tile, "fp64", e1, e1, 0, ws, wsb)
    nl = torch.full((1,), 7.0, dtype=torch.float64, device=dev)
    lib.gpr_nlml(K, 0, tile, "fp64", e1, e1, nl)
    grad = torch.full((3,), 7.0, dtype=torch.float64, device=dev)
    lib.gpr_nlml_grad(empty, 0, d, h, K, tile, "fp64", e1, (1, 1, 1), grad, ws, wsb)
    mean = torch.full((m,), 7.0, dtype=torch.float64, device=dev)
    lib.gpr_predict(empty, 0, Zst, m, d, h, e1, mean, ws, wsb)
    var = torch.empty(m, dtype=torch.float64, device=dev)
    lib.gpr_predict_var(empty, 0, Zst, m, d, h, K, tile, "fp64", False, True, var, ws, wsb)
    cov = torch.empty((m, m), dtype=torch.float64, device=dev)
    lib.gpr_predict_var(empty, 0, Zst, m, d, h, K, tile, "fp64", True, False, cov, ws, wsb)
    torch.cuda.synchronize()
    assert nl.item() == 0.0 and torch.all(grad == 0.0) and torch.all(mean == 0.0)
    np.testing.assert_allclose(var.cpu().numpy(), np.full(m, h.signal_var + h.noise_var), rtol=1e-15)
    np.testing.assert_allclose(cov.cpu().numpy(), oracle.cov(Zs, Zs, h), rtol=1e-13, atol=1e-15)
    # m = 0 with data: outputs untouched
    n = 40
    Z = rng.normal(size=(n, d))
    y = np.sin(Z[:, 0])
    g = _gpu_fit(lib, Z, y, h, 16)
    sentinel = torch.full((4,), 3.0, dtype=torch.float64, device=dev)
    lib.gpr_predict(g["Z"], n, Zst, 0, d, h, g["alpha"], sentinel, g["ws"], g["wsb"])
    lib.gpr_predict_var(g["Z"], n, Zst, 0, d, h, g["K"], 16, "fp64", True, False, sentinel, g["ws"], g["wsb"])
    torch.cuda.synchronize()
    assert torch.all(sentinel == 3.0)
