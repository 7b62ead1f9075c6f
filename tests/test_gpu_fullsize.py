"""GPU checks at the benchmark's full size: n = 65536 training points, D = 128, 8192 test
points, tile 2048, the hyperparameters and data of bench.py (so the same launches run).

The oracle cannot factor K at this size, so the checks use outputs it computes one at a
time -- sampled rows of K alpha, sampled entries of L L^T, sampled posterior means -- and
properties that hold at any size: the variance lies in [0, nu] and the var-only path
agrees with the diagonal of the full covariance, the gradient agrees with central
differences of the library's own NLML, and the mixed paths (float32 trailing updates,
3-way split bfloat16) agree with the float64 one within the mixed-precision bounds.

Tolerances (float64, kappa(K) ~ 1e4 here): a backward-stable factorisation gives
|L L^T - K|_ij <= c n eps nu (n eps = 7e-12), hence 1e-10 nu; the solve residual
|K alpha - y|_i is bounded the same way times |alpha|, hence 1e-9 max|y|; a posterior
mean recomputed from the same alpha differs only in summation order, hence 1e-12.
"""
import math

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from tests.tiles import lower_row  # noqa: E402

N, M, D, TILE, SEED = 65536, 8192, 128, 2048, 3
H = (math.sqrt(D), 1.0, 0.01)


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_00136_amd import _lib
    _lib.load()
    print(f"[fullsize] n={N} m={M} D={D} tile={TILE}: data", flush=True)
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=N, n_test=M, D=D, seed=SEED))
    dev = torch.device("cuda:0")
    Z, Zs, y = (torch.tensor(a, device=dev) for a in (ds.Z, ds.Zs, ds.y))
    wsb = max(_lib.gpr_workspace_size(N, M, D, TILE, p) for p in ("fp64", "fp32", "bf16x6"))
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    K = torch.empty(_lib.gpr_tiles_bytes(N, TILE, "fp64"), dtype=torch.uint8, device=dev)

    def fit(h, prec="fp64", Kbuf=None, sweeps=0):
        Kb = K if Kbuf is None else Kbuf
        alpha = torch.empty(N, dtype=torch.float64, device=dev)
        nl = torch.empty(1, dtype=torch.float64, device=dev)
        _lib.gpr_assemble(Z, N, D, h, TILE, prec, Kb)
        info = _lib.gpr_cholesky(Kb, N, TILE, prec, ws, wsb)
        assert info == 0
        _lib.gpr_solve(Kb, Z, N, D, h, TILE, prec, y, alpha, sweeps, ws, wsb)
        _lib.gpr_nlml(Kb, N, TILE, prec, y, alpha, nl)
        return alpha, float(nl.item())

    print("[fullsize] float64 fit", flush=True)
    alpha, nlml = fit(H)
    mean = torch.empty(M, dtype=torch.float64, device=dev)
    var = torch.empty(M, dtype=torch.float64, device=dev)
    _lib.gpr_predict(Z, N, Zs, M, D, H, alpha, mean, ws, wsb)
    _lib.gpr_predict_var(Z, N, Zs, M, D, H, K, TILE, "fp64", False, False, var, ws, wsb)
    # variance at training inputs (the first M training points)
    var_train = torch.empty(M, dtype=torch.float64, device=dev)
    Zt = Z[:M].contiguous()
    _lib.gpr_predict_var(Z, N, Zt, M, D, H, K, TILE, "fp64", False, False, var_train, ws, wsb)
    torch.cuda.synchronize()
    return dict(lib=_lib, ds=ds, Z=Z, Zs=Zs, y=y, K=K, ws=ws, wsb=wsb, fit=fit, alpha=alpha,
                alpha_h=alpha.cpu().numpy(), nlml=nlml, mean=mean.cpu().numpy(), var=var.cpu().numpy(),
                var_train=var_train.cpu().numpy())


def test_sampled_solve_residual(full):
    ds, a = full["ds"], full["alpha_h"]
    ell, nu, s2 = H
    rows = np.random.default_rng(11).choice(N, 64, replace=False)
    r = oracle.se_cov(ds.Z[rows], ds.Z, ell, nu) @ a + s2 * a[rows] - ds.y[rows]
    assert np.max(np.abs(r)) <= 1e-9 * np.max(np.abs(ds.y))


def test_sampled_factor_entries(full):
    ds, K = full["ds"], full["K"]
    ell, nu, s2 = H
    rng = np.random.default_rng(12)
    pairs = [(int(i), int(rng.integers(0, i + 1))) for i in rng.choice(N, 24, replace=False)]
    pairs += [(N - 1, N - 1), (N - 1, 0), (TILE, TILE - 1), (0, 0)]
    for i, j in pairs:
        li, lj = lower_row(K, N, TILE, 8, i), lower_row(K, N, TILE, 8, j)
        llt = float(np.dot(li[: j + 1], lj[: j + 1]))
        kij = float(oracle.se_cov(ds.Z[i:i + 1], ds.Z[j:j + 1], ell, nu)[0, 0]) + (s2 if i == j else 0.0)
        assert abs(llt - kij) <= 1e-10 * nu, (i, j, llt, kij)


def test_sampled_posterior_mean(full):
    ds, a = full["ds"], full["alpha_h"]
    ell, nu, _ = H
    rows = np.random.default_rng(13).choice(M, 64, replace=False)
    ref = oracle.se_cov(ds.Zs[rows], ds.Z, ell, nu) @ a
    got = full["mean"][rows]
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(np.max(np.abs(ref)), 1.0)


def test_variance_bounds_and_full_covariance(full):
    lib, var = full["lib"], full["var"]
    _, nu, _ = H
    assert np.all(var >= -1e-12 * nu) and np.all(var <= nu * (1 + 1e-12))
    m = 256
    Zs = full["Zs"][:m].contiguous()
    S = torch.empty((m, m), dtype=torch.float64, device="cuda:0")
    lib.gpr_predict_var(full["Z"], N, Zs, m, D, H, full["K"], TILE, "fp64", True, False, S, full["ws"], full["wsb"])
    S = S.cpu().numpy()
    assert np.max(np.abs(np.diag(S) - var[:m])) <= 1e-12 * nu
    assert np.max(np.abs(S - S.T)) <= 1e-12 * nu


def test_training_point_variance_bound(full):
    """Conditioning on more points only shrinks the variance, so at a training input it is
    at most the one-point posterior variance nu sigma^2 / (nu + sigma^2)."""
    _, nu, s2 = H
    v = full["var_train"]
    assert np.all(v >= -1e-12 * nu)
    assert np.all(v <= nu * s2 / (nu + s2) * (1 + 1e-9) + 1e-12 * nu), float(np.max(v))


def test_factorisation_bitwise_reproducible(full):
    """A repeated factorisation (and solve) gives the same bits."""
    alpha2, nlml2 = full["fit"](H)
    assert torch.equal(alpha2, full["alpha"]) and nlml2 == full["nlml"]


def test_lookahead_matches_single_stream_bitwise(full):
    """The two-stream factorisation (look-ahead) and the one-stream schedule perform the
    same arithmetic per element, so they give the same bits; repeated look-ahead
    factorisations agree too.  (A read-modify-write of the LDS exchange vector in the
    diagonal-block kernel once raced with other waves and made the look-ahead differ.)"""
    lib = full["lib"]
    lib.gpr_set_lookahead(False)
    try:
        a0, n0 = full["fit"](H)
    finally:
        lib.gpr_set_lookahead(True)
    runs = [full["fit"](H) for _ in range(3)]
    for a1, n1 in runs:
        assert torch.equal(a1, a0) and n1 == n0


def test_device_schedule_matches_lookahead_bitwise(full):
    """The task graph executed on the device gives the factor and alpha of the stream
    schedules, bit for bit, at the full size (3693 tasks, 2.4 million work items)."""
    lib = full["lib"]
    a0, n0 = full["fit"](H)
    lib.gpr_set_schedule("device")
    try:
        a1, n1 = full["fit"](H)
    finally:
        lib.gpr_set_schedule("lookahead")
    assert torch.equal(a1, a0) and n1 == n0


def test_gradient_against_central_differences(full):
    lib = full["lib"]
    grad = torch.empty(3, dtype=torch.float64, device="cuda:0")
    lib.gpr_nlml_grad(full["Z"], N, D, H, full["K"], TILE, "fp64", full["alpha"], (1, 1, 1), grad, full["ws"],
                      full["wsb"])
    g = grad.cpu().numpy()
    th = np.log(np.array(H))
    hstep = 5e-4
    fd = np.zeros(3)
    for k in range(3):
        f = []
        for sgn in (1.0, -1.0):
            t = th.copy()
            t[k] += sgn * hstep
            f.append(full["fit"](tuple(np.exp(t)))[1])
        fd[k] = (f[0] - f[1]) / (2 * hstep)
        print(f"[fullsize] d nlml / d log theta[{k}]: analytic {g[k]:.10e} central difference {fd[k]:.10e}", flush=True)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-6 * np.max(np.abs(fd)))


def test_gradient_bitwise_reproducible(full):
    """The inversion and trace kernels of the gradient (eight waves per workgroup) give the
    same bits when the factorisation and the gradient are repeated."""
    lib = full["lib"]
    out = []
    for _ in range(2):
        alpha, _ = full["fit"](H)
        grad = torch.empty(3, dtype=torch.float64, device="cuda:0")
        lib.gpr_nlml_grad(full["Z"], N, D, H, full["K"], TILE, "fp64", alpha, (1, 1, 1), grad, full["ws"],
                          full["wsb"])
        out.append(grad.cpu().numpy())
    assert np.array_equal(out[0], out[1]), out


@pytest.mark.parametrize("prec,tol_alpha,tol_var", [("fp32", 1e-8, 1e-4), ("bf16x6", 1e-8, 1e-4),
                                                    ("bf16x3", 1e-6, 1e-3)])
def test_mixed_paths_within_bounds(full, prec, tol_alpha, tol_var):
    """FP32 trailing updates and the 3-way split-bfloat16 products (hi/mid/lo; six or three
    products), float64 diagonal tiles, the precision's default refinement sweeps: mean and
    NLML within 1e-6 of float64."""
    lib = full["lib"]
    K32 = torch.empty(lib.gpr_tiles_bytes(N, TILE, prec), dtype=torch.uint8, device="cuda:0")
    a32, nl32 = full["fit"](H, prec, K32, -1)
    assert abs(nl32 - full["nlml"]) / abs(full["nlml"]) <= 1e-6
    a = full["alpha_h"]
    assert np.linalg.norm(a32.cpu().numpy() - a) / np.linalg.norm(a) <= tol_alpha
    mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
    lib.gpr_predict(full["Z"], N, full["Zs"], M, D, H, a32, mean, full["ws"], full["wsb"])
    mref = full["mean"]
    assert np.linalg.norm(mean.cpu().numpy() - mref) / np.linalg.norm(mref) <= 1e-6
    var = torch.empty(M, dtype=torch.float64, device="cuda:0")
    lib.gpr_predict_var(full["Z"], N, full["Zs"], M, D, H, K32, TILE, prec, False, False, var, full["ws"],
                        full["wsb"])
    assert np.max(np.abs(var.cpu().numpy() - full["var"])) <= tol_var


def test_nearly_diagonal_closed_form_at_full_size(full):
    """l = 1 on the D = 128 standardised features: every off-diagonal kernel value is below
    exp(-min r^2 / 2), checked on the factor in the run, so K = (nu + sigma^2) I to far below
    rounding and alpha = y / c, NLML = n/2 log c + y^T y / (2 c) + n/2 log 2 pi, the posterior
    mean is 0 and the variance nu, and nu sigma^2 / c at training inputs (c = nu + sigma^2).
    (Run last: it refactors the shared buffer at other hyperparameters.)"""
    lib, ds = full["lib"], full["ds"]
    h = (1.0, 1.0, 0.01)
    nu, s2 = h[1], h[2]
    c = nu + s2
    alpha, nlml = full["fit"](h)
    K = full["K"]
    T = N // TILE
    dreg = K[: T * TILE * TILE * 8].view(torch.float64).view(T, TILE, TILE)
    off_diag_tiles = float(torch.tril(dreg, diagonal=-1).abs().max().item())
    off_region = float(K[2 * T * TILE * TILE * 8:].view(torch.float64).abs().max().item())
    max_off = max(off_diag_tiles, off_region)
    print(f"[fullsize] l = 1: largest off-diagonal factor entry {max_off:.3e}", flush=True)
    assert max_off <= 1e-20
    y = ds.y
    np.testing.assert_allclose(alpha.cpu().numpy(), y / c, rtol=1e-14, atol=1e-15 * np.max(np.abs(y)))
    want = 0.5 * N * math.log(c) + float(y @ y) / (2 * c) + 0.5 * N * math.log(2 * math.pi)
    assert abs(nlml - want) <= 1e-13 * abs(want)
    mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
    var = torch.empty(M, dtype=torch.float64, device="cuda:0")
    lib.gpr_predict(full["Z"], N, full["Zs"], M, D, h, alpha, mean, full["ws"], full["wsb"])
    lib.gpr_predict_var(full["Z"], N, full["Zs"], M, D, h, K, TILE, "fp64", False, False, var, full["ws"],
                        full["wsb"])
    vt = torch.empty(M, dtype=torch.float64, device="cuda:0")
    Zt = full["Z"][:M].contiguous()
    lib.gpr_predict_var(full["Z"], N, Zt, M, D, h, K, TILE, "fp64", False, False, vt, full["ws"], full["wsb"])
    torch.cuda.synchronize()
    assert np.max(np.abs(mean.cpu().numpy())) <= 1e-15
    np.testing.assert_allclose(var.cpu().numpy(), nu, rtol=1e-14)
    np.testing.assert_allclose(vt.cpu().numpy(), nu * s2 / c, rtol=1e-12)
