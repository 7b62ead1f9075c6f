"""Mixed-precision paths against the float64 oracle at n = 16384, tile 1024.

16 x 16 tiles of 1024 run the same specialised (whole-macro-tile, MC/MC-operand) main loops
as the benchmark's 2048-wide tiles, unlike the small ragged cases of test_gpu_mixed.py.
The workload is the benchmark's (D = 128 lagged inputs, l = sqrt(D), nu = 1, sigma^2 =
0.01, a dense K with kappa ~ 1e4) at n = 16384 training and 4096 test points, which the
oracle still solves completely on the host.

Stated bounds (relative; normwise ||a - b|| / ||b||, per entry against
max(|b_i|, 1e-3 max|b|), tests/checks.py):
* alpha and the posterior mean after the precision's default refinement sweeps (float64
  residuals): 1e-6 normwise for every mode, the target for mean and NLML;
* NLML (log-determinant from the mixed factor): 1e-6;
* variance (mixed factor, no refinement, float64 sums): 1e-4 normwise, 1e-3 per entry;
  bf16x3 (about 16 significant bits per product) 1e-3 and 1e-2;
* gradient (mixed factor and inverse): 1e-3 normwise; bf16x3 1e-2;
* the full covariance's diagonal equals the var-only output to 1e-12 nu: both sum the
  same float32 V in float64.
Each error reached is printed.
"""
import math

import numpy as np
import pytest

import datagen
import oracle
from oracle import Hyper

from tests.checks import assert_close, elementwise_err, normwise_err  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, M, D, TILE, SEED = 16384, 4096, 128, 1024, 3
H = Hyper(math.sqrt(D), 1.0, 0.01)
MC = 1024   # test points of the full-covariance check
BOUNDS = {  # prec: (variance normwise, variance per entry, gradient)
    "fp32": (1e-4, 1e-3, 1e-3), "bf16x6": (1e-4, 1e-3, 1e-3), "bf16x3": (1e-3, 1e-2, 1e-2)}


@pytest.fixture(scope="module")
def ref():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=N, n_test=M, D=D, seed=SEED))
    print("[mixed16384] oracle fit", flush=True)
    L, a, f = oracle.fit(ds.Z, ds.y, H)
    print("[mixed16384] oracle mean and variance", flush=True)
    r = dict(ds=ds, alpha=a, nlml=f, mean=oracle.predict_mean(ds.Z, ds.Zs, H, a),
             var=oracle.predict_var(ds.Z, ds.Zs, H, L))
    print("[mixed16384] oracle gradient", flush=True)
    r["grad"] = oracle.nlml_grad(ds.Z, H, L, a)
    return r


@pytest.fixture(scope="module")
def dev_inputs(ref):
    from paper_2505_00136_amd import _lib
    _lib.load()
    ds = ref["ds"]
    dev = torch.device("cuda:0")
    Z, Zs, y = (torch.tensor(x, device=dev) for x in (ds.Z, ds.Zs, ds.y))
    wsb = max(_lib.gpr_workspace_size(N, M, D, TILE, p) for p in BOUNDS)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    return dict(lib=_lib, Z=Z, Zs=Zs, y=y, ws=ws, wsb=wsb)


def _run(d, prec, sweeps=-1):
    lib, Z, Zs, y, ws, wsb = (d[k] for k in ("lib", "Z", "Zs", "y", "ws", "wsb"))
    dev = "cuda:0"
    h = (H.lengthscale, H.signal_var, H.noise_var)
    K = torch.empty(lib.gpr_tiles_bytes(N, TILE, prec), dtype=torch.uint8, device=dev)
    alpha = torch.empty(N, dtype=torch.float64, device=dev)
    nl = torch.empty(1, dtype=torch.float64, device=dev)
    mean = torch.empty(M, dtype=torch.float64, device=dev)
    var = torch.empty(M, dtype=torch.float64, device=dev)
    cov = torch.empty((MC, MC), dtype=torch.float64, device=dev)
    grad = torch.empty(3, dtype=torch.float64, device=dev)
    lib.gpr_assemble(Z, N, D, h, TILE, prec, K)
    assert lib.gpr_cholesky(K, N, TILE, prec, ws, wsb) == 0
    lib.gpr_solve(K, Z, N, D, h, TILE, prec, y, alpha, sweeps, ws, wsb)
    lib.gpr_nlml(K, N, TILE, prec, y, alpha, nl)
    lib.gpr_predict(Z, N, Zs, M, D, h, alpha, mean, ws, wsb)
    lib.gpr_predict_var(Z, N, Zs, M, D, h, K, TILE, prec, False, False, var, ws, wsb)
    Zc = Zs[:MC].contiguous()
    lib.gpr_predict_var(Z, N, Zc, MC, D, h, K, TILE, prec, True, False, cov, ws, wsb)
    lib.gpr_nlml_grad(Z, N, D, h, K, TILE, prec, alpha, (1, 1, 1), grad, ws, wsb)
    torch.cuda.synchronize()
    return dict(alpha=alpha.cpu().numpy(), nlml=float(nl.item()), mean=mean.cpu().numpy(), var=var.cpu().numpy(),
                cov=cov.cpu().numpy(), grad=grad.cpu().numpy())


@pytest.mark.parametrize("prec", ["fp32", "bf16x6", "bf16x3"])
def test_mixed_against_oracle(ref, dev_inputs, prec):
    g = _run(dev_inputs, prec)
    v_norm, v_elem, g_tol = BOUNDS[prec]
    errs = {"alpha": normwise_err(g["alpha"], ref["alpha"]), "mean": normwise_err(g["mean"], ref["mean"]),
            "mean_elem": elementwise_err(g["mean"], ref["mean"]),
            "nlml": abs(g["nlml"] - ref["nlml"]) / abs(ref["nlml"]),
            "var": normwise_err(g["var"], ref["var"]), "var_elem": elementwise_err(g["var"], ref["var"]),
            "var_maxabs": float(np.max(np.abs(g["var"] - ref["var"]))),
            "grad": normwise_err(g["grad"], ref["grad"]),
            "diag_cov_vs_var": float(np.max(np.abs(np.diag(g["cov"]) - g["var"][:MC])))}
    print(f"[mixed16384] {prec}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    assert errs["alpha"] <= 1e-6
    assert errs["mean"] <= 1e-6
    assert errs["nlml"] <= 1e-6
    assert_close(g["var"], ref["var"], v_norm, v_elem, what=f"{prec} variance")
    assert errs["grad"] <= g_tol
    assert errs["diag_cov_vs_var"] <= 1e-12 * H.signal_var


def test_bf16x3_refinement_sweeps(ref, dev_inputs):
    """The error of alpha after s sweeps of the three-product split contracts by roughly a
    constant factor per sweep; the default number of sweeps reaches the 1e-6 target."""
    errs = []
    for s in (0, 1, 2, 3, 4, 6, 8):
        g = _run(dev_inputs, "bf16x3", sweeps=s)
        errs.append((s, normwise_err(g["alpha"], ref["alpha"]), normwise_err(g["mean"], ref["mean"])))
    print("[mixed16384] bf16x3 (sweeps, alpha err, mean err): " +
          "; ".join(f"{s}: {a:.2e} {m:.2e}" for s, a, m in errs), flush=True)
    a_errs = [e[1] for e in errs]
    assert a_errs[1] < a_errs[0] and a_errs[3] < a_errs[1]
    assert dict((s, a) for s, a, _ in errs)[6] <= 1e-6
