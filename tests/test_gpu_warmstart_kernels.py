"""GPU parity of the warm-start kernels (summary statistics, network forward/backward/Adam)
against the FP64 oracle.  The statistics are float64 (tolerance 1e-12); the network is
float32 (forward 1e-5, gradient 1e-4 relative in norm)."""
import numpy as np
import pytest

import datagen
import oracle

from tests.checks import assert_elementwise  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from tests.test_gpu_parity import lib  # noqa: E402,F401

DEV = "cuda:0"


@pytest.mark.parametrize("n,D,nsub", [(1000, 8, 256), (600, 128, 256), (50, 3, 7)])
def test_summary_stats_parity(lib, n, D, nsub):
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=n, n_test=1, D=D, seed=n + D))
    idx = datagen.subsample_indices(n, nsub, 99)
    want = oracle.summary_stats(ds.Z_raw, ds.Z, ds.y_raw, idx)
    t = lambda a: torch.tensor(a, device=DEV)
    s64 = torch.empty(32, dtype=torch.float64, device=DEV)
    s32 = torch.empty(32, dtype=torch.float32, device=DEV)
    wsb = lib.gpr_stats_workspace(nsub)
    ws = torch.empty(wsb, dtype=torch.uint8, device=DEV)
    lib.gpr_summary_stats(t(ds.Z_raw), t(ds.Z), t(ds.y_raw), n, D, t(idx), nsub, s64, s32, ws, wsb)
    torch.cuda.synchronize()
    np.testing.assert_allclose(s64.cpu().numpy(), want, rtol=1e-12, atol=1e-13)
    np.testing.assert_array_equal(s32.cpu().numpy(), s64.cpu().numpy().astype(np.float32))


def _params(seed):
    p = oracle.mlp_init(seed)
    p[4096:4096 + 128] = np.random.default_rng(seed).normal(0, 0.1, 128)
    return p


def test_mlp_forward_and_gradient_parity(lib):
    rng = np.random.default_rng(3)
    B = 128
    p = _params(7)
    X = rng.normal(size=(B, 32))
    Y = rng.normal(size=(B, 3))
    assert lib.gpr_mlp_nparams() == oracle.N_PARAMS
    pt = torch.tensor(p, dtype=torch.float32, device=DEV)
    Xt = torch.tensor(X, dtype=torch.float32, device=DEV)
    Yt = torch.tensor(Y, dtype=torch.float32, device=DEV)
    wsb = lib.gpr_mlp_workspace(B)
    ws = torch.empty(wsb, dtype=torch.uint8, device=DEV)
    out = torch.empty((B, 3), dtype=torch.float32, device=DEV)
    lib.gpr_mlp_forward(pt, Xt, B, out, ws, wsb)
    # the oracle runs on the float32-rounded inputs so only the arithmetic differs
    p32, X32, Y32 = (a.astype(np.float32).astype(np.float64) for a in (p, X, Y))
    np.testing.assert_allclose(out.cpu().numpy(), oracle.mlp_forward(p32, X32), rtol=1e-5, atol=1e-5)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    grad = torch.empty(oracle.N_PARAMS, dtype=torch.float32, device=DEV)
    lib.gpr_mlp_loss_grad(pt, Xt, Yt, B, loss, grad, ws, wsb)
    lo, go = oracle.mlp_loss_and_grad(p32, X32, Y32)
    assert loss.item() == pytest.approx(lo, rel=1e-5)
    g = grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(g - go) / np.linalg.norm(go) < 1e-4
    for blk in (slice(0, 4096), slice(4096, 4224), slice(4224, 20608), slice(20608, 20736), slice(20736, 21123)):
        assert np.linalg.norm(g[blk] - go[blk]) / max(np.linalg.norm(go[blk]), 1e-30) < 1e-4
        # per entry, within each layer's weights or biases: float32 accumulation over the
        # batch and the layer width (~128 terms) against the float64 oracle
        assert_elementwise(g[blk], go[blk], 1e-3, what=f"mlp gradient {blk}")


def test_mlp_train_step_adam(lib):
    rng = np.random.default_rng(4)
    B = 64
    p = _params(8)
    X = rng.normal(size=(B, 32))
    Y = rng.normal(size=(B, 3))
    pt = torch.tensor(p, dtype=torch.float32, device=DEV)
    m = torch.zeros(oracle.N_PARAMS, dtype=torch.float32, device=DEV)
    v = torch.zeros(oracle.N_PARAMS, dtype=torch.float32, device=DEV)
    wsb = lib.gpr_mlp_workspace(B)
    ws = torch.empty(wsb, dtype=torch.uint8, device=DEV)
    Xt = torch.tensor(X, dtype=torch.float32, device=DEV)
    Yt = torch.tensor(Y, dtype=torch.float32, device=DEV)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    pr = p.astype(np.float32).astype(np.float64)
    mr, vr = np.zeros(oracle.N_PARAMS), np.zeros(oracle.N_PARAMS)
    losses = []
    for t in range(1, 4):
        lib.gpr_mlp_train_step(pt, m, v, t, Xt, Yt, B, 1e-3, 0.9, 0.999, 1e-8, loss, ws, wsb)
        losses.append(loss.item())
        _, go = oracle.mlp_loss_and_grad(pr, X.astype(np.float32), Y.astype(np.float32))
        pr, mr, vr = oracle.mlp_adam_step(pr, go, mr, vr, t)
    # first Adam steps move each parameter by about lr * sign(g): compare the displacement
    disp_gpu = pt.cpu().numpy().astype(np.float64) - p.astype(np.float32).astype(np.float64)
    disp_ref = pr - p.astype(np.float32).astype(np.float64)
    big = np.abs(disp_ref) > 1e-3
    assert big.mean() > 0.5
    np.testing.assert_allclose(disp_gpu[big], disp_ref[big], rtol=2e-3, atol=2e-6)
    assert losses[-1] < losses[0]
