"""Host-side behaviour of the C-ABI on the GPU: calls that launch tile products return
while their stream is still busy (the job tables go through a ring of pinned staging
slots), the factorisation schedule is chosen by a call, and the autograd wrapper keeps
each forward's theta."""
import math
import time

import numpy as np
import pytest

import datagen
import oracle
from oracle import Hyper

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_00136_amd import _lib
    _lib.load()
    return _lib


def test_calls_return_while_the_stream_is_busy(lib):
    """gpr_cholesky, gpr_predict_var and gpr_nlml_grad queue their work and return; the
    host is not held until the GPU reaches an earlier call's table upload."""
    n, m, tile, d = 2048, 256, 256, 6
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=n, n_test=m, D=d, seed=41))
    h = (1.0, 1.0, 0.05)
    dev = "cuda:0"
    Z, Zs, y = (torch.tensor(a, device=dev) for a in (ds.Z, ds.Zs, ds.y))
    lib.gpr_init(n, m, tile, "fp64")
    K = torch.empty(lib.gpr_tiles_bytes(n, tile, "fp64"), dtype=torch.uint8, device=dev)
    wsb = lib.gpr_workspace_size(n, m, d, tile, "fp64")
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    alpha = torch.empty(n, dtype=torch.float64, device=dev)
    var = torch.empty(m, dtype=torch.float64, device=dev)
    grad = torch.empty(3, dtype=torch.float64, device=dev)
    nl = torch.empty(1, dtype=torch.float64, device=dev)

    def calls():
        lib.gpr_assemble(Z, n, d, h, tile, "fp64", K)
        lib.gpr_cholesky(K, n, tile, "fp64", ws, wsb, want_info=False)
        lib.gpr_solve(K, Z, n, d, h, tile, "fp64", y, alpha, 0, ws, wsb)
        lib.gpr_nlml(K, n, tile, "fp64", y, alpha, nl)
        lib.gpr_predict_var(Z, n, Zs, m, d, h, K, tile, "fp64", False, False, var, ws, wsb)
        lib.gpr_nlml_grad(Z, n, d, h, K, tile, "fp64", alpha, (1, 1, 1), grad, ws, wsb)

    calls()
    torch.cuda.synchronize()
    ref = (float(nl.item()), var.clone(), grad.clone())
    # occupy the stream with float64 products (several hundred milliseconds), then issue
    # two rounds of calls (eight table uploads, the ring's size) behind them
    a = torch.randn(8192, 8192, dtype=torch.float64, device=dev)
    c = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(24):
        torch.mm(a, a, out=c)
    for _ in range(2):
        calls()
    t_host = time.perf_counter() - t0
    busy = not torch.cuda.current_stream().query()
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    print(f"[boundary] host {t_host * 1e3:.1f} ms, stream drained after {t_all * 1e3:.1f} ms", flush=True)
    assert busy, "the calls returned only after the stream had drained"
    assert t_host < 0.5 * t_all
    assert float(nl.item()) == ref[0]
    assert torch.equal(var, ref[1]) and torch.equal(grad, ref[2])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "bf16x3"])
def test_lookahead_switch(lib, prec):
    """gpr_set_lookahead(0) and (1) give the same bits, in every precision, and repeated
    look-ahead factorisations agree."""
    n, tile, d = 1536, 256, 5
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=n, n_test=4, D=d, seed=42))
    dev = "cuda:0"
    Z = torch.tensor(ds.Z, device=dev)
    wsb = lib.gpr_workspace_size(n, 0, d, tile, prec)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    out = []
    for la in (False, True, True):
        K = torch.empty(lib.gpr_tiles_bytes(n, tile, prec), dtype=torch.uint8, device=dev)
        lib.gpr_set_lookahead(la)
        try:
            lib.gpr_assemble(Z, n, d, (1.1, 0.9, 0.03), tile, prec, K)
            assert lib.gpr_cholesky(K, n, tile, prec, ws, wsb) == 0
        finally:
            lib.gpr_set_lookahead(True)
        out.append(K)
    assert torch.equal(out[0], out[1]) and torch.equal(out[1], out[2])


def test_autograd_two_forwards_then_two_backwards(lib):
    """Each backward differentiates at its own forward's theta, whatever the GP was
    refitted at in between, and returns all three entries whatever the trainable flags."""
    from paper_2505_00136_amd.gp import GP, nlml
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=700, n_test=4, D=4, seed=43))
    gp = GP(ds.Z, ds.y, hyper=(1.0, 1.0, 0.1), tile=128, trainable=(0, 1, 1))
    thetas = [np.log([1.3, 0.8, 0.05]), np.log([0.7, 1.4, 0.2])]
    ts = [torch.tensor(t, dtype=torch.float64, requires_grad=True) for t in thetas]
    losses = [nlml(t, gp) for t in ts]
    for loss in reversed(losses):
        loss.backward()
    for t, th, loss in zip(ts, thetas, losses):
        h = Hyper(*np.exp(th))
        L, a, f = oracle.fit(ds.Z, ds.y, h)
        assert float(loss.item()) == pytest.approx(f, rel=1e-10)
        g = oracle.nlml_grad(ds.Z, h, L, a)
        assert np.all(g != 0)
        np.testing.assert_allclose(t.grad.numpy(), g, rtol=1e-9, atol=1e-12 * np.max(np.abs(g)))
    # a backward after an optimisation of the same GP still uses its own theta
    t3 = torch.tensor(thetas[0], dtype=torch.float64, requires_grad=True)
    l3 = nlml(t3, gp)
    gp.optimize(2, lr=0.05)
    l3.backward()
    np.testing.assert_allclose(t3.grad.numpy(), ts[0].grad.numpy(), rtol=1e-12)
    assert math.isfinite(float(l3.item()))
