"""The device-side task-graph schedule of the factorisation (GPR_SCHEDULE_DEVICE) on the GPU.

The graph's items run the same tile-product, diagonal-block, copy and transpose code as the
stream schedules and every tile receives its updates in ascending step order, so the factor
(regions D, W and O), alpha and the NLML are the same bits as the one-stream schedule; they
are also checked against the oracle.  A non-positive pivot is reported as with the streams,
and the mixed precisions (which have no task form) fall back to the look-ahead."""
import math

import numpy as np
import pytest

import datagen
import oracle
from oracle import Hyper

from tests.checks import assert_close  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_00136_amd import _lib
    _lib.load()
    yield _lib
    _lib.gpr_set_schedule("lookahead")


def _factor(lib, Z, y, h, tile, schedule, prec="fp64"):
    dev = "cuda:0"
    n, d = Z.shape
    Zt, yt = torch.tensor(Z, device=dev), torch.tensor(y, device=dev)
    K = torch.empty(lib.gpr_tiles_bytes(n, tile, prec), dtype=torch.uint8, device=dev)
    wsb = lib.gpr_workspace_size(n, 0, d, tile, prec)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    alpha = torch.empty(n, dtype=torch.float64, device=dev)
    nl = torch.empty(1, dtype=torch.float64, device=dev)
    lib.gpr_set_schedule(schedule)
    try:
        lib.gpr_assemble(Zt, n, d, h, tile, prec, K)
        info = lib.gpr_cholesky(K, n, tile, prec, ws, wsb)
    finally:
        lib.gpr_set_schedule("lookahead")
    assert info == 0
    lib.gpr_solve(K, Zt, n, d, h, tile, prec, yt, alpha, -1, ws, wsb)
    lib.gpr_nlml(K, n, tile, prec, yt, alpha, nl)
    torch.cuda.synchronize()
    return K, alpha, float(nl.item())


@pytest.mark.parametrize("n,tile,d", [(1024, 256, 8), (3000, 256, 6), (1000, 128, 5), (700, 64, 4), (64, 64, 3),
                                      (5000, 1024, 8)])
def test_device_schedule_matches_streams_bitwise(lib, n, tile, d):
    print(f"[device-schedule] n={n} tile={tile} d={d}", flush=True)
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=n, n_test=4, D=d, seed=60 + d))
    h = Hyper(1.0, 1.0, 0.02)
    K0, a0, f0 = _factor(lib, ds.Z, ds.y, h, tile, "stream")
    K1, a1, f1 = _factor(lib, ds.Z, ds.y, h, tile, "device")
    K2, a2, f2 = _factor(lib, ds.Z, ds.y, h, tile, "device")
    assert torch.equal(K1, K0) and torch.equal(a1, a0) and f1 == f0
    assert torch.equal(K2, K1)
    L, a, f = oracle.fit(ds.Z, ds.y, h)
    assert_close(a1.cpu().numpy(), a, 1e-10, what="alpha")
    assert abs(f1 - f) <= 1e-10 * abs(f)


def test_device_schedule_at_16384(lib):
    """16 x 16 tiles of 1024: the whole-macro-tile main loops and 949 tasks."""
    n, tile, d = 16384, 1024, 8
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=n, n_test=4, D=d, seed=2))
    h = Hyper(1.0, 1.0, 0.1)
    K0, a0, f0 = _factor(lib, ds.Z, ds.y, h, tile, "lookahead")
    K1, a1, f1 = _factor(lib, ds.Z, ds.y, h, tile, "device")
    assert torch.equal(K1, K0) and torch.equal(a1, a0) and f1 == f0


def test_device_schedule_reports_not_spd(lib):
    rng = np.random.default_rng(4)
    n, tile, D = 256, 64, 3
    Z = rng.normal(size=(n, D))
    h = Hyper(1.0, 1.0, 0.1)
    dev = "cuda:0"
    for col in (1, 70, 256):
        Zt = torch.tensor(Z, device=dev)
        K = torch.empty(lib.gpr_tiles_bytes(n, tile, "fp64"), dtype=torch.uint8, device=dev)
        wsb = lib.gpr_workspace_size(n, 0, D, tile, "fp64")
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        lib.gpr_assemble(Zt, n, D, h, tile, "fp64", K)
        k, r = (col - 1) // tile, (col - 1) % tile
        K.view(torch.float64)[k * tile * tile + r * tile + r] = -3.0
        lib.gpr_set_schedule("device")
        try:
            info = lib.gpr_cholesky(K, n, tile, "fp64", ws, wsb)
        finally:
            lib.gpr_set_schedule("lookahead")
        assert info == col


def test_mixed_precision_falls_back_to_the_lookahead(lib):
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=2048, n_test=4, D=8, seed=65))
    h = Hyper(math.sqrt(8), 1.0, 0.01)
    K0, a0, _ = _factor(lib, ds.Z, ds.y, h, 256, "lookahead", prec="fp32")
    K1, a1, _ = _factor(lib, ds.Z, ds.y, h, 256, "device", prec="fp32")
    assert torch.equal(K1, K0) and torch.equal(a1, a0)
