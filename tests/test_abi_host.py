"""Host-side checks of the C-ABI library: it loads, exports every declared entry point,
and rejects bad arguments before touching the GPU."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "gpr.h")).read()
    return sorted(set(re.findall(r"GPR_API\s+[\w\s\*]+?\b(gpr_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2505_00136_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgpr.so not built")
    return _lib


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 13
    so = lib.load()
    for n in names:
        assert hasattr(so, n), n
    assert set(names) <= set(lib.exported_symbols())


def test_version_and_sizes(lib):
    assert lib.gpr_version() >> 16 == 1
    n, b = 1024, 256
    T = n // b
    assert lib.gpr_tiles_bytes(n, b, "fp64") == 2 * T * b * b * 8 + T * (T - 1) // 2 * b * b * 8
    assert lib.gpr_tiles_bytes(n, b, "fp32") == 2 * T * b * b * 8 + T * (T - 1) // 2 * b * b * 4
    assert lib.gpr_workspace_size(n, 512, 8, b, "fp64") > 0


def test_argument_errors(lib):
    with pytest.raises(lib.GprError) as e:
        lib.gpr_tiles_bytes(-1000, 256, "fp64")
    assert e.value.code == lib.GPR_ERR_SHAPE
    with pytest.raises(lib.GprError) as e:
        lib.gpr_tiles_bytes(1024, 0, "fp64")
    assert e.value.code == lib.GPR_ERR_SHAPE
    with pytest.raises(lib.GprError) as e:
        lib.gpr_tiles_bytes(1024, 256, 9)
    assert e.value.code == lib.GPR_ERR_ARG
    for h in [(0.0, 1.0, 0.1), (1.0, -1.0, 0.1), (1.0, 1.0, -0.1), (float("nan"), 1.0, 0.1), (1.0, float("inf"), 0.1)]:
        with pytest.raises(lib.GprError) as e:
            lib.gpr_assemble(0x1000, 16, 2, h, 4, "fp64", 0x2000, stream=0)
        assert e.value.code == lib.GPR_ERR_ARG
    with pytest.raises(lib.GprError) as e:
        lib.gpr_assemble(0x1000, -18, 2, (1.0, 1.0, 0.1), 4, "fp64", 0x2000, stream=0)
    assert e.value.code == lib.GPR_ERR_SHAPE
    with pytest.raises(lib.GprError) as e:
        lib.gpr_cholesky(0x2000, 16, 4, "fp64", 0x3000, 16, stream=0)
    assert e.value.code == lib.GPR_ERR_WORKSPACE
    with pytest.raises(lib.GprError) as e:
        lib.gpr_solve(0x2000, None, 16, 2, (1.0, 1.0, 0.1), 4, "fp64", 0x10, 0x10, 0, 0x3000, 1 << 30, stream=0)
    assert e.value.code == lib.GPR_ERR_ARG


def test_census_matches_fig1(lib):
    import math
    assert lib.gpr_cholesky_census(4) == dict(potrf=4, trsm=6, syrk=6, gemm=4)
    for T in (1, 4, 16, 32):
        c = lib.gpr_cholesky_census(T)
        assert c == dict(potrf=T, trsm=math.comb(T, 2), syrk=math.comb(T, 2), gemm=math.comb(T, 3))


# ------------------------------------------------ dependency order of the two-stream schedule
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_cholesky_schedule_has_no_unordered_conflicts(lib, prec):
    """Every pair of launches on different streams that touch common bytes (one writing)
    is ordered by an event, for 1..24 tiles of 128 and of 256 (1 and 4 inner blocks), and
    the look-ahead really overlaps work (concurrent pairs exist from 3 tiles on)."""
    for b in (64, 128, 256):
        for T in list(range(1, 13)) + [17, 24]:
            r = lib.gpr_cholesky_schedule_check(T * b, b, prec)
            assert r["conflicts"] == 0, (b, T, r)
            assert r["unannotated"] == 0 and r["early_waits"] == 0, (b, T, r)
            assert r["launches_main"] >= 1 and r["launches_aux"] >= 1
            if T >= 3:
                assert r["concurrent_pairs"] > 0, (b, T, r)
            # per step: e1 (auxiliary; and e0 in the mixed modes), e2 (caller's); start and end
            assert r["waits"] == (2 * T if prec == "fp64" else 3 * T - 1)


@pytest.mark.parametrize("prec", ["fp64", "bf16x6"])
def test_cholesky_schedule_every_wait_is_needed(lib, prec):
    """The check is not vacuous: dropping the waits on any one event that the schedule
    waits for leaves a conflicting pair unordered."""
    T, b = 8, 128
    assert lib.gpr_cholesky_schedule_check(T * b, b, prec)["conflicts"] == 0
    # event 0: start; 1 + 3k: diagonal tile k+1 updated by step k; 2 + 3k: the rest of
    # block column k+1 updated; 3 + 3k: panel k solved
    # (the last step's U1 covers no tile -- block column T-1 has none below its diagonal
    # tile -- so its event 2 + 3(T-2) orders nothing beyond event 1 + 3(T-2))
    waited = [0] + [3 + 3 * k for k in range(T)]
    if prec == "fp64":   # one update launch for block column k+1: the diagonal tile waits for e1
        waited += [2 + 3 * k for k in range(T - 1)]
    else:
        waited += [1 + 3 * k for k in range(T - 1)] + [2 + 3 * k for k in range(T - 2)]
    for ev in waited:
        r = lib.gpr_cholesky_schedule_check(T * b, b, prec, ev)
        assert r["conflicts"] > 0, (ev, r)
    # an event nobody waits for changes nothing
    assert lib.gpr_cholesky_schedule_check(T * b, b, prec, 1 + 3 * (T - 1))["conflicts"] == 0


def test_cholesky_schedule_check_arguments(lib):
    assert lib.gpr_cholesky_schedule_check(0, 4, "fp64")["launches"] == 0
    with pytest.raises(lib.GprError) as e:
        lib.gpr_cholesky_schedule_check(100, 0, "fp64")
    assert e.value.code == lib.GPR_ERR_SHAPE
    # a tile that does not divide n: the padded matrix has ceil(n / tile) tiles per dimension
    assert lib.gpr_cholesky_schedule_check(100, 64, "fp64") == lib.gpr_cholesky_schedule_check(128, 64, "fp64")


def test_unknown_kernel_is_rejected_before_the_gpu(lib):
    for bad in (-1, 4, 9):
        with pytest.raises(lib.GprError) as e:
            lib.gpr_assemble(0x1000, 16, 2, (1.0, 1.0, 0.1, bad), 4, "fp64", 0x2000, stream=0)
        assert e.value.code == lib.GPR_ERR_ARG
    with pytest.raises(lib.GprError) as e:
        lib.gpr_optimize(0x1000, 0x1000, 16, 2, 4, "fp64", (0.0, 0.0, -2.0), (1, 1, 1), 1, 0.1, 0.9, 0.999, 1e-8,
                         None, 0x2000, 0x3000, 1 << 30, stream=0, kernel=5)
    assert e.value.code == lib.GPR_ERR_ARG
    assert lib.hyper((1.0, 2.0, 0.5, "matern32")).kernel == 2 and lib.hyper((1.0, 2.0, 0.5)).kernel == 0


def test_tile_candidates():
    from paper_2505_00136_amd.tile_select import candidate_tiles
    assert candidate_tiles(65536) == [1024, 2048, 4096, 8192, 65536]
    assert candidate_tiles(4096) == [256, 512, 1024, 2048, 4096]
    assert candidate_tiles(1000) == [256, 512, 1000]
    assert candidate_tiles(8) == [8]
    assert candidate_tiles(50000) == [1024, 2048, 4096, 8192, 50000]
    for n in (1024, 3072, 16384, 98304, 12345):
        assert all(b == n or (b < n and -(-n // b) <= 64) for b in candidate_tiles(n))


def test_padded_sizes(lib):
    """A tile that does not divide n pads the matrix to T = ceil(n / tile) tiles."""
    for n, b in [(1000, 256), (77, 128), (300, 100), (1, 64)]:
        T = -(-n // b)
        for prec, es in (("fp64", 8), ("fp32", 4)):
            assert lib.gpr_tiles_bytes(n, b, prec) == 2 * T * b * b * 8 + T * (T - 1) // 2 * b * b * es
        assert lib.gpr_workspace_size(n, 16, 3, b, "fp64") > 0
