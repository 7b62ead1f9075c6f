"""Host model of the device-side task-graph schedule of the factorisation.

gpr_dag_check builds the graph that gpr_cholesky executes on the device (GPR_SCHEDULE_DEVICE)
and runs the executor's own claim / wait / finish code (the same source, host atomics) with
threads standing in for workgroups.  Checked here: every item starts only after all its
task's predecessors finished, every item runs exactly once and nothing gives up, whatever
the number of threads; every pair of tasks whose byte ranges overlap with one writing is
ordered by a path of edges; a dependency that can never be satisfied makes the waits give
up after the time limit and every thread return; and dropping edges is seen by the ordering
check (the check is not vacuous)."""
import pytest


@pytest.fixture(scope="module")
def lib():
    import os
    from paper_2505_00136_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgpr.so not built")
    return _lib


@pytest.mark.parametrize("n,tile", [(1024, 256), (1000, 128), (3000, 256), (700, 64), (64, 64), (8192, 1024)])
@pytest.mark.parametrize("threads", [1, 3, 16, 64])
def test_graph_runs_in_dependency_order(lib, n, tile, threads):
    r = lib.gpr_dag_check(n, tile, threads)
    assert r["tasks"] > 0 and r["items"] >= r["tasks"]
    assert r["items_run"] == r["items"]
    assert r["violations"] == 0
    assert r["aborted"] == 0 and r["timed_out"] == 0
    assert r["threads_returned"] == threads
    assert r["unordered_conflicts"] == 0


def test_full_size_graph(lib):
    """n = 65536, tile 2048: the benchmark's graph (ordering check skipped above 4096 tasks)."""
    r = lib.gpr_dag_check(65536, 2048, 32)
    assert r["items_run"] == r["items"] and r["violations"] == 0 and r["aborted"] == 0
    assert r["threads_returned"] == 32


@pytest.mark.parametrize("withhold", [0, 17, 66])
def test_unsatisfiable_dependency_gives_up(lib, withhold):
    r = lib.gpr_dag_check(1024, 256, 8, withhold=withhold, limit_ms=50.0)
    assert r["aborted"] == 1 and r["timed_out"] >= 1
    assert r["threads_returned"] == 8
    assert r["items_run"] < r["items"]
    assert r["violations"] == 0


def test_dropped_edges_are_seen(lib):
    n, tile = 1024, 256
    edges = lib.gpr_dag_check(n, tile, 2)["edges"]
    seen = sum(lib.gpr_dag_check(n, tile, 2, withhold=-2 - e)["unordered_conflicts"] > 0 for e in range(edges))
    # edges implied by others (a writer before a reader before the next writer) can go
    # unnoticed; the rest must not
    assert seen >= edges // 2
