"""Element-wise comparison used by the parity tests, next to the normwise ones."""
import numpy as np


def elementwise_err(a, b, floor: float = 1e-3) -> float:
    """max_i |a_i - b_i| / max(|b_i|, floor * max_j |b_j|): a relative error per entry,
    with entries much smaller than the largest one measured against floor times it."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    if b.size == 0:
        return 0.0
    scale = np.maximum(np.abs(b), floor * max(float(np.max(np.abs(b))), 1e-300))
    return float(np.max(np.abs(a - b) / scale))


def assert_elementwise(a, b, tol: float, floor: float = 1e-3, what: str = ""):
    e = elementwise_err(a, b, floor)
    assert e <= tol, f"{what}: element-wise error {e:.3e} > {tol:.1e}"
    return e


def normwise_err(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def assert_close(a, b, tol: float, elem_tol: float | None = None, floor: float = 1e-3, what: str = ""):
    """Normwise relative error ||a - b|| / ||b|| <= tol (the reading of "relative" for
    vectors and matrices), and the element-wise error of elementwise_err <= elem_tol,
    10 tol by default: an entry far below the largest is measured against floor times
    the largest, and a backward-stable float64 result has per-entry errors of about
    kappa u (max|b| / |b_i|) <= kappa u / floor, i.e. 1e-9 at kappa = 1e4."""
    e = normwise_err(a, b)
    assert e <= tol, f"{what}: normwise error {e:.3e} > {tol:.1e}"
    elem_tol = 10.0 * tol if elem_tol is None else elem_tol
    return e, assert_elementwise(a, b, elem_tol, floor, what)
