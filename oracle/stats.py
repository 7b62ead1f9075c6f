"""FP64 oracle of the warm-start summary statistics (test infrastructure).

32 numbers per dataset, the input of the warm-start network:
* s[0:8]   quantiles at 0, 1/7, ..., 1 of the D per-feature variances
           (population variance) of the raw, unstandardised features;
* s[8:31]  quantiles at k/24, k = 1..23, of the log Euclidean distance over all
           pairs i < j of a seeded subsample (given as row indices) of the
           standardised features;
* s[31]    log of the population variance of the raw targets.
Quantiles use linear interpolation between order statistics (position
q (n - 1) in the sorted sample).
"""
from __future__ import annotations

import numpy as np

N_STATS = 32


def _quantile_linear(x: np.ndarray, qs) -> np.ndarray:
    xs = np.sort(np.asarray(x, dtype=np.float64))
    n = xs.shape[0]
    out = []
    for q in qs:
        h = q * (n - 1)
        lo = int(np.floor(h))
        hi = min(lo + 1, n - 1)
        out.append(xs[lo] + (h - lo) * (xs[hi] - xs[lo]))
    return np.array(out)


def summary_stats(Z_raw: np.ndarray, Z_std: np.ndarray, y_raw: np.ndarray, sub_idx: np.ndarray) -> np.ndarray:
    Z_raw = np.asarray(Z_raw, dtype=np.float64)
    var = Z_raw.var(axis=0)
    s_var = _quantile_linear(var, [k / 7.0 for k in range(8)])
    P = np.asarray(Z_std, dtype=np.float64)[np.asarray(sub_idx)]
    m = P.shape[0]
    logd = []
    for i in range(m):
        diff = P[i + 1:] - P[i]
        logd.append(0.5 * np.log(np.einsum("jd,jd->j", diff, diff)))
    logd = np.concatenate(logd)
    s_dist = _quantile_linear(logd, [k / 24.0 for k in range(1, 24)])
    s_y = np.log(np.asarray(y_raw, dtype=np.float64).var())
    return np.concatenate([s_var, s_dist, [s_y]])
