"""Automatic tile-size selection (named as future work in Section 6) by measurement.

The tile edge b sets the task granularity of the tiled factorisation (Fig. 1): few large
tiles serialise the factorisation of the diagonal tiles, many small ones add launches.
The best b depends on n, on the device and on the precision, so the selector times the
covariance assembly and the factorisation for every candidate b on the device and
returns the fastest.  Candidates are the powers of two from 256 to 8192 below n with at
most 64 tiles per dimension (a tile that does not divide n pads the matrix with an
identity block to ceil(n / b) b rows), plus n itself (one tile, the sequential baseline
of Section 5.2), limited to those whose buffers fit in the memory budget.  Choices are cached per (device, n, d,
precision) in a JSON file.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import _lib

CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gprat_mi355x_tiles.json")


def candidate_tiles(n: int, max_tiles_per_dim: int = 64) -> list[int]:
    """256, 512, ..., 8192 below n with at most max_tiles_per_dim tiles per dimension
    (ceil(n / b), padded when b does not divide n), and n itself; ascending."""
    cands = {n}
    b = 256
    while b <= 8192:
        if b < n and -(-n // b) <= max_tiles_per_dim:
            cands.add(b)
        b *= 2
    return sorted(cands)


def _time_tile(torch, Z, n, d, b, prec, reps):
    dev = Z.device
    K = torch.empty(_lib.gpr_tiles_bytes(n, b, prec), dtype=torch.uint8, device=dev)
    wsb = _lib.gpr_workspace_size(n, 0, d, b, prec)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    h = (math.sqrt(d), 1.0, 0.01)
    ts = []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _lib.gpr_assemble(Z, n, d, h, b, prec, K)
        _lib.gpr_cholesky(K, n, b, prec, ws, wsb, want_info=False)
        torch.cuda.synchronize()
        if r:
            ts.append(time.perf_counter() - t0)
    del K, ws
    return min(ts)


def select_tile(n: int, d: int, prec: str = "fp64", Z=None, reps: int = 2, mem_gib: float = 200.0,
                use_cache: bool = True, cache_path: str = CACHE) -> tuple[int, dict]:
    """Returns (tile, {candidate: seconds}) for n points with d features.  Z (n x d,
    float64, on the device) is used when given, else standard normal inputs."""
    import torch
    dev = torch.device("cuda:0") if Z is None else Z.device
    key = f"{torch.cuda.get_device_name(dev)}|{n}|{d}|{prec}"
    if use_cache and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cached = json.load(f).get(key)
            if cached:
                return int(cached["tile"]), {int(k): v for k, v in cached["times"].items()}
        except (OSError, ValueError):
            pass
    if Z is None:
        g = torch.Generator(device="cpu").manual_seed(0)
        Z = torch.randn(n, d, generator=g, dtype=torch.float64).to(dev)
    times = {}
    for b in candidate_tiles(n):
        need = _lib.gpr_tiles_bytes(n, b, prec) + _lib.gpr_workspace_size(n, 0, d, b, prec)
        if need > mem_gib * 2 ** 30:
            continue
        times[b] = _time_tile(torch, Z, n, d, b, prec, reps)
    best = min(times, key=times.get)
    if use_cache:
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            data = {}
            if os.path.exists(cache_path):
                with open(cache_path) as f:
                    data = json.load(f)
            data[key] = {"tile": best, "times": {str(k): v for k, v in times.items()}}
            with open(cache_path, "w") as f:
                json.dump(data, f, indent=1)
        except (OSError, ValueError):
            pass
    return best, times
