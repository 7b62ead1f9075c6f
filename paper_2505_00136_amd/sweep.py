"""Problem-size x tile-count sweep of the exact GP path on one GPU (the experiment of
Section 5.2, Figs. 5-7: N = M = 2^3 .. 2^17, 1, 4 and 16 tiles per dimension, eight
lagged inputs, float64).

For every (N, tiles per dimension) it times three calls sequences, each starting from
the training inputs resident in device memory, as the paper's library calls do:

* ``opt``: hyperparameter optimisation, ``gpr_optimize`` with a fixed number of Adam
  steps (each: assembly, Cholesky, alpha, NLML, gradient) from theta = (0, 0, log 0.1);
* ``pred_full``: prediction with the full posterior covariance (assembly, Cholesky,
  alpha, mean, M x M covariance);
* ``pred_var``: the same with the variance only.

Each case is run once untimed, then repeated until about a second has been timed (at
most 5 repetitions); the median wall time (host clock around a synchronised call
sequence) is reported.  Cases whose buffers would not fit in the memory budget are
skipped.  Prints one JSON object per case; ``--out`` also writes them to a file.

Usage: ``python -m paper_2505_00136_amd.sweep --max-log2 16 --tiles 1,4,16``
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from . import _lib  # noqa: E402

D = 8
THETA0 = (0.0, 0.0, math.log(0.1))
ADAM = (0.9, 0.999, 1e-8)


def _timed(torch, fn, budget_s=1.0, max_reps=5):
    fn()
    torch.cuda.synchronize()
    ts = []
    while len(ts) < max_reps and sum(ts) < budget_s:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), len(ts)


def run_case(torch, N, tpd, opt_steps, mem_budget):
    import datagen
    b = N // tpd
    dev = torch.device("cuda:0")
    kb = _lib.gpr_tiles_bytes(N, b, "fp64")
    wsb = _lib.gpr_workspace_size(N, N, D, b, "fp64")
    need = kb + wsb + N * N * 8
    if need > mem_budget:
        return dict(N=N, tiles_per_dim=tpd, tile=b, skipped=f"needs {need / 2**30:.1f} GiB")
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=N, n_test=N, D=D, seed=5))
    Z = torch.tensor(ds.Z, device=dev)
    Zs = torch.tensor(ds.Zs, device=dev)
    y = torch.tensor(ds.y, device=dev)
    K = torch.empty(kb, dtype=torch.uint8, device=dev)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    alpha = torch.empty(N, dtype=torch.float64, device=dev)
    mean = torch.empty(N, dtype=torch.float64, device=dev)
    var = torch.empty(N, dtype=torch.float64, device=dev)
    cov = torch.empty((N, N), dtype=torch.float64, device=dev)
    h = tuple(math.exp(t) for t in THETA0)

    def opt():
        _lib.gpr_optimize(Z, y, N, D, b, "fp64", THETA0, (1, 1, 1), opt_steps, 0.1, *ADAM, None, K, ws, wsb)

    def pred(full):
        def f():
            _lib.gpr_assemble(Z, N, D, h, b, "fp64", K)
            _lib.gpr_cholesky(K, N, b, "fp64", ws, wsb, want_info=False)
            _lib.gpr_solve(K, Z, N, D, h, b, "fp64", y, alpha, 0, ws, wsb)
            _lib.gpr_predict(Z, N, Zs, N, D, h, alpha, mean, ws, wsb)
            _lib.gpr_predict_var(Z, N, Zs, N, D, h, K, b, "fp64", full, False, cov if full else var, ws, wsb)
        return f

    row = dict(N=N, tiles_per_dim=tpd, tile=b)
    for name, fn in (("opt", opt), ("pred_full", pred(True)), ("pred_var", pred(False))):
        t, reps = _timed(torch, fn)
        row[name + "_s"] = t
        row[name + "_reps"] = reps
    del K, ws, cov
    torch.cuda.empty_cache()
    return row


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--min-log2", type=int, default=3)
    ap.add_argument("--max-log2", type=int, default=16)
    ap.add_argument("--tiles", default="1,4,16")
    ap.add_argument("--opt-steps", type=int, default=10)
    ap.add_argument("--mem-gib", type=float, default=200.0)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the sweep runs on the GPU")
    _lib.load()
    out = open(args.out, "w") if args.out else None
    for p in range(args.min_log2, args.max_log2 + 1):
        N = 1 << p
        for tpd in (int(t) for t in args.tiles.split(",")):
            if tpd > N or N % tpd:
                continue
            row = run_case(torch, N, tpd, args.opt_steps, args.mem_gib * 2**30)
            line = json.dumps(row)
            print(line, flush=True)
            if out:
                out.write(line + "\n")
                out.flush()
    if out:
        out.close()


if __name__ == "__main__":
    main()
