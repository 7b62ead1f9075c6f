"""Problem-size x tile-count sweep of the exact GP path on one GPU (the experiment of
Section 5.2, Figs. 5-7: N = M = 2^3 .. 2^17, 1, 4 and 16 tiles per dimension, eight
lagged inputs, float64).

For every (N, tiles per dimension) it times three calls sequences, each starting from
the training inputs resident in device memory, as the paper's library calls do:

* ``opt``: hyperparameter optimisation, ``gpr_optimize`` with a fixed number of Adam
  steps (each: assembly, Cholesky, alpha, NLML, gradient) from theta = (0, 0, log 0.1);
  from N = 2^16 on a smaller number of steps (``--opt-steps-large``), whose time is also
  reported per step;
* ``pred_full``: prediction with the full posterior covariance (assembly, Cholesky,
  alpha, mean, M x M covariance);
* ``pred_var``: the same with the variance only.

Each case is run once untimed, then repeated until about a second has been timed (at
most 5 repetitions); the median wall time (host clock around a synchronised call
sequence) is reported.  From N = 2^16 on a case is timed once, without the untimed run.
Each sequence allocates what it needs (tiled matrix, workspace, the M x M output of the
full covariance) and is skipped when that exceeds the memory budget: at N = M = 2^17 the
full covariance (137 GB) with the cross-covariance solve (137 GB) and the factor (73 GB)
exceeds the 288 GB of one GPU, and one tile per dimension needs 275 GB for the diagonal
tile and its inverse alone.  Prints one JSON object per case and a progress line per
sequence; ``--out`` also writes the objects to a file.

Usage: ``python -m paper_2505_00136_amd.sweep --max-log2 16 --tiles 1,4,16 --d 8``
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

THETA0 = (0.0, 0.0, math.log(0.1))
ADAM = (0.9, 0.999, 1e-8)
LARGE = 1 << 16


def _timed(torch, fn, budget_s=1.0, max_reps=5, warm=True):
    if warm:
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_case(torch, N, tpd, D, opt_steps, mem_budget):
    import datagen
    b = N // tpd
    dev = torch.device("cuda:0")
    kb = _lib.gpr_tiles_bytes(N, b, "fp64")
    need = {"opt": kb + _lib.gpr_workspace_size(N, 0, D, b, "fp64"),
            "pred_var": kb + _lib.gpr_workspace_size(N, N, D, b, "fp64")}
    need["pred_full"] = need["pred_var"] + N * N * 8
    row = dict(N=N, tiles_per_dim=tpd, tile=b, D=D)
    if need["opt"] > mem_budget:
        row["skipped"] = f"needs {need['opt'] / 2**30:.1f} GiB"
        return row
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=N, n_test=N, D=D, seed=5))
    Z = torch.tensor(ds.Z, device=dev)
    Zs = torch.tensor(ds.Zs, device=dev)
    y = torch.tensor(ds.y, device=dev)
    alpha = torch.empty(N, dtype=torch.float64, device=dev)
    mean = torch.empty(N, dtype=torch.float64, device=dev)
    var = torch.empty(N, dtype=torch.float64, device=dev)
    h = tuple(math.exp(t) for t in THETA0)
    large = N >= LARGE
    steps = opt_steps

    for name in ("opt", "pred_full", "pred_var"):
        if need[name] > mem_budget:
            row[name + "_skipped"] = f"needs {need[name] / 2**30:.1f} GiB"
            continue
        m = 0 if name == "opt" else N
        wsb = _lib.gpr_workspace_size(N, m, D, b, "fp64")
        K = torch.empty(kb, dtype=torch.uint8, device=dev)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        cov = torch.empty((N, N), dtype=torch.float64, device=dev) if name == "pred_full" else None
        _lib.gpr_init(N, m, b, "fp64")

        if name == "opt":
            def fn():
                _lib.gpr_optimize(Z, y, N, D, b, "fp64", THETA0, (1, 1, 1), steps, 0.1, *ADAM, None, K, ws, wsb)
        else:
            full = name == "pred_full"

            def fn():
                _lib.gpr_assemble(Z, N, D, h, b, "fp64", K)
                _lib.gpr_cholesky(K, N, b, "fp64", ws, wsb, want_info=False)
                _lib.gpr_solve(K, Z, N, D, h, b, "fp64", y, alpha, 0, ws, wsb)
                _lib.gpr_predict(Z, N, Zs, N, D, h, alpha, mean, ws, wsb)
                _lib.gpr_predict_var(Z, N, Zs, N, D, h, K, b, "fp64", full, False, cov if full else var, ws, wsb)
        log(f"[sweep] N={N} tiles={tpd} D={D}: {name} start")
        t, reps = _timed(torch, fn, warm=not large)
        row[name + "_s"] = t
        row[name + "_reps"] = reps
        if name == "opt":
            row["opt_steps"] = steps
            row["opt_s_per_step"] = t / max(steps, 1)
        log(f"[sweep] N={N} tiles={tpd} D={D}: {name} {t:.4g} s")
        del K, ws, cov
        torch.cuda.empty_cache()
    return row


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--min-log2", type=int, default=3)
    ap.add_argument("--max-log2", type=int, default=16)
    ap.add_argument("--tiles", default="1,4,16")
    ap.add_argument("--opt-steps", type=int, default=10)
    ap.add_argument("--opt-steps-large", type=int, default=2, help="Adam steps timed from N = 2^16 on")
    ap.add_argument("--d", type=int, default=8, help="lagged inputs (features)")
    ap.add_argument("--mem-gib", type=float, default=270.0)
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
            steps = args.opt_steps if N < LARGE else args.opt_steps_large
            row = run_case(torch, N, tpd, args.d, steps, args.mem_gib * 2**30)
            line = json.dumps(row)
            print(line, flush=True)
            if out:
                out.write(line + "\n")
                out.flush()
    if out:
        out.close()


if __name__ == "__main__":
    main()
