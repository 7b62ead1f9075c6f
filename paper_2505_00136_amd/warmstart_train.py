"""Warm-start pipeline: labels -> training -> held-out evaluation (run on one GPU).

    python -m paper_2505_00136_amd.warmstart_train --train-sets 2000 --heldout 200 --out DIR

Writes DIR/labels.npz (statistics and labels, extended incrementally so a long run can be
resumed), DIR/warmstart_mlp.npz (the trained network) and DIR/report.json (per-dataset
NLML/n after 20 Adam steps from the default and from the warm-start initialisation).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import warmstart as W


def log(msg):
    print(msg, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-sets", type=int, default=400)
    ap.add_argument("--heldout", type=int, default=100)
    ap.add_argument("--label-steps", type=int, default=100)
    ap.add_argument("--eval-steps", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--out", required=True)
    ap.add_argument("--skip-labels", action="store_true")
    ap.add_argument("--labels-only", action="store_true", help="extend labels.npz and stop (resumable)")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    runner = W.Runner()
    lab_path = os.path.join(args.out, "labels.npz")
    X, Y, info = [], [], []
    if os.path.exists(lab_path):
        with np.load(lab_path, allow_pickle=False) as f:
            X, Y = list(f["X"]), list(f["Y"])
            info = json.loads(str(f["info"]))
        log(f"[warmstart] resuming with {len(X)} labels")
    t0 = time.time()
    if not args.skip_labels:
        for i in range(len(X), args.train_sets):
            s64, theta, inf = W.make_label(runner, 10000 + i, steps=args.label_steps)
            X.append(s64)
            Y.append(theta)
            info.append(inf)
            if (i + 1) % 10 == 0 or i + 1 == args.train_sets:
                np.savez(lab_path, X=np.array(X), Y=np.array(Y), info=json.dumps(info))
                log(f"[warmstart] labels {i + 1}/{args.train_sets} ({time.time() - t0:.0f} s); last D={inf['D']} "
                    f"nlml {inf['nlml0']:.1f} -> {inf['nlml']:.1f}")
    if args.labels_only:
        log(f"[warmstart] {len(X)} labels in {lab_path}")
        return 0
    X, Y = np.array(X), np.array(Y)
    model, hist = W.train_model(X, Y, epochs=args.epochs, log=log)
    model.save(os.path.join(args.out, "warmstart_mlp.npz"))
    rows = W.evaluate(runner, model, [20000 + j for j in range(args.heldout)], steps=args.eval_steps, log=log)
    rep = dict(summary=W.summarise(rows), train_sets=int(X.shape[0]), label_steps=args.label_steps,
               eval_steps=args.eval_steps, epochs=args.epochs, final_train_mse=hist[-1], rows=rows)
    with open(os.path.join(args.out, "report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    log("[warmstart] summary " + json.dumps(rep["summary"]))
    return 0


if __name__ == "__main__":
    sys.exit(main())
