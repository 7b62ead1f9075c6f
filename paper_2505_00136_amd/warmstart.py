"""Learned warm start for the hyperparameter optimisation (an addition to the paper's method).

A small network (32 -> 128 -> 128 -> 3, exact GELU) maps 32 summary statistics of a
dataset to initial log-hyperparameters theta = log(l, nu, sigma^2) for the Adam
optimisation of Section 4.1.  Everything numeric runs in the library's kernels:
the statistics (gpr_summary_stats), the network (gpr_mlp_forward /
gpr_mlp_train_step) and the labels and evaluations (gpr_optimize).  The default
initialisation theta = (0, 0, log 0.1) stays the fallback and the yardstick: the learned
initialisation is used only when its NLML is lower.

Workload: mass-spring-damper datasets with m ~ U[0.5, 2], c ~ U[0.1, 1], k ~ U[0.5, 2],
measurement noise sigma ~ U[0.01, 0.2], D uniform on {8, 16, 32, 64, 128}, 4096
training points; dataset i of the training collection uses seed 10000 + i, held-out
dataset j uses seed 20000 + j, and the 256-point subsample of the statistics uses
seed + 7.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

from . import _lib

DEFAULT_THETA = (0.0, 0.0, math.log(0.1))
N_SUB = 256
MEDIAN_STAT = 8 + 11      # quantile 12/24 of the log pairwise distances
ADAM = dict(beta1=0.9, beta2=0.999, eps=1e-8)


def make_c5_dataset(seed: int, n_train: int = 4096):
    import datagen
    p = datagen.draw_c5_params(seed)
    cfg = datagen.MSDConfig(n_train=n_train, n_test=1, D=p["D"], seed=seed, mass=p["mass"], damping=p["damping"],
                            stiffness=p["stiffness"], sigma_meas=p["sigma_meas"])
    return datagen.make_dataset(cfg), p


class Runner:
    """Device buffers reused across datasets of one size (n fixed, D up to 128)."""

    def __init__(self, n: int = 4096, tile: int = 4096, device: str = "cuda:0", max_d: int = 128):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.n, self.tile = n, tile
        self.K = torch.empty(_lib.gpr_tiles_bytes(n, tile, "fp64"), dtype=torch.uint8, device=self.dev)
        self.wsb = max(_lib.gpr_workspace_size(n, 0, max_d, tile, "fp64"), _lib.gpr_stats_workspace(N_SUB))
        self.ws = torch.empty(self.wsb, dtype=torch.uint8, device=self.dev)
        self.s64 = torch.empty(32, dtype=torch.float64, device=self.dev)
        self.s32 = torch.empty(32, dtype=torch.float32, device=self.dev)

    def upload(self, ds):
        t = lambda a: self.torch.tensor(np.ascontiguousarray(a), device=self.dev)
        return dict(Z=t(ds.Z), y=t(ds.y), Z_raw=t(ds.Z_raw), y_raw=t(ds.y_raw), d=ds.Z.shape[1])

    def stats(self, dev_ds, seed: int):
        import datagen
        idx = self.torch.tensor(datagen.subsample_indices(self.n, N_SUB, seed + 7), device=self.dev)
        _lib.gpr_summary_stats(dev_ds["Z_raw"], dev_ds["Z"], dev_ds["y_raw"], self.n, dev_ds["d"], idx, N_SUB,
                               self.s64, self.s32, self.ws, self.wsb)
        return self.s64.cpu().numpy(), self.s32.clone()

    def optimize(self, dev_ds, theta0, steps: int, lr: float):
        th, st, tr = _lib.gpr_optimize(dev_ds["Z"], dev_ds["y"], self.n, dev_ds["d"], self.tile, "fp64", theta0,
                                       (1, 1, 1), steps, lr, ADAM["beta1"], ADAM["beta2"], ADAM["eps"], None, self.K,
                                       self.ws, self.wsb)
        return np.array(th), np.array(tr)

    def nlml_at(self, dev_ds, theta):
        return float(self.optimize(dev_ds, theta, 0, 0.1)[1][0])


def median_heuristic_theta(stats64):
    """log l = log(median pairwise distance / sqrt 2), default nu and sigma^2."""
    return (float(stats64[MEDIAN_STAT]) - 0.5 * math.log(2.0), 0.0, math.log(0.1))


def make_label(runner: Runner, seed: int, steps: int = 100, lr: float = 0.1):
    """(stats64, theta label, info) for training dataset `seed`.

    The optimisation starts from whichever of the default and the median-heuristic
    initialisations has the lower NLML and runs `steps` Adam steps of the float64 method.
    """
    ds, p = make_c5_dataset(seed, runner.n)
    dd = runner.upload(ds)
    s64, _ = runner.stats(dd, seed)
    inits = [DEFAULT_THETA, median_heuristic_theta(s64)]
    f0 = [runner.nlml_at(dd, t) for t in inits]
    start = inits[int(np.argmin(f0))]
    theta, trace = runner.optimize(dd, start, steps, lr)
    return s64, theta, dict(seed=seed, D=p["D"], start=list(start), nlml0=float(trace[0]), nlml=float(trace[-1]))


@dataclass
class WarmStartModel:
    """Network parameters acting on raw statistics and producing theta directly (the
    input and label standardisation of training are folded into the first and last layer)."""
    params: np.ndarray   # float32[21123]

    def save(self, path: str):
        np.savez(path, params=self.params.astype(np.float32))

    @staticmethod
    def load(path: str) -> "WarmStartModel":
        with np.load(path, allow_pickle=False) as f:
            return WarmStartModel(params=np.asarray(f["params"], dtype=np.float32))

    def predict(self, stats32, device="cuda:0"):
        import torch
        dev = torch.device(device)
        p = torch.tensor(self.params, device=dev)
        x = stats32.reshape(1, 32).to(dev, torch.float32)
        out = torch.empty((1, 3), dtype=torch.float32, device=dev)
        wsb = _lib.gpr_mlp_workspace(1)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        _lib.gpr_mlp_forward(p, x, 1, out, ws, wsb)
        return out[0].double().cpu().numpy()


def he_normal_init(seed: int) -> np.ndarray:
    """Seeded He-normal weights (std sqrt(2 / fan_in)) and zero biases, in the parameter order."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((128, 32), (128, 128), (3, 128)):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / fan_in), size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def fold_standardisation(p_norm: np.ndarray, x_mean, x_std, y_mean, y_std) -> np.ndarray:
    """Parameters of the same network acting on raw inputs and returning raw labels."""
    p = p_norm.astype(np.float64).copy()
    W1 = p[0:4096].reshape(128, 32)
    b1 = p[4096:4224]
    W3 = p[20736:21120].reshape(3, 128)
    b3 = p[21120:21123]
    b1 -= W1 @ (x_mean / x_std)
    W1 /= x_std[None, :]
    W3 *= y_std[:, None]
    b3[:] = b3 * y_std + y_mean
    return p.astype(np.float32)


def train_model(X: np.ndarray, Y: np.ndarray, epochs: int = 300, batch: int = 128, lr: float = 1e-3, seed: int = 0,
                device: str = "cuda:0", log=None) -> tuple[WarmStartModel, list]:
    """Trains the network on the GPU with the fused train-step kernel (Adam, MSE on
    standardised inputs and labels, He-normal initialisation, seeded batch order)."""
    import torch
    dev = torch.device(device)
    x_mean, x_std = X.mean(0), X.std(0)
    x_std = np.where(x_std > 1e-12, x_std, 1.0)
    y_mean, y_std = Y.mean(0), Y.std(0)
    y_std = np.where(y_std > 1e-12, y_std, 1.0)
    Xn = torch.tensor(((X - x_mean) / x_std).astype(np.float32), device=dev)
    Yn = torch.tensor(((Y - y_mean) / y_std).astype(np.float32), device=dev)
    p = torch.tensor(he_normal_init(seed), device=dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    N = X.shape[0]
    wsb = _lib.gpr_mlp_workspace(batch)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed + 1)
    t = 0
    hist = []
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(N), device=dev)
        tot = 0.0
        for b0 in range(0, N, batch):
            idx = perm[b0:b0 + batch]
            xb = Xn.index_select(0, idx).contiguous()
            yb = Yn.index_select(0, idx).contiguous()
            t += 1
            _lib.gpr_mlp_train_step(p, m, v, t, xb, yb, idx.numel(), lr, 0.9, 0.999, 1e-8, loss, ws, wsb)
            tot += float(loss.item()) * idx.numel()
        hist.append(tot / N)
        if log and (ep % 50 == 0 or ep == epochs - 1):
            log(f"[warmstart] epoch {ep}: mse {hist[-1]:.4f}")
    params = fold_standardisation(p.cpu().numpy(), x_mean, x_std, y_mean, y_std)
    return WarmStartModel(params), hist


def choose_init(runner: Runner, dev_ds, model: WarmStartModel, stats32):
    """Learned theta if its NLML beats the default initialisation's, else the default."""
    learned = tuple(float(x) for x in model.predict(stats32, device=str(runner.dev)))
    f_l = runner.nlml_at(dev_ds, learned) if all(np.isfinite(learned)) else float("inf")
    f_d = runner.nlml_at(dev_ds, DEFAULT_THETA)
    return (learned, True, f_l, f_d) if f_l < f_d else (DEFAULT_THETA, False, f_l, f_d)


def evaluate(runner: Runner, model: WarmStartModel, seeds, steps: int = 20, lr: float = 0.1, log=None):
    """NLML/n after `steps` Adam steps from the default and from the warm-start choice."""
    rows = []
    for j, seed in enumerate(seeds):
        ds, p = make_c5_dataset(seed, runner.n)
        dd = runner.upload(ds)
        _, s32 = runner.stats(dd, seed)
        theta_ws, used, f_l, f_d = choose_init(runner, dd, model, s32)
        _, tr_d = runner.optimize(dd, DEFAULT_THETA, steps, lr)
        _, tr_w = runner.optimize(dd, theta_ws, steps, lr)
        rows.append(dict(seed=seed, D=p["D"], used_learned=bool(used), nlml0_learned=f_l / runner.n,
                         nlml0_default=f_d / runner.n, final_default=float(tr_d[-1]) / runner.n,
                         final_warm=float(tr_w[-1]) / runner.n))
        if log and (j % 10 == 0 or j == len(seeds) - 1):
            log(f"[warmstart] held-out {j + 1}/{len(seeds)}: default {rows[-1]['final_default']:.4f} "
                f"warm {rows[-1]['final_warm']:.4f}")
    return rows


def summarise(rows):
    d = np.array([r["final_default"] - r["final_warm"] for r in rows])
    out = dict(n=len(rows), mean_gain_nlml_per_n=float(d.mean()), median_gain_nlml_per_n=float(np.median(d)),
               win_rate=float(np.mean(d > 0)), learned_used_rate=float(np.mean([r["used_learned"] for r in rows])),
               per_D={})
    for D in sorted({r["D"] for r in rows}):
        sel = [r for r in rows if r["D"] == D]
        dd = np.array([r["final_default"] - r["final_warm"] for r in sel])
        out["per_D"][str(D)] = dict(n=len(sel), mean_default=float(np.mean([r["final_default"] for r in sel])),
                                    mean_warm=float(np.mean([r["final_warm"] for r in sel])),
                                    mean_gain=float(dd.mean()), win_rate=float(np.mean(dd > 0)))
    return out


MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "warmstart_mlp.npz")
