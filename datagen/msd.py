"""Mass-spring-damper (MSD) system-identification data with lagged-input regressors.

The paper (Section 5) measures on a simulated mass-spring-damper system whose
feature vectors are lagged system inputs ("regressors"), with 8 regressors in
the figures and up to 128 in the text.  Its dataset is not available here, so a
synthetic linear MSD stands in, with the shapes of the paper's workloads:

* dynamics  m x'' = u - c x' - k x, state s = (x, v), v = x';
* classic fourth-order Runge-Kutta with step dt; the input u_t is held constant
  over the step that starts at sample t (zero-order hold);
* u_t ~ i.i.d. Uniform[-1, 1]; a burn-in prefix is discarded;
* target y_t = x_t + eps_t, eps_t ~ N(0, sigma_meas^2);
* features z_t = (u_{t-1}, ..., u_{t-D}) (column j holds u_{t-1-j});
* one trajectory gives the training samples first and the test samples next
  (a time-series split); features and targets are standardised with the
  training mean and population standard deviation, and the same shift/scale is
  applied to the test set.

Random draws come from ``numpy.random.default_rng(seed)``: all inputs u first,
then all measurement noise.  Everything is float64.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class MSDConfig:
    n_train: int
    n_test: int
    D: int
    seed: int
    mass: float = 1.0
    damping: float = 0.4
    stiffness: float = 1.0
    sigma_meas: float = 0.1
    dt: float = 0.1
    burn_in: int = 1000


@dataclass
class Dataset:
    Z: np.ndarray        # (n_train, D) standardised features, float64, C-contiguous
    y: np.ndarray        # (n_train,) standardised targets
    Zs: np.ndarray       # (n_test, D) test features, standardised with the training stats
    ys: np.ndarray       # (n_test,) test targets, standardised with the training stats
    Z_raw: np.ndarray    # (n_train, D) unstandardised training features
    y_raw: np.ndarray    # (n_train,) unstandardised training targets
    config: MSDConfig = field(repr=False, default=None)


def _rhs(x, v, u, m, c, k):
    return v, (u - c * v - k * x) / m


def simulate_msd(u: np.ndarray, mass, damping, stiffness, dt: float) -> np.ndarray:
    """Positions x_t (t = 0..len(u)) of the MSD driven by u, starting at rest.

    ``u`` may be 1-D (one trajectory) or 2-D ``(batch, steps)``; mass, damping
    and stiffness are scalars or per-batch arrays.  x_0 = v_0 = 0 and
    x_{t+1} = RK4(x_t, v_t; u_t held over [t dt, (t+1) dt)).
    """
    u = np.asarray(u, dtype=np.float64)
    squeeze = u.ndim == 1
    if squeeze:
        u = u[None, :]
    nb, steps = u.shape
    m = np.broadcast_to(np.asarray(mass, dtype=np.float64), (nb,))
    c = np.broadcast_to(np.asarray(damping, dtype=np.float64), (nb,))
    k = np.broadcast_to(np.asarray(stiffness, dtype=np.float64), (nb,))
    xs = np.empty((nb, steps + 1), dtype=np.float64)
    x = np.zeros(nb)
    v = np.zeros(nb)
    xs[:, 0] = x
    h = dt
    for t in range(steps):
        ut = u[:, t]
        k1x, k1v = _rhs(x, v, ut, m, c, k)
        k2x, k2v = _rhs(x + 0.5 * h * k1x, v + 0.5 * h * k1v, ut, m, c, k)
        k3x, k3v = _rhs(x + 0.5 * h * k2x, v + 0.5 * h * k2v, ut, m, c, k)
        k4x, k4v = _rhs(x + h * k3x, v + h * k3v, ut, m, c, k)
        x = x + (h / 6.0) * (k1x + 2.0 * k2x + 2.0 * k3x + k4x)
        v = v + (h / 6.0) * (k1v + 2.0 * k2v + 2.0 * k3v + k4v)
        xs[:, t + 1] = x
    return xs[0] if squeeze else xs


def _standardise(train: np.ndarray, test: np.ndarray):
    mu = train.mean(axis=0)
    sd = train.std(axis=0)          # population std (ddof=0)
    sd = np.where(sd > 0, sd, 1.0)
    return (train - mu) / sd, (test - mu) / sd


def _lagged(u: np.ndarray, t0: int, count: int, D: int) -> np.ndarray:
    """Rows t = t0..t0+count-1 of the lag matrix, column j = u_{t-1-j}."""
    idx = np.arange(t0, t0 + count)[:, None] - 1 - np.arange(D)[None, :]
    return np.ascontiguousarray(u[idx])


def make_dataset(cfg: MSDConfig) -> Dataset:
    """Generate one standardised train/test split for ``cfg`` (see module doc)."""
    rng = np.random.default_rng(cfg.seed)
    n_tot = cfg.n_train + cfg.n_test
    steps = cfg.burn_in + cfg.D + n_tot
    u = rng.uniform(-1.0, 1.0, size=steps)
    eps = rng.normal(0.0, cfg.sigma_meas, size=n_tot)
    x = simulate_msd(u, cfg.mass, cfg.damping, cfg.stiffness, cfg.dt)
    t0 = cfg.burn_in + cfg.D
    Zall = _lagged(u, t0, n_tot, cfg.D)
    yall = x[t0:t0 + n_tot] + eps
    Z_raw, Zs_raw = Zall[:cfg.n_train], Zall[cfg.n_train:]
    y_raw, ys_raw = yall[:cfg.n_train], yall[cfg.n_train:]
    Z, Zs = _standardise(Z_raw, Zs_raw)
    y, ys = _standardise(y_raw[:, None], ys_raw[:, None])
    return Dataset(Z=np.ascontiguousarray(Z), y=np.ascontiguousarray(y[:, 0]),
                   Zs=np.ascontiguousarray(Zs), ys=np.ascontiguousarray(ys[:, 0]),
                   Z_raw=np.ascontiguousarray(Z_raw), y_raw=np.ascontiguousarray(y_raw), config=cfg)


def subsample_indices(n: int, count: int, seed: int) -> np.ndarray:
    """Seeded subsample of ``count`` distinct row indices out of ``n`` (sorted, int64)."""
    rng = np.random.default_rng(seed)
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


def draw_c5_params(seed: int) -> dict:
    """Per-dataset draw for the warm-start collection: m, c, k, sigma_meas and D."""
    rng = np.random.default_rng((seed, 5))   # own stream, distinct from the data stream of ``seed``
    return dict(mass=float(rng.uniform(0.5, 2.0)), damping=float(rng.uniform(0.1, 1.0)),
                stiffness=float(rng.uniform(0.5, 2.0)), sigma_meas=float(rng.uniform(0.01, 0.2)),
                D=int(rng.choice([8, 16, 32, 64, 128])))
