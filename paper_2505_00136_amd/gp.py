"""Torch-facing front end: the GP object of the paper's Python API (Section 4.3) on one GPU.

A ``GP`` holds the training data, the kernel function and its hyperparameters, the
trainable flags and the tile configuration, and offers prediction with or without
uncertainty, the loss (NLML), its gradient and Adam optimisation.  torch only
allocates device memory and supplies the current stream; every step runs in the
HIP kernels behind the C-ABI (``_lib``).
"""
from __future__ import annotations

import math
from typing import Sequence

import torch

from . import _lib


def _dev_f64(x, device):
    t = torch.as_tensor(x, dtype=torch.float64, device=device)
    return t.contiguous()


class GP:
    def __init__(self, Z, y, hyper: Sequence[float] = (1.0, 1.0, 0.1), tile: int | str | None = None,
                 prec: str = "fp64", trainable: Sequence[int] = (1, 1, 1), device="cuda:0",
                 refine_sweeps: int | None = None, kernel: str = "se"):
        self.device = torch.device(device)
        self.Z = _dev_f64(Z, self.device)
        self.y = _dev_f64(y, self.device).reshape(-1)
        self.n, self.d = self.Z.shape
        if self.y.shape[0] != self.n:
            raise ValueError("Z and y disagree on n")
        if tile == "auto":
            from .tile_select import select_tile
            tile, _ = select_tile(self.n, self.d, prec, Z=self.Z)
        self.tile = int(tile) if tile else self.n
        self.prec = prec
        self.trainable = tuple(int(t) for t in trainable)
        self.hyper = tuple(float(v) for v in hyper)
        if kernel not in _lib.KERNELS:
            raise ValueError(f"kernel must be one of {sorted(_lib.KERNELS)}")
        self.kernel = kernel
        # None: the library's default for the precision (none in float64)
        self.refine_sweeps = -1 if refine_sweeps is None else int(refine_sweeps)
        self._K = torch.empty(_lib.gpr_tiles_bytes(self.n, self.tile, prec), dtype=torch.uint8, device=self.device)
        self._ws = torch.empty(0, dtype=torch.uint8, device=self.device)
        self.alpha = None
        self._factored = False

    # ---------------------------------------------------------------- workspace
    def _workspace(self, m: int = 0):
        need = _lib.gpr_workspace_size(self.n, m, self.d, self.tile, self.prec)
        if self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws, self._ws.numel()

    @property
    def K_tiles(self):
        return self._K

    @property
    def _h(self):
        return (*self.hyper, self.kernel)

    # ---------------------------------------------------------------- training-side steps
    def fit(self):
        """Assemble K (Eq. 2), factor it tile by tile and solve for alpha."""
        ws, wsb = self._workspace()
        _lib.gpr_assemble(self.Z, self.n, self.d, self._h, self.tile, self.prec, self._K)
        info = _lib.gpr_cholesky(self._K, self.n, self.tile, self.prec, ws, wsb, want_info=True)
        if info != 0:
            raise _lib.GprError(_lib.GPR_ERR_NOT_SPD, f"covariance is not positive definite (column {info})")
        self.alpha = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _lib.gpr_solve(self._K, self.Z, self.n, self.d, self._h, self.tile, self.prec, self.y, self.alpha,
                       self.refine_sweeps, ws, wsb)
        self._factored = True
        return self

    def _need_factor(self):
        if not self._factored:
            self.fit()

    def nlml(self) -> torch.Tensor:
        """Negative log marginal likelihood (negative of Eq. 5), a device scalar."""
        self._need_factor()
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        _lib.gpr_nlml(self._K, self.n, self.tile, self.prec, self.y, self.alpha, out)
        return out[0]

    def grad(self, trainable: Sequence[int] | None = None) -> torch.Tensor:
        """dNLML/dlog(l, nu, sigma^2); consumes the factor (the next call refactors).
        Entries whose `trainable` flag is 0 (default: the GP's flags) are returned as 0."""
        self._need_factor()
        ws, wsb = self._workspace()
        g = torch.empty(3, dtype=torch.float64, device=self.device)
        _lib.gpr_nlml_grad(self.Z, self.n, self.d, self._h, self._K, self.tile, self.prec, self.alpha,
                           self.trainable if trainable is None else tuple(trainable), g, ws, wsb)
        self._factored = False
        return g

    # ---------------------------------------------------------------- prediction
    def predict(self, Zs) -> torch.Tensor:
        """Posterior mean at the test inputs (Eq. 3)."""
        self._need_factor()
        Zs = _dev_f64(Zs, self.device)
        m = Zs.shape[0]
        ws, wsb = self._workspace(m)
        mean = torch.empty(m, dtype=torch.float64, device=self.device)
        _lib.gpr_predict(self.Z, self.n, Zs, m, self.d, self._h, self.alpha, mean, ws, wsb)
        return mean

    def predict_var(self, Zs, full_cov: bool = False, add_noise: bool = False) -> torch.Tensor:
        """Posterior variance, or the full posterior covariance (Eq. 4)."""
        self._need_factor()
        Zs = _dev_f64(Zs, self.device)
        m = Zs.shape[0]
        ws, wsb = self._workspace(m)
        out = torch.empty((m, m) if full_cov else (m,), dtype=torch.float64, device=self.device)
        _lib.gpr_predict_var(self.Z, self.n, Zs, m, self.d, self._h, self._K, self.tile, self.prec, full_cov,
                             add_noise, out, ws, wsb)
        return out

    def predict_with_uncertainty(self, Zs, full_cov: bool = False):
        return self.predict(Zs), self.predict_var(Zs, full_cov=full_cov)

    # ---------------------------------------------------------------- optimisation
    def optimize(self, steps: int, lr: float = 0.1, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                 adam_state=None):
        """Adam on log(l, nu, sigma^2); returns the NLML trace (steps + 1 values)."""
        ws, wsb = self._workspace()
        theta = [math.log(v) for v in self.hyper]
        theta, state, trace = _lib.gpr_optimize(self.Z, self.y, self.n, self.d, self.tile, self.prec, theta,
                                                self.trainable, steps, lr, beta1, beta2, eps, adam_state, self._K,
                                                ws, wsb, kernel=self.kernel)
        self.hyper = tuple(math.exp(t) for t in theta)
        self.adam_state = state
        self._factored = False
        return trace


class NLMLFunction(torch.autograd.Function):
    """NLML(theta_log) with the hand-written backward kernel behind it.

    forward(theta_log[3], gp) -> device scalar; backward returns gout * dNLML/dtheta_log,
    all three entries (the GP's trainable flags do not mask it).  The GP object supplies
    data, tile configuration and precision; forward sets its hyperparameters from
    theta_log.  Each forward keeps its own theta: a backward whose GP has been refitted
    at another theta since (another forward, a fit, an optimisation) or whose factor was
    consumed refits at the saved theta first, so any number of forwards may precede the
    backwards.
    """

    @staticmethod
    def forward(ctx, theta_log, gp: GP):
        vals = theta_log.detach().to("cpu", torch.float64).tolist()
        hyper = tuple(math.exp(v) for v in vals)
        gp.hyper = hyper
        gp.fit()
        out = gp.nlml().clone().to(theta_log.device)
        ctx.gp = gp
        ctx.hyper = hyper
        ctx.theta_device = theta_log.device
        return out

    @staticmethod
    def backward(ctx, gout):
        gp = ctx.gp
        if gp.hyper != ctx.hyper or not gp._factored:
            gp.hyper = ctx.hyper
            gp.fit()
        g = gp.grad(trainable=(1, 1, 1)).to(ctx.theta_device)
        return gout * g, None


def nlml(theta_log: torch.Tensor, gp: GP) -> torch.Tensor:
    return NLMLFunction.apply(theta_log, gp)
