"""FP64 oracle of the Gaussian-process hot path (test infrastructure; never on the product path).

Paper, Section 4.1:
* squared-exponential kernel with length scale l, vertical scale nu and noise
  variance sigma^2, the noise entering through a Kronecker delta on equal
  indices (Eq. 2);
* the covariance matrix K from all pairs of training feature vectors;
* posterior mean  K_{Zs,Z} K^{-1} y  (Eq. 3);
* posterior covariance  K_{Zs,Zs} - K_{Zs,Z} K^{-1} K_{Zs,Z}^T, whose diagonal
  is the predictive variance (Eq. 4);
* log-likelihood  -1/2 log|K| - 1/2 y^T K^{-1} y - N/2 log(2 pi)  (Eq. 5),
  minimised (as its negative) with Adam on the gradient.
Section 4.2: K^{-1} is applied through the Cholesky factor K = L L^T, which is
reused for mean and uncertainty; the forward substitution V = L^{-1} K_{Z,Zs}
serves the variance without a second solve (Section 5.1).

Section 6 names Matern kernels as further kernel functions without giving them; the
oracle uses the standard half-integer members of the Matern family with the same
length scale l and vertical scale nu (s = r / l, r the Euclidean distance):
  nu = 1/2:  nu exp(-s)
  nu = 3/2:  nu (1 + sqrt(3) s) exp(-sqrt(3) s)
  nu = 5/2:  nu (1 + sqrt(5) s + 5 s^2 / 3) exp(-sqrt(5) s)
(the smoothness is named by the kernel tag, "matern12", "matern32", "matern52"; "se"
is the squared-exponential kernel of Eq. 2).

Readings where the paper is silent (each one is listed in the design notes):
* sigma^2 enters K only (delta by index); cross-covariances and the test prior
  carry no noise; ``add_noise`` adds sigma^2 to the predictive variance;
* hyperparameters are optimised in log coordinates theta = log(l, nu, sigma^2);
* Adam uses beta1 = 0.9, beta2 = 0.999, eps = 1e-8 with bias correction.

The oracle is the plain dense definition: no tiling, no blocking, no fusion.
Tiling in the paper only reorders the same arithmetic (Section 4.2, Fig. 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack

LOG2PI = math.log(2.0 * math.pi)


KERNELS = ("se", "matern12", "matern32", "matern52")


@dataclass(frozen=True)
class Hyper:
    """Kernel hyperparameters of Eq. 2: length scale l, vertical scale nu, noise variance
    sigma^2, and the kernel function (squared exponential unless a Matern tag is given)."""
    lengthscale: float
    signal_var: float
    noise_var: float
    kernel: str = "se"

    @staticmethod
    def from_log(theta, kernel: str = "se") -> "Hyper":
        t = np.asarray(theta, dtype=np.float64)
        return Hyper(float(np.exp(t[0])), float(np.exp(t[1])), float(np.exp(t[2])), kernel)

    def log(self) -> np.ndarray:
        return np.log(np.array([self.lengthscale, self.signal_var, self.noise_var], dtype=np.float64))


def sq_dist(A: np.ndarray, B: np.ndarray, block: int = 512) -> np.ndarray:
    """R^2_ij = sum_d (a_id - b_jd)^2 formed from explicit differences (the sum inside Eq. 2)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    out = np.empty((A.shape[0], B.shape[0]), dtype=np.float64)
    for i0 in range(0, A.shape[0], block):
        a = A[i0:i0 + block]
        diff = a[:, None, :] - B[None, :, :]
        out[i0:i0 + block] = np.einsum("ijd,ijd->ij", diff, diff)
    return out


def se_cov(A: np.ndarray, B: np.ndarray, ell: float, nu: float) -> np.ndarray:
    """Noise-free part of Eq. 2 for every pair (a_i, b_j): nu * exp(-R^2 / (2 l^2))."""
    return nu * np.exp(-sq_dist(A, B) / (2.0 * ell * ell))


def matern_of_r2(R2: np.ndarray, ell: float, nu: float, kernel: str) -> np.ndarray:
    """Matern kernel values from squared distances: s = sqrt(R^2) / l, the forms in the
    module docstring."""
    s = np.sqrt(R2) / ell
    if kernel == "matern12":
        return nu * np.exp(-s)
    if kernel == "matern32":
        q = math.sqrt(3.0) * s
        return nu * (1.0 + q) * np.exp(-q)
    if kernel == "matern52":
        q = math.sqrt(5.0) * s
        return nu * (1.0 + q + q * q / 3.0) * np.exp(-q)
    raise ValueError(f"unknown kernel {kernel!r}")


def cov(A: np.ndarray, B: np.ndarray, h: Hyper) -> np.ndarray:
    """Noise-free covariance of every pair (a_i, b_j) under h's kernel function."""
    if h.kernel == "se":
        return se_cov(A, B, h.lengthscale, h.signal_var)
    return matern_of_r2(sq_dist(A, B), h.lengthscale, h.signal_var, h.kernel)


def dcov_dlog_ell(R2: np.ndarray, h: Hyper) -> np.ndarray:
    """Derivative of the noise-free covariance with respect to log l, elementwise:
    se: K_f R^2 / l^2; with s = r / l, matern12: nu s exp(-s); matern32: 3 nu s^2
    exp(-sqrt(3) s); matern52: (5/3) nu s^2 (1 + sqrt(5) s) exp(-sqrt(5) s)."""
    ell, nu = h.lengthscale, h.signal_var
    if h.kernel == "se":
        return nu * np.exp(-R2 / (2.0 * ell * ell)) * R2 / (ell * ell)
    s = np.sqrt(R2) / ell
    if h.kernel == "matern12":
        return nu * s * np.exp(-s)
    if h.kernel == "matern32":
        return 3.0 * nu * s * s * np.exp(-math.sqrt(3.0) * s)
    if h.kernel == "matern52":
        q = math.sqrt(5.0) * s
        return (5.0 / 3.0) * nu * s * s * (1.0 + q) * np.exp(-q)
    raise ValueError(f"unknown kernel {h.kernel!r}")


def train_cov(Z: np.ndarray, h: Hyper) -> np.ndarray:
    """K of Eq. 2 over all training pairs; sigma^2 on the diagonal (delta_ij, equal indices)."""
    K = cov(Z, Z, h)
    K[np.diag_indices_from(K)] += h.noise_var
    return K


def cholesky(K: np.ndarray) -> np.ndarray:
    """Lower factor L with positive diagonal, K = L L^T (Section 4.2), via LAPACK dpotrf."""
    return sla.cholesky(K, lower=True, check_finite=False)


def potrf_info(K: np.ndarray) -> int:
    """LAPACK convention: 0 if K is positive definite, else the 1-based column of the first
    bad pivot -- non-positive or NaN.  Some BLAS builds of dpotrf test only for <= 0; a NaN
    pivot then leaves a NaN diagonal entry of the factor (the earlier ones are finite, the
    later ones NaN too), so the first NaN on the diagonal names that column."""
    L, info = lapack.dpotrf(np.array(K, dtype=np.float64, order="F"), lower=1, clean=1)
    if info == 0:
        bad = np.flatnonzero(np.isnan(np.diag(L)))
        if bad.size:
            return int(bad[0]) + 1
    return int(info)


def solve_alpha(L: np.ndarray, y: np.ndarray) -> np.ndarray:
    """alpha = K^{-1} y = L^{-T} (L^{-1} y): forward then backward substitution (Section 4.2)."""
    z = sla.solve_triangular(L, y, lower=True, check_finite=False)
    return sla.solve_triangular(L, z, lower=True, trans="T", check_finite=False)


def predict_mean(Z, Zs, h: Hyper, alpha, block: int = 4096) -> np.ndarray:
    """Posterior mean of Eq. 3: K_{Zs,Z} alpha (no noise on the cross-covariance)."""
    Zs = np.asarray(Zs, dtype=np.float64)
    out = np.empty(Zs.shape[0], dtype=np.float64)
    for j0 in range(0, Zs.shape[0], block):
        out[j0:j0 + block] = cov(Zs[j0:j0 + block], Z, h) @ alpha
    return out


def predict_var(Z, Zs, h: Hyper, L, full_cov: bool = False, add_noise: bool = False):
    """Posterior variance (diagonal of Eq. 4) or the full posterior covariance.

    V = L^{-1} K_{Z,Zs} comes from the same forward substitution as the mean
    (Section 5.1); then Sigma = K_{Zs,Zs} - V^T V.  The test prior carries no
    noise (latent f); ``add_noise`` adds sigma^2 to the variances.
    """
    Ksz = cov(Z, Zs, h)
    V = sla.solve_triangular(L, Ksz, lower=True, check_finite=False)
    if full_cov:
        S = cov(Zs, Zs, h) - V.T @ V
        if add_noise:
            S[np.diag_indices_from(S)] += h.noise_var
        return S
    var = h.signal_var - np.einsum("ij,ij->j", V, V)
    if add_noise:
        var = var + h.noise_var
    return var


def nlml(L: np.ndarray, y: np.ndarray, alpha: np.ndarray) -> float:
    """Negative of Eq. 5: 1/2 y^T alpha + 1/2 log|K| + N/2 log(2 pi), with log|K| = 2 sum log L_ii."""
    n = y.shape[0]
    return float(0.5 * np.dot(y, alpha) + np.sum(np.log(np.diag(L))) + 0.5 * n * LOG2PI)


def nlml_grad(Z, h: Hyper, L, alpha, trainable=(1, 1, 1)) -> np.ndarray:
    """Gradient of the negative of Eq. 5 in log coordinates theta = log(l, nu, sigma^2).

    dNLML/dtheta_k = 1/2 tr(K^{-1} dK/dtheta_k) - 1/2 alpha^T (dK/dtheta_k) alpha
                   = 1/2 sum_ij (K^{-1} - alpha alpha^T)_ij (dK/dtheta_k)_ij,
    with dK/dlog l = K_f o R^2 / l^2, dK/dlog nu = K_f, dK/dlog sigma^2 = sigma^2 I,
    K_f = nu exp(-R^2/(2 l^2)) for the squared exponential; for a Matern kernel K_f is
    that kernel and dK/dlog l is given at ``dcov_dlog_ell``.  Entries whose ``trainable``
    flag is 0 are 0.
    """
    n = L.shape[0]
    Kinv = sla.cho_solve((L, True), np.eye(n), check_finite=False)
    W = Kinv - np.outer(alpha, alpha)
    R2 = sq_dist(Z, Z)
    Kf = (h.signal_var * np.exp(-R2 / (2.0 * h.lengthscale ** 2)) if h.kernel == "se"
          else matern_of_r2(R2, h.lengthscale, h.signal_var, h.kernel))
    g = np.zeros(3)
    if trainable[0]:
        g[0] = 0.5 * np.sum(W * dcov_dlog_ell(R2, h))
    if trainable[1]:
        g[1] = 0.5 * np.sum(W * Kf)
    if trainable[2]:
        g[2] = 0.5 * h.noise_var * np.trace(W)
    return g


def fit(Z, y, h: Hyper):
    """Assemble K, factor it and solve for alpha; returns (L, alpha, nlml)."""
    K = train_cov(Z, h)
    L = cholesky(K)
    a = solve_alpha(L, y)
    return L, a, nlml(L, y, a)


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, trainable=(1, 1, 1)):
    """One Adam update (Kingma and Ba, 2015) with bias correction; t is the 1-based step count.

    Parameters whose trainable flag is 0 keep their value and their moments.
    Returns new (theta, m, v).
    """
    theta = np.array(theta, dtype=np.float64)
    m = np.array(m, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    for k in range(theta.shape[0]):
        if not trainable[k]:
            continue
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k]
        mhat = m[k] / (1.0 - beta1 ** t)
        vhat = v[k] / (1.0 - beta2 ** t)
        theta[k] = theta[k] - lr * mhat / (math.sqrt(vhat) + eps)
    return theta, m, v


def optimize(Z, y, theta0, steps, lr, beta1=0.9, beta2=0.999, eps=1e-8, trainable=(1, 1, 1), kernel="se"):
    """Adam on theta = log(l, nu, sigma^2) minimising the NLML (Section 4.1).

    Returns (theta_N, nlml_trace) where nlml_trace[i] is the NLML at theta_i,
    i = 0..steps (steps + 1 forward evaluations and ``steps`` gradients).
    """
    theta = np.array(theta0, dtype=np.float64)
    m = np.zeros(3)
    v = np.zeros(3)
    trace = []
    for t in range(1, steps + 1):
        h = Hyper.from_log(theta, kernel)
        L, a, f = fit(Z, y, h)
        trace.append(f)
        g = nlml_grad(Z, h, L, a, trainable)
        theta, m, v = adam_step(theta, g, m, v, t, lr, beta1, beta2, eps, trainable)
    L, a, f = fit(Z, y, Hyper.from_log(theta, kernel))
    trace.append(f)
    return theta, np.array(trace)


def cholesky_flops(n: int) -> float:
    """Flop count of an n x n Cholesky factorisation: n^3/3 + n^2/2 + n/6."""
    return n ** 3 / 3.0 + n ** 2 / 2.0 + n / 6.0


def tile_task_census(T: int, step: int | None = None) -> dict:
    """Number of POTRF/TRSM/SYRK/GEMM tile operations of the tiled right-looking Cholesky.

    Fig. 1 shows step 0 for 1, 4 and 16 tiles per dimension: one POTRF on the
    diagonal tile, a TRSM for every tile below it, a SYRK on every later
    diagonal tile and a GEMM on every strictly-lower trailing tile.  With
    ``step=None`` the totals over all T steps are returned.
    """
    def one(k):
        r = T - k - 1
        return dict(potrf=1, trsm=r, syrk=r, gemm=r * (r - 1) // 2)
    if step is not None:
        return one(step)
    tot = dict(potrf=0, trsm=0, syrk=0, gemm=0)
    for k in range(T):
        for key, val in one(k).items():
            tot[key] += val
    return tot
