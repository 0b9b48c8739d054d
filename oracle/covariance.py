"""Covariance kernels Gamma(x, x') of the oracle (FP64).

Paper passages followed: Sec. 3.1, eq. (kernel) and Fig. (kernels): stationary
isotropic kernels of the Euclidean distance, the exponential kernel (C^0 at x = x')
and the squared exponential (Gaussian) kernel (C^infinity), with variance sigma^2 and
correlation length bL.

Reading (the formulas are not printed): with rho = || diag(ell)^{-1} (x - x') ||_2,
    exp    Gamma = sigma^2 exp(-rho)
    sqexp  Gamma = sigma^2 exp(-rho^2)
Test-only kernels (used by pins, not by the paper):
    exp_l1 Gamma = sigma^2 exp(-sum_k |x_k - x'_k| / ell_k)   (separable)
    const  Gamma = sigma^2
    lin    Gamma = sigma^2 (1 + x . x')                          (rank d + 1, PSD)
"""

import numpy as np


def gamma(cov, X, Y):
    """Kernel matrix G[a, b] = Gamma(X[a], Y[b]) for point arrays of shape (na, d), (nb, d)."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    Y = np.atleast_2d(np.asarray(Y, dtype=np.float64))
    kind = cov["kind"]
    s2 = float(cov.get("sigma2", 1.0))
    d = X.shape[1]
    ell = np.asarray(cov.get("corr_len", [1.0] * d), dtype=np.float64)[:d]
    if kind in ("exp", "sqexp"):
        diff = (X[:, None, :] - Y[None, :, :]) / ell[None, None, :]
        r2 = np.sum(diff * diff, axis=2)
        if kind == "exp":
            return s2 * np.exp(-np.sqrt(r2))
        return s2 * np.exp(-r2)
    if kind == "exp_l1":
        diff = np.abs(X[:, None, :] - Y[None, :, :]) / ell[None, None, :]
        return s2 * np.exp(-np.sum(diff, axis=2))
    if kind == "const":
        return np.full((X.shape[0], Y.shape[0]), s2)
    if kind == "lin":
        return s2 * (1.0 + X @ Y.T)
    raise ValueError("unknown covariance kind %r" % kind)
