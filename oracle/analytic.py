"""Closed-form eigenpairs of the 1D exponential kernel (oracle pin source).

Paper passage: Sec. 6.1, remark on the spectral reference solution: the leading
eigenvalues of the 1D exponential kernel are validated against the analytical approach
of Ghanem and Spanos (Stochastic Finite Elements, Ch. 2.3.3), which solves
transcendental equations for the frequencies.

Restated for Gamma(x, x') = exp(-|x - x'| / ell) on [0, 1] (centred interval [-a, a]
with a = 1/2, c = 1/ell):
  even modes: c - w tan(w a) = 0,   phi = cos(w (x - 1/2)) / sqrt(a + sin(2 w a) / (2 w))
  odd modes:  w + c tan(w a) = 0,   phi = sin(w (x - 1/2)) / sqrt(a - sin(2 w a) / (2 w))
  lambda = 2 c / (w^2 + c^2).
Even and odd roots interlace; sorting lambda descending interleaves the two families.
"""

import math

import numpy as np
from scipy.optimize import brentq


def exponential_1d(nmodes, ell=1.0, sigma2=1.0):
    """Returns (lam[nmodes], list of callables phi_i) sorted by decreasing lambda."""
    a = 0.5
    c = 1.0 / ell
    eps = 1e-12
    modes = []
    i = 0
    while len(modes) < 2 * nmodes + 2:
        # even root in ((i) pi / a, (i + 1/2) pi / a) of w tan(w a) - c
        lo, hi = i * math.pi / a + eps, (i + 0.5) * math.pi / a - eps
        w = brentq(lambda t: t * math.tan(t * a) - c, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        modes.append(("even", w))
        # odd root in ((i + 1/2) pi / a, (i + 1) pi / a) of w + c tan(w a)
        lo, hi = (i + 0.5) * math.pi / a + eps, (i + 1) * math.pi / a - eps
        w = brentq(lambda t: t + c * math.tan(t * a), lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        modes.append(("odd", w))
        i += 1
    lam = np.array([sigma2 * 2.0 * c / (w * w + c * c) for _, w in modes])
    order = np.argsort(lam)[::-1][:nmodes]
    funcs = []
    for j in order:
        kind, w = modes[j]
        if kind == "even":
            nrm = math.sqrt(a + math.sin(2 * w * a) / (2 * w))
            funcs.append(lambda x, w=w, nrm=nrm: np.cos(w * (np.asarray(x) - 0.5)) / nrm)
        else:
            nrm = math.sqrt(a - math.sin(2 * w * a) / (2 * w))
            funcs.append(lambda x, w=w, nrm=nrm: np.sin(w * (np.asarray(x) - 0.5)) / nrm)
    return lam[order], funcs
