"""Oracle (test infrastructure only): the truncated KL expansion at the Greville points.

Only tests/, the smoke check and the benchmark's CPU baseline may import this module.

Sec. 3.2: the field truncated after M terms is mu + sum_i sqrt(lambda_i) phi_i(x) xi_i and
its variance is sum_i lambda_i phi_i(x)^2 (it tends to Gamma(x, x) as M grows).
Sec. 3.4: the discrete eigenfunction is phi_h = sum_j v_j B_j / sqrt(det DF) with the
tensor-product B-splines B_j of the trial space.
Sec. 4.1: v = L^{-T} v' for an eigenvector v' of the standard-form operator.

The functions are evaluated at the mapped Greville points x = F(xhat) of the
interpolation space, in vec order (first index fastest), with the mean mu taken as 0.
"""

import numpy as np

from . import kron, splines


def greville_evaluation(P):
    """Values of the trial B-splines at the interpolation Greville grid: the Kronecker product
    of the univariate nt_k x n_k matrices B_j(g_i) (dense, small problems only)."""
    mats = [splines.basis_matrix(P.knots[k], P.p[k], splines.greville(P.knots_t[k], P.pt[k]),
                                 splines.greville_sides(P.knots_t[k], P.pt[k]))
            for k in range(P.d)]
    return kron.kron_dense(mats)


def eigenfunctions(P, Vp):
    """phi_i at the Greville points (Nt x M) for standard-form eigenvectors Vp (N x M)."""
    coeff = P.to_coefficients(np.asarray(Vp, dtype=np.float64))      # v = L^{-T} v'
    return (greville_evaluation(P) @ coeff) / P.J[:, None]


def sample_field(P, lam, Vp, xi):
    """Zero-mean truncated fields sum_i sqrt(lambda_i) phi_i xi_i: one column per column of
    xi (M x m)."""
    Phi = eigenfunctions(P, Vp)
    return Phi @ (np.sqrt(np.asarray(lam, dtype=np.float64))[:, None] * np.asarray(xi, dtype=np.float64))


def variance_field(P, lam, Vp):
    """sum_i lambda_i phi_i^2 at the Greville points."""
    Phi = eigenfunctions(P, Vp)
    return (Phi ** 2) @ np.asarray(lam, dtype=np.float64)
