"""Brute-force full Galerkin matrix A of eq. (GalA_mat) on tiny meshes (oracle pin).

Paper passages: Sec. 3.5, eq. (GalA_mat):
  A_ij = int int Gamma(F(xhat), F(xhat')) B_i(xhat) B_j(xhat') sqrt(det DF(xhat) det DF(xhat'))
and Sec. 6.2 (Tables ex1-1-opnorms, ex1-2-opnorms), where the exact operator is estimated by
Gauss quadrature to measure || A - A~ || / || A ||.  Here every element is subdivided and
integrated with a tensor Gauss rule (the exponential kernel's kink at x = x' makes plain
Gauss slow to converge; subdividing reduces that error).  Cost is the 2d-dimensional
quadrature the method avoids, so only tiny meshes are used.
"""

import numpy as np

from . import covariance, geometry, kron, splines


def full_galerkin_A(prob, q=4, nsub=4):
    d = prob.d
    t, w = splines.gauss_legendre(q)
    xs1, ws1, Bs1 = [], [], []
    for k in range(d):
        br = np.unique(prob.knots[k])
        xk, wk = [], []
        for a, b in zip(br[:-1], br[1:]):
            for s in range(nsub):
                sa = a + (b - a) * s / nsub
                sb = a + (b - a) * (s + 1) / nsub
                xk.append(0.5 * (sb - sa) * t + 0.5 * (sa + sb))
                wk.append(0.5 * (sb - sa) * w)
        xk = np.concatenate(xk)
        wk = np.concatenate(wk)
        xs1.append(xk)
        ws1.append(wk)
        Bs1.append(splines.basis_matrix(prob.knots[k], prob.p[k], xk))
    grids = np.meshgrid(*xs1, indexing="ij")
    u = np.stack([g.reshape(-1, order="F") for g in grids], axis=1)
    wq = kron.kron_dense([wk[:, None] for wk in ws1]).ravel()
    Bq = kron.kron_dense(Bs1)                       # (nq, N), first index fastest
    X, det = geometry.map_points(prob.desc["map"], u)
    s = np.sqrt(det) * wq
    G = covariance.gamma(prob.cov, X, X)
    W = Bq * s[:, None]
    return W.T @ G @ W


def relative_operator_errors(prob, **kw):
    """(||A - A~||_2 / ||A||_2, ||A - A~||_F / ||A||_F)."""
    A = full_galerkin_A(prob, **kw)
    At = prob.dense_A_tilde()
    E = A - At
    return (np.linalg.norm(E, 2) / np.linalg.norm(A, 2),
            np.linalg.norm(E, "fro") / np.linalg.norm(A, "fro"))
