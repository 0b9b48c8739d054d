"""Eigenpairs of the standard-form problem A~' v' = lambda v' (oracle, FP64).

Paper passages followed:
  * Sec. 4.1: the generalized problem A v = lambda Z v is rewritten as the standard
    problem A' v' = lambda v' with unchanged eigenvalues.
  * Sec. 4.4.2: the paper solves it with the implicitly restarted Lanczos method;
    the oracle uses ARPACK (scipy eigsh, the same method family) on a LinearOperator
    wrapping Algorithm 1, and dense LAPACK eigh on the assembled matrix for small N.
  * Sec. 3.1: eigenvalues are ordered lambda_1 >= lambda_2 >= ... >= 0 and the
    eigenfunctions are L2-orthonormal; since ||phi_h||_{L2}^2 = v^T Z v = ||v'||_2^2
    (volume-form identity of eq. (basis) and v' = L^T v), unit v' means unit phi_h.
"""

import numpy as np
import scipy.sparse.linalg as ssla


def dense_eigs(prob, k=None):
    """All (or the k largest) eigenpairs of the dense A~', descending, unit columns."""
    A = prob.dense_operator()
    w, V = np.linalg.eigh(A)
    order = np.argsort(w)[::-1]
    w, V = w[order], V[:, order]
    if k is not None:
        w, V = w[:k], V[:, :k]
    return w, V


def iterative_eigs(prob, k, tol=1e-12, stage5=None, v0=None, ncv=None):
    """k largest eigenpairs with ARPACK on the matrix-free Algorithm 1."""
    N = prob.N
    op = ssla.LinearOperator((N, N), dtype=np.float64,
                             matvec=lambda v: prob.apply(v.reshape(-1), stage5=stage5),
                             matmat=lambda V: prob.apply(V, stage5=stage5))
    w, V = ssla.eigsh(op, k=k, which="LA", tol=tol, v0=v0, ncv=ncv)
    order = np.argsort(w)[::-1]
    return w[order], V[:, order]


def residual_norms(prob, w, V):
    """||A~' v_i - lambda_i v_i||_2 per column (FP64 apply)."""
    R = prob.apply(V) - V * w[None, :]
    return np.linalg.norm(R, axis=0)


def clusters(w, rel_gap=1e-3):
    """Maximal runs of consecutive (descending) eigenvalues whose relative gap is
    below rel_gap; degenerate clusters make eigenvectors non-unique."""
    groups = [[0]]
    for i in range(1, len(w)):
        gap = abs(w[i - 1] - w[i]) / max(abs(w[i - 1]), 1e-300)
        if gap < rel_gap:
            groups[-1].append(i)
        else:
            groups.append([i])
    return groups
