"""Kronecker matrix-vector products as mode-k tensor contractions (oracle, FP64).

Paper passage followed: Sec. 2.2.  vec ordering puts the first index fastest,
i = i_1 + (i_2 - 1) n_1 + ... , and (D_d x ... x D_1) vec(X) equals the tensor
contraction Y_{i_1..i_d} = sum_j D_{i_1 j_1} ... D_{i_d j_d} X_{j_1..j_d}.
"""

import numpy as np


def to_tensor(v, shape):
    """vec^{-1}: first index fastest (Fortran order); extra trailing axis for columns."""
    v = np.asarray(v)
    if v.ndim == 1:
        return v.reshape(tuple(shape), order="F")
    return v.reshape(tuple(shape) + (v.shape[1],), order="F")


def to_vec(T, nd):
    """vec: inverse of to_tensor; `nd` is the number of tensor axes."""
    if T.ndim == nd:
        return T.reshape(-1, order="F")
    return T.reshape(-1, T.shape[-1], order="F")


def mode_apply(T, k, fn):
    """Apply fn (acting on the leading axis of a 2D array) along tensor axis k."""
    Tm = np.moveaxis(T, k, 0)
    sh = Tm.shape
    R = fn(Tm.reshape(sh[0], -1))
    R = R.reshape((R.shape[0],) + sh[1:])
    return np.moveaxis(R, 0, k)


def kron_matvec(mats, v, shape):
    """(D_d x ... x D_1) v with mats = [D_1, ..., D_d] via d mode contractions."""
    nd = len(mats)
    T = to_tensor(v, shape)
    for k, D in enumerate(mats):
        T = mode_apply(T, k, lambda A, D=D: D @ A)
    return to_vec(T, nd)


def kron_dense(mats):
    """Explicit D_d x ... x D_1 (for tiny sizes only)."""
    K = np.array([[1.0]])
    for D in mats:
        K = np.kron(D, K)
    return K
