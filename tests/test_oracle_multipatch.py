"""Pins of the oracle's multipatch problems (Sec. 3.6: non-conforming multipatch domains;
every patch keeps its own spaces and map, stage 5 couples all patches).

* Two boxes side by side are the single box with a discontinuous (C^-1) knot where they
  meet (pinned in test_oracle_interfaces.py): the standard forms differ only by the
  per-patch scaling of the basis (1 / sqrt(det DF)), so the spectra agree.
* An L-shaped domain of three unit squares with the rank-three kernel 1 + x . x': its
  eigenvalues are those of the Gram matrix of (1, x_1, x_2) on the L-shape, computed by
  hand below, and every patch space contains the linear functions, so the method is exact.
"""

import numpy as np
import pytest

from oracle import multipatch, operator

G_L = np.array([[3.0, 2.5, 2.5],          # int 1, int x1, int x2 over the L-shape
                [2.5, 3.0, 1.75],         # int x1^2 = 8/3 + 1/3, int x1 x2 = 1 + 3/4
                [2.5, 1.75, 3.0]])        # int x2^2 = 2/3 + 7/3


def box(lo, hi, p, ne, kind="lin", ell=(1.0, 1.0), **kw):
    d = dict({"dim": 2, "degree": list(p), "nelem": list(ne), "map": {"kind": "box", "lo": list(lo), "hi": list(hi)},
              "cov": {"kind": kind, "sigma2": 1.0, "corr_len": list(ell)}}, **kw)
    return d


def l_shape(kind="lin", ell=(1.0, 1.0)):
    return [box((0, 0), (1, 1), (2, 2), (3, 3), kind, ell),
            box((1, 0), (2, 1), (3, 2), (4, 2), kind, ell),
            box((0, 1), (1, 2), (2, 3), (2, 4), kind, ell)]


def test_l_shape_linear_kernel_closed_form():
    M = multipatch.MultipatchProblem(l_shape())
    w = np.sort(np.linalg.eigvalsh(M.dense_operator()))[::-1]
    ref = np.sort(np.linalg.eigvalsh(G_L))[::-1]
    assert np.max(np.abs(w[:3] - ref)) < 1e-12, (w[:4], ref)
    assert np.max(np.abs(w[3:])) < 1e-12


def test_l_shape_loses_a_patch_loses_the_spectrum():
    """Dropping the third square changes the Gram matrix (a plausible assembly slip, e.g.
    stage 5 over the first patches only, shows up)."""
    M = multipatch.MultipatchProblem(l_shape()[:2])
    w = np.sort(np.linalg.eigvalsh(M.dense_operator()))[::-1]
    assert np.max(np.abs(w[:3] - np.sort(np.linalg.eigvalsh(G_L))[::-1])) > 1e-2


@pytest.mark.parametrize("kind,ell", [("exp", (0.5, 0.3)), ("sqexp", (0.4, 0.7))])
def test_two_boxes_equal_one_box_with_a_discontinuous_knot(kind, ell):
    p = 2
    left = box((0, 0), (1, 1), (p, 3), (3, 4), kind, ell, interp_degree=[2, 3], interp_nelem=[4, 5])
    right = box((1, 0), (2, 1), (p, 3), (3, 4), kind, ell, interp_degree=[2, 3], interp_nelem=[4, 5])
    M = multipatch.MultipatchProblem([left, right])
    t = [0.0] * (p + 1) + [1 / 6, 2 / 6] + [0.5] * (p + 1) + [4 / 6, 5 / 6] + [1.0] * (p + 1)
    tt = [0.0] * 3 + [1 / 8, 2 / 8, 3 / 8] + [0.5] * 3 + [5 / 8, 6 / 8, 7 / 8] + [1.0] * 3
    single = operator.Problem({"dim": 2, "degree": [p, 3], "knots": [t, None], "nelem": [0, 4],
                               "interp_degree": [2, 3], "interp_knots": [tt, None], "interp_nelem": [0, 5],
                               "map": {"kind": "box", "lo": [0, 0], "hi": [2, 1]},
                               "cov": {"kind": kind, "sigma2": 1.0, "corr_len": list(ell)}})
    assert single.N == M.N and single.Nt == M.Nt
    w1 = np.sort(np.linalg.eigvalsh(M.dense_operator()))
    w2 = np.sort(np.linalg.eigvalsh(single.dense_operator()))
    assert np.max(np.abs(w1 - w2)) < 1e-13 * w2[-1]
    # the same set of points
    key = lambda X: X[np.lexsort(X.T[::-1])]   # noqa: E731
    assert np.max(np.abs(key(M.X) - key(single.X))) < 1e-15


def test_patch_order_is_a_permutation():
    """Listing the patches in another order permutes the operator's rows and columns."""
    a = multipatch.MultipatchProblem(l_shape("exp", (0.6, 0.6)))
    perm = [2, 0, 1]
    b = multipatch.MultipatchProblem([l_shape("exp", (0.6, 0.6))[i] for i in perm])
    idx = np.concatenate([np.arange(a.noff[i], a.noff[i + 1]) for i in perm])
    assert np.max(np.abs(b.dense_operator() - a.dense_operator()[np.ix_(idx, idx)])) < 1e-14


def test_patches_must_share_dim_and_covariance():
    L = l_shape()
    with pytest.raises(ValueError):
        multipatch.MultipatchProblem([L[0], dict(L[1], cov={"kind": "exp", "sigma2": 1.0, "corr_len": [1.0, 1.0]})])
