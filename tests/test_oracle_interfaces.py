"""Pins of the oracle's discontinuous (C^-1) spaces and one-sided evaluation (Sec. 6: the
interpolation space is made discontinuous across a C^0 line of a two-patch geometry, where
det DF jumps; Sec. 3.6: non-conforming C^-1 discretizations of multipatch domains).

Checked against closed forms: interpolation with a C^-1 knot reproduces piecewise
polynomials with a jump; a kinked (C^0) map has the one-sided Jacobians of its two pieces;
and the rank-two kernel 1 + x x' keeps its closed-form eigenvalues through a kinked
parametrization exactly when both spaces are discontinuous at the kink and every
coincident Greville point takes its own side, while a continuous space misses them.
"""

import math

import numpy as np
import pytest

from oracle import geometry, operator, splines

LIN1 = sorted([(4 + math.sqrt(13)) / 6, (4 - math.sqrt(13)) / 6], reverse=True)


def _f_left(x):
    return 1.0 - 2.0 * x + 3.0 * x ** 3


def _f_right(x):
    return -0.5 + x * x - x ** 3


def test_greville_points_and_sides_at_a_discontinuous_knot():
    kn = np.array([0, 0, 0, 0.3, 0.3, 0.3, 1, 1, 1], dtype=float)      # p = 2, C^-1 at 0.3
    g = splines.greville(kn, 2)
    s = splines.greville_sides(kn, 2)
    assert np.array_equal(g, [0.0, 0.15, 0.3, 0.3, 0.65, 1.0])
    assert np.array_equal(s, [1, 1, -1, 1, 1, -1])
    B = splines.collocation_matrix(kn, 2)
    # the left point sees only the left function, the right point only the right one
    assert np.array_equal(B[2], [0, 0, 1, 0, 0, 0]) and np.array_equal(B[3], [0, 0, 0, 1, 0, 0])
    # evaluated from one side only, the two rows coincide: the matrix is singular
    B1 = splines.basis_matrix(kn, 2, g)
    assert np.linalg.matrix_rank(B1) < 6 and np.linalg.matrix_rank(B) == 6


def test_discontinuous_interpolation_reproduces_a_jump():
    """Cubic space with a C^-1 knot at 0.4 (and a C^1 knot at 0.7): collocation at the
    Greville points, each from its side, reproduces a piecewise cubic with a jump."""
    p, tau = 3, 0.4
    kn = np.array([0] * 4 + [tau] * 4 + [0.7, 0.7] + [1] * 4, dtype=float)
    g, s = splines.greville(kn, p), splines.greville_sides(kn, p)
    left = (g < tau) | ((g == tau) & (s < 0))
    f = np.where(left, _f_left(g), _f_right(g))
    c = np.linalg.solve(splines.collocation_matrix(kn, p), f)
    x = np.random.default_rng(0).random(200)
    vals = splines.basis_matrix(kn, p, x) @ c
    assert np.max(np.abs(vals - np.where(x < tau, _f_left(x), _f_right(x)))) < 1e-12
    # both one-sided values at the knot itself
    assert abs(splines.basis_matrix(kn, p, [tau], [-1]) @ c - _f_left(tau)) < 1e-12
    assert abs(splines.basis_matrix(kn, p, [tau], [1]) @ c - _f_right(tau)) < 1e-12


def kinked_map_1d(a=0.2, tau=0.5):
    """F: [0,1] -> [0,1] piecewise linear, F(tau) = a: slopes a/tau and (1-a)/(1-tau)."""
    return {"kind": "tensor_nurbs", "degree": [1], "knots": [[0, 0, tau, 1, 1]],
            "ctrl": np.array([[0.0], [a], [1.0]])}


def kinked_map_2d(a=0.2, tau=0.5):
    """The unit square, kinked along u_1 = tau (identity in u_2)."""
    ctrl = np.zeros((3, 2, 2))
    for i, x in enumerate((0.0, a, 1.0)):
        for j, y in enumerate((0.0, 1.0)):
            ctrl[i, j] = (x, y)
    return {"kind": "tensor_nurbs", "degree": [1, 1], "knots": [[0, 0, tau, 1, 1], [0, 0, 1, 1]], "ctrl": ctrl}


def test_one_sided_jacobian_of_a_kinked_map():
    g = kinked_map_1d(0.2, 0.5)
    u = np.array([[0.5], [0.5], [0.25], [0.75]])
    X, det = geometry.map_points(g, u, np.array([[-1], [1], [1], [1]]))
    assert np.allclose(X[:, 0], [0.2, 0.2, 0.1, 0.6], atol=1e-15)
    assert np.allclose(det, [0.4, 1.6, 0.4, 1.6], atol=1e-15)


def _kinked_problem(d, p, trial_mult, interp_mult, nelem=4):
    """Trial and interpolation spaces of degree p on `nelem` uniform elements along u_1 with
    the breakpoint 0.5 repeated `trial_mult` / `interp_mult` times (the other breakpoints
    once), the linear kernel 1 + x x', the kinked map."""
    def knots(mult):
        inner = []
        for j in range(1, nelem):
            inner += [j / nelem] * (mult if j / nelem == 0.5 else 1)
        return [0.0] * (p + 1) + inner + [1.0] * (p + 1)
    desc = {"dim": d, "degree": [p] * d, "nelem": [nelem] * d,
            "knots": [knots(trial_mult)] + [None] * (d - 1),
            "interp_knots": [knots(interp_mult)] + [None] * (d - 1),
            "map": kinked_map_1d() if d == 1 else kinked_map_2d(),
            "cov": {"kind": "lin", "sigma2": 1.0, "corr_len": [1.0] * d}}
    if d > 1:
        desc["interp_nelem"] = [nelem] * d
    return operator.Problem(desc)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_linear_kernel_exact_through_a_kinked_map_1d(p):
    """1 + x x' on [0, 1] has eigenvalues (4 +- sqrt 13) / 6.  Through the kinked map its
    eigenfunctions times sqrt(det DF) jump at the kink, and so does the interpolated
    J Gamma J: with both spaces C^-1 there (p + 1 repeated knots) the method is exact."""
    P = _kinked_problem(1, p, p + 1, p + 1)
    w = np.sort(np.linalg.eigvalsh(P.dense_operator()))[::-1]
    assert np.max(np.abs(w[:2] - LIN1)) < 1e-13, w[:3]
    assert np.max(np.abs(w[2:])) < 1e-13


@pytest.mark.parametrize("trial_mult,interp_mult", [(3, 2), (2, 3), (1, 3), (3, 1)])
def test_continuous_spaces_miss_the_kinked_spectrum(trial_mult, interp_mult):
    """With either space continuous at the kink the same problem is no longer exact."""
    P = _kinked_problem(1, 2, trial_mult, interp_mult)
    w = np.sort(np.linalg.eigvalsh(P.dense_operator()))[::-1]
    assert np.max(np.abs(w[:2] - LIN1)) > 1e-6, w[:3]


def test_jacobian_from_one_side_only_misses_the_kinked_spectrum(monkeypatch):
    """The plausible slip: one-sided collocation but det DF at both coincident points taken
    from the same side (the map evaluated without sides).  Exactness is lost, so the sides
    of J are pinned as well as those of the collocation.  (Swapping every side at once only
    permutes the interpolation conditions and changes nothing.)"""
    orig = geometry.map_points
    monkeypatch.setattr(geometry, "map_points", lambda geom, u, side=None: orig(geom, u))
    P = _kinked_problem(1, 2, 3, 3)
    w = np.sort(np.linalg.eigvalsh(P.dense_operator()))[::-1]
    assert np.max(np.abs(w[:2] - LIN1)) > 1e-6, w[:3]


def test_linear_kernel_exact_through_a_kinked_map_2d():
    """1 + x . x' on the unit square (the same rank-three spectrum as through the identity
    map) through the map kinked along u_1 = 1/2, C^-1 spaces along u_1."""
    ref = operator.Problem({"dim": 2, "degree": [2, 2], "nelem": [3, 3], "map": {"kind": "identity"},
                            "cov": {"kind": "lin", "sigma2": 1.0, "corr_len": [1.0, 1.0]}})
    w_ref = np.sort(np.linalg.eigvalsh(ref.dense_operator()))[::-1][:3]
    assert np.allclose(w_ref, [(19 + math.sqrt(313)) / 24, 1 / 12, (19 - math.sqrt(313)) / 24], atol=1e-13)
    P = _kinked_problem(2, 2, 3, 3)
    w = np.sort(np.linalg.eigvalsh(P.dense_operator()))[::-1]
    assert np.max(np.abs(w[:3] - w_ref)) < 1e-13, w[:4]
    assert np.max(np.abs(w[3:])) < 1e-13


def test_discontinuous_trial_space_is_two_independent_patches():
    """A trial knot repeated p + 1 times splits the space into two patches (the non-conforming
    multipatch form of Sec. 3.6): no function straddles the knot, so the Gramian is block
    diagonal, while the covariance still couples the patches."""
    P = _kinked_problem(1, 2, 3, 3, nelem=4)
    n_left = 3 + 1              # p + 1 + (elements left of the knot - 1)
    assert np.all(splines.basis_matrix(P.knots[0], 2, [0.25, 0.49])[:, n_left:] == 0.0)
    assert np.all(splines.basis_matrix(P.knots[0], 2, [0.51, 0.75])[:, :n_left] == 0.0)
    Z = P.Z[0]
    assert np.max(np.abs(Z[:n_left, n_left:])) == 0.0
    A = P.dense_operator()
    # the linear kernel couples the patches (rank two over the whole interval)
    assert np.max(np.abs(A[:n_left, n_left:])) > 1e-3
