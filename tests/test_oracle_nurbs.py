"""Pins of the oracle's general tensor-product NURBS map (Sec. 2.3-2.4: the geometry is a
NURBS map F from the parametric cube, det DF > 0).

Checked against closed forms (circles of the exact rational quadratic arc, areas and
volumes), against refinement invariance (inserting a knot changes the control net but not
the map: Boehm's algorithm, applied here in homogeneous coordinates), linear precision, and
finite differences of the map itself.
"""

import math

import numpy as np
import pytest

from oracle import geometry, operator

W2 = 1.0 / math.sqrt(2.0)


def quarter_annulus(r0=1.0, r1=2.0):
    """Radial degree 1 x angular degree 2, weights (1, 1/sqrt 2, 1): ctrl (2, 3, 2)."""
    ctrl = np.zeros((2, 3, 2))
    w = np.zeros((2, 3))
    for a, r in enumerate((r0, r1)):
        ctrl[a] = [(r, 0.0), (r, r), (0.0, r)]
        w[a] = (1.0, W2, 1.0)
    return {"kind": "tensor_nurbs", "degree": [1, 2], "knots": [[0, 0, 1, 1], [0, 0, 0, 1, 1, 1]],
            "ctrl": ctrl, "weights": w}


def quarter_cylinder_shell(r0=1.0, r1=1.5, h=2.0):
    """3D: the quarter annulus extruded linearly along z: ctrl (2, 3, 2, 3)."""
    ctrl = np.zeros((2, 3, 2, 3))
    w = np.zeros((2, 3, 2))
    for a, r in enumerate((r0, r1)):
        for c, z in enumerate((0.0, h)):
            ctrl[a, :, c] = [(r, 0.0, z), (r, r, z), (0.0, r, z)]
            w[a, :, c] = (1.0, W2, 1.0)
    return {"kind": "tensor_nurbs", "degree": [1, 2, 1],
            "knots": [[0, 0, 1, 1], [0, 0, 0, 1, 1, 1], [0, 0, 1, 1]], "ctrl": ctrl, "weights": w}


def insert_knot(geom, axis, xb):
    """The same map with knot xb inserted in direction `axis` (Boehm): homogeneous control
    points Q_i = a_i P_i + (1 - a_i) P_{i-1}, a_i = 1 up to the span's first function, 0
    past the span, (xb - t_i) / (t_{i+p} - t_i) in between."""
    d = len(geom["degree"])
    p = geom["degree"][axis]
    t = np.asarray(geom["knots"][axis], dtype=np.float64)
    w = np.asarray(geom["weights"], dtype=np.float64)
    Pw = np.concatenate([np.asarray(geom["ctrl"]) * w[..., None], w[..., None]], axis=-1)
    Pw = np.moveaxis(Pw, axis, 0)
    m = Pw.shape[0]
    s = int(np.searchsorted(t, xb, side="right")) - 1
    Q = np.zeros((m + 1,) + Pw.shape[1:])
    for i in range(m + 1):
        if i <= s - p:
            a = 1.0
        elif i >= s + 1:
            a = 0.0
        else:
            a = (xb - t[i]) / (t[i + p] - t[i])
        if i < m:
            Q[i] += a * Pw[i]
        if i >= 1:
            Q[i] += (1.0 - a) * Pw[i - 1]
    Q = np.moveaxis(Q, 0, axis)
    out = dict(geom)
    out["knots"] = [list(k) for k in geom["knots"]]
    out["knots"][axis] = sorted(list(t) + [xb])
    out["weights"] = Q[..., d]
    out["ctrl"] = Q[..., :d] / Q[..., d:]
    return out


def test_annulus_exact_circles_and_area():
    g = quarter_annulus()
    u = np.random.default_rng(0).random((300, 2))
    X, det = geometry.map_points(g, u)
    assert np.max(np.abs(np.linalg.norm(X, axis=1) - (1.0 + u[:, 0]))) < 1e-14
    assert det.min() > 0
    assert abs(geometry.domain_measure(g, 2) - 0.75 * math.pi) < 1e-12
    # the same map as the built-in exact annulus
    Xb, detb = geometry.map_points({"kind": "annulus_nurbs", "r0": 1.0, "r1": 2.0}, u)
    assert np.max(np.abs(X - Xb)) < 1e-14 and np.max(np.abs(det - detb)) < 1e-13


def test_cylinder_shell_exact_radius_height_and_volume():
    g = quarter_cylinder_shell(1.0, 1.5, 2.0)
    u = np.random.default_rng(1).random((200, 3))
    X, det = geometry.map_points(g, u)
    assert np.max(np.abs(np.linalg.norm(X[:, :2], axis=1) - (1.0 + 0.5 * u[:, 0]))) < 1e-14
    assert np.max(np.abs(X[:, 2] - 2.0 * u[:, 2])) < 1e-14
    assert abs(geometry.domain_measure(g, 3, q=10, nsub=4) - 0.25 * math.pi * (1.5 ** 2 - 1.0) * 2.0) < 1e-12


@pytest.mark.parametrize("make,axes", [(quarter_annulus, [(0, 0.3), (1, 0.5), (1, 0.5), (1, 0.8)]),
                                       (quarter_cylinder_shell, [(1, 0.25), (2, 0.6), (0, 0.5)])])
def test_knot_insertion_leaves_the_map_unchanged(make, axes):
    g = make()
    d = len(g["degree"])
    u = np.random.default_rng(2).random((150, d))
    X0, det0 = geometry.map_points(g, u)
    for axis, xb in axes:
        g = insert_knot(g, axis, xb)
        X, det = geometry.map_points(g, u)
        assert np.max(np.abs(X - X0)) < 1e-13 and np.max(np.abs(det - det0)) < 1e-12, (axis, xb)
    assert g["ctrl"].shape[:d] != make()["ctrl"].shape[:d]


def test_linear_precision_box():
    """Control points at the Greville abscissae of the knot vectors reproduce the affine box
    map exactly (any degree, unit weights)."""
    from oracle import splines
    lo, hi = np.array([0.5, -1.0]), np.array([2.0, 1.5])
    degs = [3, 2]
    knots = [[0, 0, 0, 0, 0.2, 0.7, 1, 1, 1, 1], [0, 0, 0, 0.5, 0.5, 1, 1, 1]]
    gx = [splines.greville(np.asarray(knots[k], dtype=float), degs[k]) for k in range(2)]
    G = np.stack(np.meshgrid(*gx, indexing="ij"), axis=-1)
    g = {"kind": "tensor_nurbs", "degree": degs, "knots": knots, "ctrl": lo + (hi - lo) * G}
    u = np.random.default_rng(3).random((100, 2))
    X, det = geometry.map_points(g, u)
    assert np.max(np.abs(X - (lo + (hi - lo) * u))) < 1e-14
    assert np.max(np.abs(det - np.prod(hi - lo))) < 1e-13


def test_jacobian_against_finite_differences():
    rng = np.random.default_rng(4)
    g = quarter_cylinder_shell()
    g = insert_knot(g, 1, 0.4)
    g["ctrl"] = g["ctrl"] + 0.03 * rng.standard_normal(g["ctrl"].shape)
    g["weights"] = g["weights"] * (1.0 + 0.2 * rng.random(g["weights"].shape))
    u = 0.05 + 0.9 * rng.random((15, 3))
    _, det = geometry.map_points(g, u)
    h = 1e-6
    for r in range(len(u)):
        D = np.zeros((3, 3))
        for j in range(3):
            up, um = u[r].copy(), u[r].copy()
            up[j] += h
            um[j] -= h
            D[:, j] = (geometry.map_points(g, up[None])[0][0] - geometry.map_points(g, um[None])[0][0]) / (2 * h)
        assert abs(np.linalg.det(D) - det[r]) < 1e-7


def test_operator_same_as_builtin_annulus():
    """The IBQ operator through the general NURBS map equals the one through the built-in
    exact annulus map (same points, same J)."""
    cov = {"kind": "exp", "sigma2": 1.0, "corr_len": [0.6, 0.6]}
    a = operator.Problem({"dim": 2, "degree": [2, 2], "nelem": [5, 4], "map": quarter_annulus(), "cov": cov})
    b = operator.Problem({"dim": 2, "degree": [2, 2], "nelem": [5, 4],
                          "map": {"kind": "annulus_nurbs", "r0": 1.0, "r1": 2.0}, "cov": cov})
    A, B = a.dense_operator(), b.dense_operator()
    assert np.max(np.abs(A - B)) < 1e-13 * np.max(np.abs(B))


def test_explicit_knots_equal_uniform():
    """Explicit open uniform knots give the same problem as the element count."""
    cov = {"kind": "sqexp", "sigma2": 1.0, "corr_len": [0.5, 0.4]}
    a = operator.Problem({"dim": 2, "degree": [2, 3], "nelem": [4, 3], "map": {"kind": "identity"}, "cov": cov})
    b = operator.Problem({"dim": 2, "degree": [2, 3], "knots": [[0, 0, 0, .25, .5, .75, 1, 1, 1],
                                                                [0, 0, 0, 0, 1 / 3, 2 / 3, 1, 1, 1, 1]],
                          "map": {"kind": "identity"}, "cov": cov})
    assert np.max(np.abs(a.dense_operator() - b.dense_operator())) < 1e-14
