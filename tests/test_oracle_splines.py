"""Pins of the oracle's spline machinery against closed forms and brute force.

Paper passages: Sec. 2.3 (B-splines), Sec. 3.5 (Remark massmatrix), Sec. 4.2-4.3
(collocation at the Greville abscissae, mixed mass matrix).
"""

import numpy as np
import pytest

from oracle import kron, splines

def _cardinal_quadratic(t):
    """Uniform quadratic B-spline on [0, 3] (closed form)."""
    t = np.asarray(t)
    out = np.zeros_like(t)
    m0 = (t >= 0) & (t < 1)
    m1 = (t >= 1) & (t < 2)
    m2 = (t >= 2) & (t < 3)
    out[m0] = 0.5 * t[m0] ** 2
    out[m1] = 0.5 * (-2 * t[m1] ** 2 + 6 * t[m1] - 3)
    out[m2] = 0.5 * (3 - t[m2]) ** 2
    return out


def test_interior_quadratic_is_cardinal_bspline():
    ne, p = 8, 2
    kn = splines.open_uniform_knots(p, ne)
    x = np.linspace(0, 1, 401)
    B = splines.basis_matrix(kn, p, x)
    h = 1.0 / ne
    for i in range(p, ne):          # interior functions with simple knots only
        expect = _cardinal_quadratic((x - kn[i]) / h)
        assert np.max(np.abs(B[:, i] - expect)) < 1e-14


def test_linear_basis_is_hat():
    kn = splines.open_uniform_knots(1, 4)
    x = np.linspace(0, 1, 101)
    B = splines.basis_matrix(kn, 1, x)
    for i in range(5):
        hat = np.maximum(0.0, 1.0 - np.abs(x - i / 4) * 4)
        assert np.max(np.abs(B[:, i] - hat)) < 1e-14


@pytest.mark.parametrize("p,ne", [(1, 3), (2, 5), (3, 7), (4, 2)])
def test_partition_of_unity_and_dimension(p, ne):
    kn = splines.open_uniform_knots(p, ne)
    assert splines.dimension(kn, p) == ne + p
    x = np.concatenate([np.random.default_rng(1).random(50), [0.0, 1.0]])
    B = splines.basis_matrix(kn, p, x)
    assert np.max(np.abs(B.sum(axis=1) - 1)) < 1e-14
    assert B.min() >= 0
    Bt = splines.collocation_matrix(kn, p)
    assert np.max(np.abs(Bt.sum(axis=1) - 1)) < 1e-14


def test_greville_examples():
    # knot averages: p = 2, knots (0,0,0,1/2,1,1,1) -> (0, 1/4, 3/4, 1)
    g = splines.greville(splines.open_uniform_knots(2, 2), 2)
    assert np.allclose(g, [0, 0.25, 0.75, 1.0], atol=1e-15)
    # p = 3, one element: Bezier -> equispaced (0, 1/3, 2/3, 1)
    g = splines.greville(splines.open_uniform_knots(3, 1), 3)
    assert np.allclose(g, [0, 1 / 3, 2 / 3, 1], atol=1e-15)
    # Greville points reproduce linear functions: sum_j xhat_j B_j(x) = x
    kn = splines.open_uniform_knots(3, 6)
    x = np.linspace(0, 1, 77)
    assert np.max(np.abs(splines.basis_matrix(kn, 3, x) @ splines.greville(kn, 3) - x)) < 1e-14


def test_mass_matrix_p1_closed_form():
    ne = 5
    h = 1.0 / ne
    Z = splines.mass_matrix(splines.open_uniform_knots(1, ne), 1)
    E = np.zeros((ne + 1, ne + 1))
    for i in range(ne + 1):
        E[i, i] = 2 * h / 3
        if i + 1 <= ne:
            E[i, i + 1] = E[i + 1, i] = h / 6
    E[0, 0] = E[ne, ne] = h / 3
    assert np.max(np.abs(Z - E)) < 1e-15


@pytest.mark.parametrize("p,ne", [(1, 4), (2, 6), (3, 5), (4, 3)])
def test_mass_row_sums_are_basis_integrals(p, ne):
    kn = splines.open_uniform_knots(p, ne)
    Z = splines.mass_matrix(kn, p)
    assert np.max(np.abs(Z.sum(axis=1) - splines.basis_integrals(kn, p))) < 1e-15
    assert np.max(np.abs(Z - Z.T)) < 1e-16


def test_mass_matrix_vs_brute_force_midpoint():
    p, ne = 3, 4
    kn = splines.open_uniform_knots(p, ne)
    Z = splines.mass_matrix(kn, p)
    m = 4000
    xs = (np.arange(m) + 0.5) / m                 # composite midpoint rule
    Bf = splines.basis_matrix(kn, p, xs)
    Zb = Bf.T @ Bf / m
    assert np.max(np.abs(Z - Zb)) < 1e-7


@pytest.mark.parametrize("pt,net,p,ne", [(2, 8, 2, 8), (3, 5, 2, 4), (1, 7, 3, 3), (4, 6, 2, 9)])
def test_mixed_mass_sums(pt, net, p, ne):
    kt = splines.open_uniform_knots(pt, net)
    kn = splines.open_uniform_knots(p, ne)
    M = splines.mixed_mass_matrix(kt, pt, kn, p)
    assert M.shape == (net + pt, ne + p)
    # partition of unity of the interpolation basis: column sums = int B_j
    assert np.max(np.abs(M.sum(axis=0) - splines.basis_integrals(kn, p))) < 1e-15
    # and of the trial basis: row sums = int Bt_i
    assert np.max(np.abs(M.sum(axis=1) - splines.basis_integrals(kt, pt))) < 1e-15


def test_mixed_mass_equals_gramian_for_equal_spaces():
    kn = splines.open_uniform_knots(3, 5)
    assert np.max(np.abs(splines.mixed_mass_matrix(kn, 3, kn, 3) - splines.mass_matrix(kn, 3))) < 1e-15


def test_cholesky_and_collocation_inverse():
    kn = splines.open_uniform_knots(3, 9)
    Z = splines.mass_matrix(kn, 3)
    L = np.linalg.cholesky(Z)
    assert np.max(np.abs(L @ L.T - Z)) < 1e-15
    Bt = splines.collocation_matrix(kn, 3)
    assert np.max(np.abs(Bt @ np.linalg.inv(Bt) - np.eye(len(Bt)))) < 1e-13


def test_kron_contraction_equals_dense_kron():
    rng = np.random.default_rng(3)
    mats = [rng.standard_normal((m, n)) for m, n in [(4, 3), (2, 5), (3, 2)]]
    shape = [3, 5, 2]
    v = rng.standard_normal((30, 4))
    dense = np.kron(mats[2], np.kron(mats[1], mats[0]))
    assert np.max(np.abs(kron.kron_matvec(mats, v, shape) - dense @ v)) < 1e-13
    # vec ordering: first index fastest
    T = kron.to_tensor(np.arange(30.0), shape)
    assert T[1, 0, 0] == 1 and T[0, 1, 0] == 3 and T[0, 0, 1] == 15


@pytest.mark.parametrize("pt", [2, 3, 4])
def test_c0_interpolation_reproduces_kinked_function(pt):
    """Reduced-continuity interpolation (Sec. 4.2): with every interior breakpoint repeated
    pt times the space holds all continuous piecewise polynomials of degree pt, so
    collocation at the Greville points reproduces |x - 1/2| (kink at a breakpoint) exactly;
    the maximally smooth space of the same mesh cannot."""
    net = 4
    kn = splines.knots_with_multiplicity(pt, [j / net for j in range(1, net)], pt)
    n = splines.dimension(kn, pt)
    assert n == pt + 1 + (net - 1) * pt == net * pt + 1
    g = splines.greville(kn, pt)
    # C^0 Greville points of a uniform mesh: the pt + 1 equispaced points of every element
    assert np.max(np.abs(g - np.arange(n) / (n - 1))) < 1e-15
    f = lambda x: np.abs(x - 0.5)
    xs = np.random.default_rng(pt).random(300)
    c = np.linalg.solve(splines.collocation_matrix(kn, pt), f(g))
    assert np.max(np.abs(splines.basis_matrix(kn, pt, xs) @ c - f(xs))) < 1e-13
    ks = splines.open_uniform_knots(pt, net)
    cs = np.linalg.solve(splines.collocation_matrix(ks, pt), f(splines.greville(ks, pt)))
    assert np.max(np.abs(splines.basis_matrix(ks, pt, xs) @ cs - f(xs))) > 1e-3
