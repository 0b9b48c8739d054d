"""Pins of the oracle's eigenpairs against the closed-form 1D exponential spectrum.

Paper passage: Sec. 6.1 (one-dimensional case study and the remark on the reference
solution): the first eigenvalues of the exponential kernel are known analytically
(Ghanem and Spanos, Ch. 2.3.3), and the IBQ Galerkin eigenvalues approach them under
refinement.
"""

import math

import numpy as np
import pytest

from oracle import analytic, eigs, operator, splines


def _exp1d(ne, p=2, ell=1.0, kind="exp"):
    return {"dim": 1, "degree": [p], "nelem": [ne], "map": {"kind": "identity"},
            "cov": {"kind": kind, "sigma2": 1.0, "corr_len": [ell]}}


def _gauss_on(a, b, q=40):
    t, w = splines.gauss_legendre(q)
    return 0.5 * (b - a) * t + 0.5 * (a + b), 0.5 * (b - a) * w


@pytest.mark.parametrize("ell", [1.0, 0.3])
def test_analytic_pairs_solve_the_integral_equation(ell):
    """(T phi)(x) = lambda phi(x), checked by quadrature split at the kink x' = x."""
    lam, phis = analytic.exponential_1d(6, ell=ell)
    assert np.all(np.diff(lam) < 0)
    for li, phi in zip(lam, phis):
        for x in (0.0, 0.13, 0.5, 0.77, 1.0):
            acc = 0.0
            for a, b in ((0.0, x), (x, 1.0)):
                if b > a:
                    xs, ws = _gauss_on(a, b)
                    acc += np.sum(ws * np.exp(-np.abs(x - xs) / ell) * phi(xs))
            assert abs(acc - li * phi(x)) < 1e-12
    # orthonormality in L2(0, 1)
    xs, ws = _gauss_on(0.0, 1.0, 200)
    G = np.array([[np.sum(ws * f(xs) * g(xs)) for g in phis] for f in phis])
    assert np.max(np.abs(G - np.eye(len(phis)))) < 1e-12


def test_ibq_eigenvalues_converge_to_analytic():
    lam, _ = analytic.exponential_1d(4, ell=1.0)
    errs = []
    for ne in (16, 32, 64, 128):
        w, _ = eigs.dense_eigs(operator.Problem(_exp1d(ne)), 4)
        errs.append(np.abs(w - lam) / lam)
    errs = np.array(errs)
    assert np.all(errs[1:] < errs[:-1])
    order = np.log2(errs[:-1, 0] / errs[1:, 0])
    assert np.all(order >= 1.5)
    assert errs[-1, 0] < 5e-5


def test_ibq_eigenfunctions_converge_to_analytic():
    lam, phis = analytic.exponential_1d(3, ell=1.0)
    errs = []
    for ne in (16, 64):
        P = operator.Problem(_exp1d(ne))
        xs, ws = splines._composite_gauss(np.unique(P.knots[0]), 10)   # exact on each element
        w, V = eigs.dense_eigs(P, 3)
        C = P.to_coefficients(V)                          # v = L^{-T} v'
        B = splines.basis_matrix(P.knots[0], P.p[0], xs)   # identity map: det DF = 1
        e = []
        for i in range(3):
            ph = B @ C[:, i]
            s = np.sign(np.sum(ws * ph * phis[i](xs)))
            e.append(math.sqrt(np.sum(ws * (s * ph - phis[i](xs)) ** 2)))
            assert abs(np.sum(ws * ph * ph) - 1.0) < 1e-12     # ||phi_h||_L2 = ||v'||_2 = 1
        errs.append(e)
    assert np.all(np.array(errs[1]) < 0.5 * np.array(errs[0]))
    assert max(errs[1]) < 1e-3


def test_separable_2d_products_of_analytic():
    """exp in the L1 norm on the unit square separates: the 2D spectrum is the set of
    products of 1D spectra, so the leading 2D eigenvalues approach analytic products."""
    lam, _ = analytic.exponential_1d(4, ell=1.0)
    prods = np.sort(np.outer(lam, lam).ravel())[::-1][:5]
    errs = []
    for ne in (16, 32):
        P = operator.Problem({"dim": 2, "degree": [2, 2], "nelem": [ne, ne], "map": {"kind": "identity"},
                              "cov": {"kind": "exp_l1", "sigma2": 1.0, "corr_len": [1.0, 1.0]}})
        w, _ = eigs.iterative_eigs(P, 5, tol=1e-12)
        errs.append(np.abs(w - prods) / prods)
    assert np.all(errs[1] < errs[0])
    assert np.max(errs[1]) < 5e-3 and errs[1][0] < 1e-3
