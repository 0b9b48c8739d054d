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


@pytest.mark.parametrize("ell", [1.0, 0.5, 0.3])
def test_ibq_eigenvalues_converge_to_analytic(ell):
    """The correlation length enters as exp(-|x - x'| / ell): the IBQ eigenvalues at ell
    other than 1 converge to the closed-form ones of that ell (at rate about h^2 for the
    C^0 kernel with quadratic splines), for the six leading modes."""
    lam, _ = analytic.exponential_1d(6, ell=ell)
    errs = []
    for ne in (16, 32, 64, 128):
        w, _ = eigs.dense_eigs(operator.Problem(_exp1d(ne, ell=ell)), 6)
        errs.append(np.abs(w - lam) / lam)
    errs = np.array(errs)
    assert np.all(errs[1:] < errs[:-1])
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all(order >= 1.8), order
    assert errs[-1, 0] < 1e-4 and np.all(errs[-1] < 2e-3)


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


def test_separable_2d_anisotropic_box_products_of_analytic():
    """exp in the L1 norm with ell = (0.5, 0.3) on the box [0, 2] x [0, 1]: the operator
    separates, so its eigenvalues are products lam_x lam_y of the two 1D spectra, and on
    [0, a] with length ell the 1D spectrum is a times the [0, 1] spectrum with ell / a.
    The box and the lengths are unequal along the two axes, so a length applied to the
    wrong axis, or multiplied instead of divided, gives another spectrum."""
    lx, _ = analytic.exponential_1d(6, ell=0.5 / 2.0)
    ly, _ = analytic.exponential_1d(6, ell=0.3)
    prods = np.sort(np.outer(2.0 * lx, ly).ravel())[::-1][:6]
    errs = []
    for ne in (8, 16, 32):
        P = operator.Problem({"dim": 2, "degree": [2, 2], "nelem": [2 * ne, ne],
                              "map": {"kind": "box", "lo": [0.0, 0.0], "hi": [2.0, 1.0]},
                              "cov": {"kind": "exp_l1", "sigma2": 1.0, "corr_len": [0.5, 0.3]}})
        w, _ = eigs.dense_eigs(P, 6) if P.N <= 1200 else eigs.iterative_eigs(P, 6, tol=1e-12)
        errs.append(np.abs(w - prods) / prods)
    errs = np.array(errs)
    assert np.all(errs[1:] < errs[:-1])
    assert np.all(np.log2(errs[:-1] / errs[1:]) >= 1.5)
    assert errs[-1, 0] < 2e-3 and np.max(errs[-1]) < 6e-3


def _double_integral(kind, ell):
    """int_0^1 int_0^1 Gamma(x, y) dx dy in closed form (sigma^2 = 1)."""
    if kind == "exp":
        return 2.0 * ell - 2.0 * ell ** 2 * (1.0 - math.exp(-1.0 / ell))
    return ell * math.sqrt(math.pi) * math.erf(1.0 / ell) - ell ** 2 * (1.0 - math.exp(-1.0 / ell ** 2))


@pytest.mark.parametrize("kind,p,order", [("exp", 2, 1.8), ("sqexp", 3, 3.5)])
@pytest.mark.parametrize("ell", [0.5, 0.3])
def test_constant_function_quadratic_form_closed_form(kind, p, order, ell):
    """The constant function 1 = sum_i B_i (partition of unity) has coefficient vector of
    ones, and 1^T A~ 1 is the IBQ approximation of <1, T 1> = int int Gamma.  Its closed
    form pins the kernel formula itself (exp(-rho), exp(-rho^2)) and the scaling by the
    correlation length, independently of the eigen-solver: the error falls at the
    interpolation rate (h^2 for the C^0 exponential kernel, h^4 with cubic splines for the
    smooth squared exponential)."""
    exact = _double_integral(kind, ell)
    errs = []
    for ne in (8, 16, 32, 64):
        P = operator.Problem(_exp1d(ne, p=p, ell=ell, kind=kind))
        one = np.ones(P.N)
        errs.append(abs(one @ P.dense_A_tilde() @ one - exact) / exact)
    errs = np.array(errs)
    assert np.all(np.log2(errs[:-1] / errs[1:]) >= order), errs
    assert errs[-1] < (5e-4 if kind == "exp" else 1e-7)


@pytest.mark.parametrize("kind", ["exp", "sqexp", "exp_l1"])
def test_box_scaling_with_correlation_length(kind):
    """Gamma depends on (x - x') / ell only: scaling the domain by (c1, c2) and ell by the
    same factors multiplies every eigenvalue of A~' by the area ratio c1 c2 (exactly, up to
    rounding: the parametric setup is the same and J^2 = c1 c2)."""
    c = (2.5, 0.4)
    base = {"dim": 2, "degree": [2, 3], "nelem": [6, 5], "map": {"kind": "identity"},
            "cov": {"kind": kind, "sigma2": 1.0, "corr_len": [0.7, 0.45]}}
    scaled = {"dim": 2, "degree": [2, 3], "nelem": [6, 5],
              "map": {"kind": "box", "lo": [0.0, 0.0], "hi": list(c)},
              "cov": {"kind": kind, "sigma2": 1.0, "corr_len": [0.7 * c[0], 0.45 * c[1]]}}
    w0 = np.linalg.eigvalsh(operator.Problem(base).dense_operator())
    w1 = np.linalg.eigvalsh(operator.Problem(scaled).dense_operator())
    assert np.max(np.abs(w1 - c[0] * c[1] * w0)) < 1e-13 * w1.max()
    # and a length applied to the other axis changes the spectrum
    swapped = dict(scaled, cov=dict(scaled["cov"], corr_len=[0.45 * c[1], 0.7 * c[0]]))
    w2 = np.linalg.eigvalsh(operator.Problem(swapped).dense_operator())
    assert np.max(np.abs(w2 - w1)) > 1e-3 * w1.max()
