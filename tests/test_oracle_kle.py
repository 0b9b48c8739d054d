"""Pins of the truncated-KLE oracle (Sec. 3.2) against closed forms.

A kernel of finite rank r is reproduced exactly by its first r eigenpairs (Mercer's
theorem), and when its eigenfunctions lie in the discrete space the Galerkin pairs are the
exact ones; the truncated variance at M = r is then Gamma(x, x) itself, and every sample
field lies in the kernel's range.  These checks fail for a dropped L^{-T}, a missing or
inverted 1 / sqrt(det DF), a missing square root of lambda, or a transposed Kronecker order.
"""

import numpy as np
import pytest

from oracle import eigs, kle, operator


def _problem(d, p, ne, kind, geom, s2=1.0, **extra):
    desc = {"dim": d, "degree": [p] * d, "nelem": [ne] * d, "map": geom,
            "cov": {"kind": kind, "sigma2": s2, "corr_len": [1.0] * d}}
    desc.update(extra)
    return operator.Problem(desc)


@pytest.mark.parametrize("d,geom", [
    (1, {"kind": "box", "lo": [0.5], "hi": [2.0]}),
    (2, {"kind": "box", "lo": [0.0, -1.0], "hi": [2.0, 0.5]}),
    (3, {"kind": "box", "lo": [0.0, 0.0, 0.0], "hi": [1.0, 2.0, 0.5]}),
])
def test_constant_kernel_variance_is_sigma2(d, geom):
    """Gamma = sigma^2 has rank one with phi_1 = |D|^{-1/2}: the M = 1 variance is sigma^2 at
    every point and a sample is the constant sigma xi_1."""
    P = _problem(d, 2, 3, "const", geom, s2=1.7)
    lam, V = eigs.dense_eigs(P, 1)
    var = kle.variance_field(P, lam, V)
    assert np.max(np.abs(var - 1.7)) < 1e-12
    f = kle.sample_field(P, lam, V, np.array([[0.3, -1.2]]))
    assert np.max(np.abs(np.abs(f) - np.sqrt(1.7) * np.array([0.3, 1.2]))) < 1e-12


@pytest.mark.parametrize("d,p,ne,geom", [
    (1, 2, 5, {"kind": "identity"}),
    (2, 2, 3, {"kind": "identity"}),
    (2, 3, 4, {"kind": "box", "lo": [0.5, -1.0], "hi": [1.5, 1.0]}),
    (3, 1, 2, {"kind": "identity"}),
])
def test_linear_kernel_variance_and_samples(d, p, ne, geom):
    """Gamma = 1 + x . x' has rank d + 1 with range span{1, x_1, .., x_d}: the variance of
    the first d + 1 terms is 1 + |x|^2 and every sample field is affine in x."""
    P = _problem(d, p, ne, "lin", geom, interp_degree=[p + 1] * d, interp_nelem=[ne + 1] * d)
    lam, V = eigs.dense_eigs(P, d + 1)
    var = kle.variance_field(P, lam, V)
    assert np.max(np.abs(var - (1.0 + np.sum(P.X ** 2, axis=1)))) < 1e-11
    xi = np.random.default_rng(d).standard_normal((d + 1, 3))
    f = kle.sample_field(P, lam, V, xi)
    A = np.hstack([np.ones((P.Nt, 1)), P.X])
    coef, *_ = np.linalg.lstsq(A, f, rcond=None)
    assert np.max(np.abs(A @ coef - f)) < 1e-11 * max(1.0, np.abs(f).max())
    # one term too few loses variance somewhere (the pin is not vacuous)
    assert np.max(np.abs(kle.variance_field(P, lam[:d], V[:, :d]) - var)) > 1e-3


def test_eigenfunctions_orthonormal_in_l2_on_annulus():
    """The discrete eigenfunctions are L2(D)-orthonormal (Sec. 3.1): with the physical
    measure det DF dxhat, the Gauss-quadrature Gram matrix of phi_i is the identity.  Checked
    through coefficients (no 1/J cancellation) against the Greville values on a curved map."""
    from oracle import geometry, splines
    P = _problem(2, 2, 6, "sqexp", {"kind": "annulus_nurbs", "r0": 1.0, "r1": 2.0})
    lam, V = eigs.dense_eigs(P, 4)
    coeff = P.to_coefficients(V)
    g, w = np.polynomial.legendre.leggauss(8)
    br = np.linspace(0.0, 1.0, 7)
    xs = np.concatenate([(a + b) / 2 + (b - a) / 2 * g for a, b in zip(br[:-1], br[1:])])
    ws = np.concatenate([(b - a) / 2 * w for a, b in zip(br[:-1], br[1:])])
    B = [splines.basis_matrix(P.knots[k], P.p[k], xs) for k in range(2)]
    U = np.stack(np.meshgrid(xs, xs, indexing="ij"), axis=-1).reshape(-1, 2, order="F")
    Wq = np.outer(ws, ws).reshape(-1, order="F")
    _, det = geometry.map_points(P.desc["map"], U)
    vals = np.kron(B[1], B[0]) @ coeff / np.sqrt(det)[:, None]
    G = vals.T @ (vals * (Wq * det)[:, None])
    assert np.max(np.abs(G - np.eye(4))) < 1e-12
    # and at the Greville points the oracle's values agree with the same formula
    Phi = kle.eigenfunctions(P, V)
    Bg = np.kron(*[splines.basis_matrix(P.knots[k], P.p[k], splines.greville(P.knots_t[k], P.pt[k]))
                   for k in (1, 0)])
    assert np.max(np.abs(Phi - Bg @ coeff / P.J[:, None])) < 1e-13
