"""Univariate B-spline machinery of the oracle (plain FP64, loops over definitions).

Paper passages followed:
  * Sec. 2.3 (B-splines): univariate basis of degree p and dimension n on [0, 1],
    tensor-product multivariate basis.
  * Sec. 6.1 and the Example sections: knot vectors are open and uniform with
    C^{p-1} continuity under h-refinement, so n = nelem + p.
  * Sec. 4.2 (interpolation based quadrature): collocation at the Greville abscissae,
    univariate collocation matrices  Bt_k[i, j] = Bt_j(xhat_i)  (eq. interpolation_matrix).
  * Sec. 3.5 + Remark massmatrix: univariate Gramian  Z_k[i, j] = int_0^1 B_i B_j,
    Gauss-Legendre with p + 1 points per element (eq. univariate_mass_matrix).
  * Sec. 4.3: univariate mixed mass matrix  M_k[i, j] = int_0^1 Bt_i B_j
    (eq. univariate_mass_matrix2), "computed up to machine precision".

Readings where the paper is silent:
  * The Greville abscissae are only cited; they are taken as the knot averages
    xhat_i = (xi_{i+1} + ... + xi_{i+p}) / p  (de Boor's definition).
  * For M_k the union of both breakpoint sets is used with ceil((p + pt + 1) / 2)
    Gauss points per span, which is exact for the degree p + pt integrand.
  * At x = 1 the basis is taken as the left limit (the last function equals 1).
  * Sec. 6 uses interpolation spaces that are discontinuous (C^-1) across a C^0 line of
    the geometry: an interior knot repeated p + 1 times.  The space then splits into the
    functions left and right of the knot, and the last function on the left and the
    first on the right have the same Greville abscissa (the knot).  Each such point is
    evaluated as a limit from the side of its own function: from the left when the
    abscissa is the right end of its function's support (which also covers x = 1), from
    the right otherwise.  With that the collocation matrix stays invertible.
"""

import math

import numpy as np


def open_uniform_knots(p, nelem):
    """Open uniform knot vector of degree p with nelem elements on [0, 1].

    End knots are repeated p + 1 times, interior breakpoints j / nelem appear once,
    giving C^{p-1} continuity and dimension n = nelem + p (Sec. 6.1).
    """
    if p < 0 or nelem < 1:
        raise ValueError("need p >= 0 and nelem >= 1")
    interior = [j / nelem for j in range(1, nelem)]
    return np.array([0.0] * (p + 1) + interior + [1.0] * (p + 1), dtype=np.float64)


def knots_with_multiplicity(p, breakpoints, mult):
    """Open knot vector with given interior breakpoints repeated `mult` times each.

    mult = p gives C^0 continuity at every breakpoint (reduced-continuity
    interpolation spaces discussed in Sec. 4.2 remark on smoothness); mult = p + 1 a
    discontinuous (C^-1) space.
    """
    interior = []
    for b in breakpoints:
        interior += [float(b)] * mult
    return np.array([0.0] * (p + 1) + interior + [1.0] * (p + 1), dtype=np.float64)


def dimension(knots, p):
    return len(knots) - p - 1


def _span_of_right_end(knots):
    """Index of the last non-empty knot span (used for the left limit at x = 1)."""
    m = len(knots) - 1
    for i in range(m - 1, -1, -1):
        if knots[i] < knots[i + 1]:
            return i
    raise ValueError("degenerate knot vector")


def basis_matrix(knots, p, x, side=None):
    """All B-splines B_{i,p}(x_r) by the Cox-de Boor recursion from its definition.

    B_{i,0}(x) = 1 on [xi_i, xi_{i+1}) and 0 otherwise;
    B_{i,q}(x) = (x - xi_i)/(xi_{i+q} - xi_i) B_{i,q-1}(x)
               + (xi_{i+q+1} - x)/(xi_{i+q+1} - xi_{i+1}) B_{i+1,q-1}(x),  0/0 := 0.
    side[r] = -1 takes the limit from the left at x_r instead: B_{i,0} = 1 on
    (xi_i, xi_{i+1}]; None or +1 the definition above (with the left limit at x = 1).
    Returns an array of shape (len(x), n).
    """
    knots = np.asarray(knots, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    sides = np.ones(len(x)) if side is None else np.broadcast_to(np.asarray(side), (len(x),))
    m = len(knots) - 1
    n = m - p
    last = _span_of_right_end(knots)
    out = np.zeros((len(x), n))
    for r, xv in enumerate(x):
        # degree-0 functions, one per knot span
        b = np.zeros(m)
        for i in range(m):
            if sides[r] < 0:
                if knots[i] < xv <= knots[i + 1]:
                    b[i] = 1.0
            elif knots[i] <= xv < knots[i + 1]:
                b[i] = 1.0
        if sides[r] >= 0 and xv == knots[-1]:
            b[last] = 1.0
        for q in range(1, p + 1):
            nb = np.zeros(m - q)
            for i in range(m - q):
                val = 0.0
                den1 = knots[i + q] - knots[i]
                if den1 > 0.0:
                    val += (xv - knots[i]) / den1 * b[i]
                den2 = knots[i + q + 1] - knots[i + 1]
                if den2 > 0.0:
                    val += (knots[i + q + 1] - xv) / den2 * b[i + 1]
                nb[i] = val
            b = nb
        out[r, :] = b[:n]
    return out


def greville(knots, p):
    """Greville abscissae xhat_i = mean(xi_{i+1}, ..., xi_{i+p})  (Sec. 4.2, cited); the
    knot itself where those p knots coincide (so that the two abscissae at a C^-1 knot are
    equal)."""
    knots = np.asarray(knots, dtype=np.float64)
    n = dimension(knots, p)
    if p == 0:
        return 0.5 * (knots[:-1] + knots[1:])[:n]
    return np.array([knots[i + 1] if knots[i + 1] == knots[i + p] else knots[i + 1:i + p + 1].sum() / p
                     for i in range(n)])


def greville_sides(knots, p):
    """-1 where the abscissa of B_i is the right end of its support [xi_i, xi_{i+p+1}] (the
    knots xi_{i+1} .. xi_{i+p+1} coincide: the left function at a C^-1 knot, and the last
    function at x = 1), else +1: the side from which the basis is evaluated there."""
    knots = np.asarray(knots, dtype=np.float64)
    n = dimension(knots, p)
    return np.array([-1.0 if p > 0 and knots[i + 1] == knots[i + p + 1] else 1.0 for i in range(n)])


def collocation_matrix(knots, p):
    """Bt_k[i, j] = Bt_j(xhat_i) at the Greville abscissae (eq. interpolation_matrix), each
    abscissa evaluated from its own side (greville_sides)."""
    return basis_matrix(knots, p, greville(knots, p), greville_sides(knots, p))


def gauss_legendre(q):
    """q-point Gauss-Legendre rule on [-1, 1] (library primitive)."""
    return np.polynomial.legendre.leggauss(q)


def _composite_gauss(breaks, q):
    """Nodes and weights of a q-point Gauss rule on every non-empty span of `breaks`."""
    t, w = gauss_legendre(q)
    xs, ws = [], []
    for a, b in zip(breaks[:-1], breaks[1:]):
        if b <= a:
            continue
        xs.append(0.5 * (b - a) * t + 0.5 * (b + a))
        ws.append(0.5 * (b - a) * w)
    return np.concatenate(xs), np.concatenate(ws)


def mass_matrix(knots, p):
    """Univariate Gramian Z_k[i, j] = int_0^1 B_i B_j dx (eq. univariate_mass_matrix).

    Gauss-Legendre with p + 1 points per element (Remark massmatrix).
    """
    breaks = np.unique(knots)
    x, w = _composite_gauss(breaks, p + 1)
    B = basis_matrix(knots, p, x)
    n = B.shape[1]
    Z = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            Z[i, j] = np.sum(w * B[:, i] * B[:, j])
    return Z


def mixed_mass_matrix(knots_t, pt, knots, p):
    """M_k[i, j] = int_0^1 Bt_i B_j dx, Bt from the interpolation space (eq.
    univariate_mass_matrix2); shape (nt, n).  Gauss points on the union of both
    breakpoint sets, ceil((p + pt + 1)/2) per span (exact for degree p + pt)."""
    breaks = np.union1d(np.unique(knots_t), np.unique(knots))
    q = int(math.ceil((p + pt + 1) / 2.0))
    x, w = _composite_gauss(breaks, q)
    Bt = basis_matrix(knots_t, pt, x)
    B = basis_matrix(knots, p, x)
    M = np.zeros((Bt.shape[1], B.shape[1]))
    for i in range(Bt.shape[1]):
        for j in range(B.shape[1]):
            M[i, j] = np.sum(w * Bt[:, i] * B[:, j])
    return M


def basis_integrals(knots, p):
    """int_0^1 B_i dx = (xi_{i+p+1} - xi_i) / (p + 1), the closed form used as a pin."""
    knots = np.asarray(knots)
    n = dimension(knots, p)
    return np.array([(knots[i + p + 1] - knots[i]) / (p + 1) for i in range(n)])
