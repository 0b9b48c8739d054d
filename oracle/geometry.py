"""Geometry maps F : [0,1]^d -> D and their Jacobian determinants (oracle, FP64).

Paper passages followed:
  * Sec. 2.4: F maps parametric points to physical points, det DF > 0 everywhere;
    F is represented by NURBS.
  * eq. (integrand): the scaled kernel needs sqrt(det DF) at the Greville points,
    and Algorithm 1 takes J = sqrt(det DF) at the Greville grid as input.

Map kinds (dicts with a "kind" key):
  identity        F(u) = u
  box             F(u) = lo + (hi - lo) * u
  annulus_nurbs   2D quarter annulus r in [r0, r1] as an exact NURBS surface: degree 1
                  in the radial and degree 2 in the angular direction, one element each,
                  angular weights (1, 1/sqrt 2, 1).  Evaluated with the generic rational
                  tensor-product formula below, derivatives by the quotient rule.
  annulus_polar   (r0 + (r1 - r0) u) (cos(pi v / 2), sin(pi v / 2)), a cross-check with
                  the same physical domain
  sine_cube       F(u) = u + eps * amp * prod_k sin(pi u_k): identity on the boundary
  tensor_nurbs    a general d-variate NURBS map (Sec. 2.3-2.4): "degree" [d], "knots" [d]
                  open knot vectors on [0, 1], "ctrl" (m_1, ..., m_d, d) control points,
                  optional "weights" (m_1, ..., m_d); F = sum_a w_a P_a N_a / sum_a w_a N_a
                  with N_a the tensor-product B-splines, derivatives by the quotient rule
  any of the above may carry "rotation" (d x d orthogonal) and "shift" (d) applied after
  F; det DF is unchanged by them.

Readings: the quarter annulus and the perturbed cube are not in the paper; they are
the synthetic stand-ins for its NURBS geometries (whose control points are not
printed).
"""

import math

import numpy as np

from . import splines


def _bspline_derivative_matrix(knots, p, x, side=None):
    """d/dx B_{i,p}(x) = p/(xi_{i+p}-xi_i) B_{i,p-1} - p/(xi_{i+p+1}-xi_{i+1}) B_{i+1,p-1}
    (one-sided at a knot where the map is only C^0: side -1 from the left, else from the right)."""
    n = splines.dimension(knots, p)
    out = np.zeros((len(x), n))
    if p == 0:
        return out
    lower = splines.basis_matrix(knots, p - 1, x, side)  # n + 1 functions
    for i in range(n):
        d1 = knots[i + p] - knots[i]
        d2 = knots[i + p + 1] - knots[i + 1]
        if d1 > 0:
            out[:, i] += p / d1 * lower[:, i]
        if d2 > 0:
            out[:, i] -= p / d2 * lower[:, i + 1]
    return out


def nurbs_surface(ku, pu, kv, pv, ctrl, weights, u, v):
    """Rational tensor-product surface S(u,v) = sum_ab N_a M_b w_ab P_ab / W and its
    parametric derivatives.  ctrl has shape (nu, nv, 2), weights (nu, nv).
    Returns (S, dS/du, dS/dv) with shapes (npts, 2)."""
    Nu = splines.basis_matrix(ku, pu, u)
    Nv = splines.basis_matrix(kv, pv, v)
    dNu = _bspline_derivative_matrix(ku, pu, u)
    dNv = _bspline_derivative_matrix(kv, pv, v)
    npts = len(u)
    S = np.zeros((npts, 2))
    Su = np.zeros((npts, 2))
    Sv = np.zeros((npts, 2))
    for r in range(npts):
        W = Wu = Wv = 0.0
        A = np.zeros(2)
        Au = np.zeros(2)
        Av = np.zeros(2)
        for a in range(ctrl.shape[0]):
            for b in range(ctrl.shape[1]):
                w = weights[a, b]
                W += Nu[r, a] * Nv[r, b] * w
                Wu += dNu[r, a] * Nv[r, b] * w
                Wv += Nu[r, a] * dNv[r, b] * w
                A += Nu[r, a] * Nv[r, b] * w * ctrl[a, b]
                Au += dNu[r, a] * Nv[r, b] * w * ctrl[a, b]
                Av += Nu[r, a] * dNv[r, b] * w * ctrl[a, b]
        S[r] = A / W
        Su[r] = (Au - S[r] * Wu) / W
        Sv[r] = (Av - S[r] * Wv) / W
    return S, Su, Sv


def _quarter_annulus_nurbs(r0, r1):
    ku = np.array([0.0, 0.0, 1.0, 1.0])
    kv = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])
    ctrl = np.zeros((2, 3, 2))
    weights = np.zeros((2, 3))
    for a, r in enumerate((r0, r1)):
        ctrl[a, 0] = (r, 0.0)
        ctrl[a, 1] = (r, r)
        ctrl[a, 2] = (0.0, r)
        weights[a] = (1.0, 1.0 / math.sqrt(2.0), 1.0)
    return ku, 1, kv, 2, ctrl, weights


def tensor_nurbs(degree, knots, ctrl, weights, u, side=None):
    """F(u) and DF(u) (shape (npts, d, d), D[r, i, j] = dF_i / du_j) of a d-variate NURBS map.
    Sums over the control net are written as tensor contractions of the per-direction basis
    matrices N_k (npts x m_k) and their derivatives, with the weights folded into the
    homogeneous control points (w P, w).  side (npts, d) of +-1: the side from which each
    coordinate is approached (it matters for DF on the C^0 lines of the map only)."""
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    npts, d = u.shape
    sd = np.ones((npts, d)) if side is None else np.asarray(side, dtype=np.float64).reshape(npts, d)
    ctrl = np.asarray(ctrl, dtype=np.float64)
    w = np.ones(ctrl.shape[:d]) if weights is None else np.asarray(weights, dtype=np.float64)
    Pw = np.concatenate([ctrl * w[..., None], w[..., None]], axis=-1)   # homogeneous (m_1..m_d, d + 1)
    N = [splines.basis_matrix(np.asarray(knots[k], dtype=np.float64), degree[k], u[:, k], sd[:, k])
         for k in range(d)]
    dN = [_bspline_derivative_matrix(np.asarray(knots[k], dtype=np.float64), degree[k], u[:, k], sd[:, k])
          for k in range(d)]
    letters = "abc"[:d]
    spec = ",".join("r" + letters[k] for k in range(d)) + "," + letters + "h->rh"

    def contract(mats):
        return np.einsum(spec, *mats, Pw)

    H = contract(N)                                   # (npts, d + 1): A and W
    X = H[:, :d] / H[:, d:]
    D = np.zeros((npts, d, d))
    for j in range(d):
        Hj = contract([dN[k] if k == j else N[k] for k in range(d)])
        D[:, :, j] = (Hj[:, :d] - X * Hj[:, d:]) / H[:, d:]
    return X, D


def map_points(geom, u, side=None):
    """Physical points F(u) and det DF(u) for parametric points u of shape (npts, d); side
    (npts, d) of +-1 selects one-sided derivatives on the C^0 lines of a tensor NURBS map
    (the other maps are smooth)."""
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    npts, d = u.shape
    kind = geom["kind"]
    if kind == "identity":
        X = u.copy()
        D = np.broadcast_to(np.eye(d), (npts, d, d)).copy()
    elif kind == "box":
        lo = np.asarray(geom["lo"], dtype=np.float64)
        hi = np.asarray(geom["hi"], dtype=np.float64)
        X = lo + (hi - lo) * u
        D = np.broadcast_to(np.diag(hi - lo), (npts, d, d)).copy()
    elif kind == "annulus_nurbs":
        if d != 2:
            raise ValueError("annulus_nurbs is a 2D map")
        ku, pu, kv, pv, ctrl, w = _quarter_annulus_nurbs(geom.get("r0", 1.0), geom.get("r1", 2.0))
        S, Su, Sv = nurbs_surface(ku, pu, kv, pv, ctrl, w, u[:, 0], u[:, 1])
        X = S
        D = np.stack([Su, Sv], axis=2)  # D[r, i, j] = dF_i / du_j
    elif kind == "annulus_polar":
        if d != 2:
            raise ValueError("annulus_polar is a 2D map")
        r0, r1 = geom.get("r0", 1.0), geom.get("r1", 2.0)
        r = r0 + (r1 - r0) * u[:, 0]
        th = 0.5 * math.pi * u[:, 1]
        X = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
        D = np.zeros((npts, 2, 2))
        D[:, 0, 0] = (r1 - r0) * np.cos(th)
        D[:, 1, 0] = (r1 - r0) * np.sin(th)
        D[:, 0, 1] = -r * 0.5 * math.pi * np.sin(th)
        D[:, 1, 1] = r * 0.5 * math.pi * np.cos(th)
    elif kind == "sine_cube":
        eps = geom.get("eps", 0.05)
        amp = np.asarray(geom.get("amp", [1.0, 0.5, 0.25])[:d], dtype=np.float64)
        s = np.prod(np.sin(math.pi * u), axis=1)
        grad = np.zeros((npts, d))
        for k in range(d):
            g = math.pi * np.cos(math.pi * u[:, k])
            for m in range(d):
                if m != k:
                    g = g * np.sin(math.pi * u[:, m])
            grad[:, k] = g
        X = u + eps * s[:, None] * amp[None, :]
        D = np.broadcast_to(np.eye(d), (npts, d, d)).copy()
        D += eps * amp[None, :, None] * grad[:, None, :]
    elif kind == "tensor_nurbs":
        X, D = tensor_nurbs(geom["degree"], geom["knots"], geom["ctrl"], geom.get("weights"), u, side)
    else:
        raise ValueError("unknown map kind %r" % kind)
    if "rotation" in geom:
        Q = np.asarray(geom["rotation"], dtype=np.float64)
        X = X @ Q.T
        D = np.einsum("ij,rjk->rik", Q, D)
    if "shift" in geom:
        X = X + np.asarray(geom["shift"], dtype=np.float64)
    det = np.linalg.det(D)
    return X, det


def domain_measure(geom, d, q=12, nsub=8):
    """|D| = int det DF over the parametric cube by a tensor Gauss rule (for pins)."""
    t, w = splines.gauss_legendre(q)
    xs, ws = [], []
    for s in range(nsub):
        a, b = s / nsub, (s + 1) / nsub
        xs.append(0.5 * (b - a) * t + 0.5 * (a + b))
        ws.append(0.5 * (b - a) * w)
    x1 = np.concatenate(xs)
    w1 = np.concatenate(ws)
    grids = np.meshgrid(*([x1] * d), indexing="ij")
    wgrid = np.ones_like(grids[0])
    for g in np.meshgrid(*([w1] * d), indexing="ij"):
        wgrid = wgrid * g
    u = np.stack([g.ravel() for g in grids], axis=1)
    _, det = map_points(geom, u)
    return float(np.sum(wgrid.ravel() * det))
