"""The standard-form IBQ operator A~' of the oracle: setup, Algorithm 1, dense assembly.

Paper passages followed:
  * Sec. 4.1, eq. (cholesky): Z = Z_d x ... x Z_1 = L L^T with L = L_d x ... x L_1, and
    the standard form A' = L^{-1} A L^{-T}, v' = L^T v.
  * Sec. 4.2: interpolation of G(xhat, xhat') = Gamma(F(xhat), F(xhat')) sqrt(det DF(xhat)
    det DF(xhat')) (eq. integrand) at the Greville grid, Bt = Bt_d x ... x Bt_1,
    G~ = Bt^{-1} G Bt^{-T}, d LU factorizations.
  * Sec. 4.3, eq. (ApproxGalA_mat): A~ = M^T G~ M with M = M_d x ... x M_1.
  * Sec. 4.4.1: A~' = L^{-1} M^T Bt^{-1} J Gamma J Bt^{-T} M L^{-T}.
  * Sec. 4.4.2, Algorithm 1 (mf_eval): the nine stages of the matrix-free product.

Reading of Algorithm 1's index notation (its subscripts are ambiguous): stages 1 and 9
apply L^{-T} and L^{-1}, stages 3 and 7 apply Bt^{-T} and Bt^{-1}, which is the only
order consistent with the operator of Sec. 4.4.1 and with "stages six to nine are
equivalent to stages four to one".
"""

import numpy as np
import scipy.linalg as sla

from . import covariance, geometry, kron, splines


def _per_dir(v, d, default=None):
    if v is None:
        return [default] * d
    v = list(v)
    return (v + [v[-1]] * d)[:d]


class Problem:
    """All host data of one problem, built in FP64 from its description dict.

    desc keys: dim, degree[d], nelem[d] (open uniform knots) or knots[d] (explicit open knot
    vectors on [0, 1]; None entries fall back to nelem), optional interp_degree[d],
    interp_nelem[d] (default: the trial space) and interp_mult[d] (multiplicity of the
    interpolation space's interior breakpoints, default (or 0) 1; interp_mult =
    interp_degree gives the C^0 interpolation of Sec. 4.2, interp_degree + 1 a C^-1 one)
    or interp_knots[d], map (geometry dict), cov (covariance dict).  Interior knots may
    be repeated up to p + 1 times (C^-1): the Greville points at such a knot coincide and
    are evaluated from their own sides (splines.greville_sides), J included.
    """

    def __init__(self, desc):
        d = int(desc["dim"])
        self.d = d
        self.desc = desc
        p = _per_dir(desc["degree"], d)
        pt = _per_dir(desc.get("interp_degree"), d) if desc.get("interp_degree") else p
        pt = [p[k] if pt[k] in (0, None) else pt[k] for k in range(d)]
        # trial knots: explicit (Sec. 2.3, any open knot vector on [0, 1]) or open uniform
        given = list(desc.get("knots") or [None] * d) + [None] * d
        ne = _per_dir(desc.get("nelem"), d) if desc.get("nelem") else [None] * d
        self.knots = [np.asarray(given[k], dtype=np.float64) if given[k] is not None
                      else splines.open_uniform_knots(p[k], ne[k]) for k in range(d)]
        ne = [len(np.unique(self.knots[k])) - 1 for k in range(d)]
        net = _per_dir(desc.get("interp_nelem"), d) if desc.get("interp_nelem") else [0] * d
        mult = _per_dir(desc.get("interp_mult"), d) if desc.get("interp_mult") else [0] * d
        gt = list(desc.get("interp_knots") or [None] * d) + [None] * d
        self.knots_t = []
        for k in range(d):
            if gt[k] is not None:
                self.knots_t.append(np.asarray(gt[k], dtype=np.float64))
            elif given[k] is not None and pt[k] == p[k] and not net[k] and not mult[k]:
                self.knots_t.append(self.knots[k])            # the trial space itself
            else:
                nek = net[k] or ne[k]
                mk = int(mult[k]) or 1                            # 0 means the default, 1
                if mk < 1 or mk > pt[k] + 1:
                    raise ValueError("interp_mult must lie in 1..interp degree + 1")
                self.knots_t.append(splines.knots_with_multiplicity(pt[k], [j / nek for j in range(1, nek)], mk))
        net = [len(np.unique(self.knots_t[k])) - 1 for k in range(d)]
        self.p, self.ne, self.pt, self.net = p, ne, pt, net
        self.n = [splines.dimension(self.knots[k], p[k]) for k in range(d)]
        self.nt = [splines.dimension(self.knots_t[k], pt[k]) for k in range(d)]
        self.N = int(np.prod(self.n))
        self.Nt = int(np.prod(self.nt))
        # univariate matrices (Sec. 3.5, 4.1-4.3)
        self.Z = [splines.mass_matrix(self.knots[k], p[k]) for k in range(d)]
        self.L = [np.linalg.cholesky(Zk) for Zk in self.Z]
        self.Bt = [splines.collocation_matrix(self.knots_t[k], pt[k]) for k in range(d)]
        self.Bt_lu = [sla.lu_factor(B) for B in self.Bt]
        self.M = [splines.mixed_mass_matrix(self.knots_t[k], pt[k], self.knots[k], p[k])
                  for k in range(d)]
        # Greville grid in vec order (first index fastest), mapped points, J
        g1 = [splines.greville(self.knots_t[k], pt[k]) for k in range(d)]
        s1 = [splines.greville_sides(self.knots_t[k], pt[k]) for k in range(d)]
        grids = np.meshgrid(*g1, indexing="ij")
        self.xhat = np.stack([g.reshape(-1, order="F") for g in grids], axis=1)
        sgrids = np.meshgrid(*s1, indexing="ij")
        self.xhat_side = np.stack([g.reshape(-1, order="F") for g in sgrids], axis=1)
        self.X, det = geometry.map_points(desc["map"], self.xhat, self.xhat_side)
        if np.any(det <= 0):
            raise ValueError("det DF <= 0 at a Greville point")
        self.J = np.sqrt(det)
        self.cov = desc["cov"]

    # ---- Algorithm 1, one stage at a time -------------------------------------------
    def _modes(self, v, shape, fn_k):
        T = kron.to_tensor(v, shape)
        for k in range(self.d):
            T = kron.mode_apply(T, k, lambda A, k=k: fn_k(k, A))
        return kron.to_vec(T, self.d)

    def stage1(self, v):
        """V = L^{-T} v: back-substitution with the upper triangular L_k^T per direction."""
        return self._modes(v, self.n, lambda k, A: sla.solve_triangular(
            self.L[k], A, trans="T", lower=True))

    def stage2(self, V):
        """X = M V (mode products with M_k)."""
        return self._modes(V, self.n, lambda k, A: self.M[k] @ A)

    def stage3(self, X):
        """Y = Bt^{-T} X using the LU factors of Bt_k."""
        return self._modes(X, self.nt, lambda k, A: sla.lu_solve(self.Bt_lu[k], A, trans=1))

    def stage4(self, Y):
        """Y' = J (.) Y."""
        return self.J[:, None] * Y if Y.ndim == 2 else self.J * Y

    def stage5(self, Yp, rows_per_block=512):
        """Z' = Gamma Y', Gamma evaluated on the fly a block of rows at a time."""
        Z = np.zeros_like(Yp)
        for r0 in range(0, self.Nt, rows_per_block):
            r1 = min(self.Nt, r0 + rows_per_block)
            G = covariance.gamma(self.cov, self.X[r0:r1], self.X)
            Z[r0:r1] = G @ Yp
        return Z

    def stage6(self, Zp):
        """Z = J (.) Z'."""
        return self.stage4(Zp)

    def stage7(self, Z):
        """Y = Bt^{-1} Z using the LU factors of Bt_k."""
        return self._modes(Z, self.nt, lambda k, A: sla.lu_solve(self.Bt_lu[k], A, trans=0))

    def stage8(self, Y):
        """V = M^T Y."""
        return self._modes(Y, self.nt, lambda k, A: self.M[k].T @ A)

    def stage9(self, V):
        """v' = L^{-1} V: forward substitution with L_k per direction."""
        return self._modes(V, self.n, lambda k, A: sla.solve_triangular(
            self.L[k], A, trans="N", lower=True))

    def forward(self, v):
        """Stages 1-4: v' -> Y' (the input of stage 5)."""
        return self.stage4(self.stage3(self.stage2(self.stage1(v))))

    def backward(self, Zp):
        """Stages 6-9: Z' -> A~' v'."""
        return self.stage9(self.stage8(self.stage7(self.stage6(Zp))))

    def apply(self, v, stage5=None):
        """Algorithm 1: v' -> A~' v' for a vector (N,) or a block (N, b)."""
        v = np.asarray(v, dtype=np.float64)
        s5 = stage5 if stage5 is not None else self.stage5
        return self.backward(s5(self.forward(v)))

    # ---- dense forms (tiny and medium problems only) ----------------------------------
    def gamma_matrix(self):
        return covariance.gamma(self.cov, self.X, self.X)

    def dense_operator(self):
        """A~' = L^{-1} M^T Bt^{-1} J Gamma J Bt^{-T} M L^{-T} with explicit Kronecker
        matrices (Sec. 4.4.1); no mode-wise contraction is used here."""
        Lk = kron.kron_dense(self.L)
        Mk = kron.kron_dense(self.M)
        Bk = kron.kron_dense(self.Bt)
        G = self.J[:, None] * self.gamma_matrix() * self.J[None, :]
        Gt = np.linalg.solve(Bk, np.linalg.solve(Bk, G).T).T   # Bt^{-1} G Bt^{-T}
        A = Mk.T @ Gt @ Mk                                      # eq. ApproxGalA_mat
        Ap = np.linalg.solve(Lk, np.linalg.solve(Lk, A).T).T    # L^{-1} A L^{-T}
        return 0.5 * (Ap + Ap.T)

    def dense_A_tilde(self):
        """A~ = M^T G~ M (eq. ApproxGalA_mat), before the standard-form transformation."""
        Mk = kron.kron_dense(self.M)
        Bk = kron.kron_dense(self.Bt)
        G = self.J[:, None] * self.gamma_matrix() * self.J[None, :]
        Gt = np.linalg.solve(Bk, np.linalg.solve(Bk, G).T).T
        return Mk.T @ Gt @ Mk

    def mass_dense(self):
        return kron.kron_dense(self.Z)

    def to_coefficients(self, vp):
        """v = L^{-T} v' (Sec. 4.1): B-spline coefficients of phi_h = sum v_i B_i / sqrt(det DF)."""
        return self.stage1(vp)
