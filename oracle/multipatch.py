"""Multipatch problems of the oracle (test infrastructure; plain FP64).

Paper passages followed:
  * Sec. 3.6 (discretization of multipatch geometries): the integral operator has no
    derivatives, so the method carries over to domains made of several patches; a
    non-conforming (C^-1) discretization needs only a minor change.  Here every patch keeps
    its own tensor-product trial space, interpolation space and geometry map; the trial
    space of the domain is the direct sum of the patch spaces.
  * Sec. 3.4-3.5: with basis functions B_i / sqrt(det DF) on each patch, the Gramian is the
    block-diagonal matrix of the patches' parametric Gramians, each a Kronecker product, so
    the standard form of Sec. 4.1 holds patch by patch.
  * Algorithm 1: stages 1-4 and 6-9 act on each patch separately (block-diagonal Kronecker
    factors); stage 5 couples all patches: Gamma is evaluated between the mapped Greville
    points of every pair of patches.

Vector layout: patch 0's N_0 standard-form coefficients (vec order), then patch 1's, ...;
points and J likewise.
"""

import numpy as np

from . import covariance, operator


class MultipatchProblem:
    """Patches described by single-patch description dicts that share dim and cov."""

    def __init__(self, descs):
        if not descs:
            raise ValueError("need at least one patch")
        self.patches = [operator.Problem(d) for d in descs]
        d0 = descs[0]
        for d in descs[1:]:
            if int(d["dim"]) != int(d0["dim"]):
                raise ValueError("patches of different dimension")
            if d["cov"] != d0["cov"]:
                raise ValueError("patches must share the covariance")
        self.d = int(d0["dim"])
        self.cov = d0["cov"]
        self.noff = np.cumsum([0] + [P.N for P in self.patches])
        self.toff = np.cumsum([0] + [P.Nt for P in self.patches])
        self.N = int(self.noff[-1])
        self.Nt = int(self.toff[-1])
        self.X = np.concatenate([P.X for P in self.patches], axis=0)
        self.J = np.concatenate([P.J for P in self.patches])

    def stage5(self, Yp, rows_per_block=512):
        """Z' = Gamma Y' over the points of all patches."""
        Z = np.zeros_like(Yp)
        for r0 in range(0, self.Nt, rows_per_block):
            r1 = min(self.Nt, r0 + rows_per_block)
            Z[r0:r1] = covariance.gamma(self.cov, self.X[r0:r1], self.X) @ Yp
        return Z

    def apply(self, v, stage5=None):
        """Algorithm 1 patch by patch around one stage 5 over all points."""
        v = np.asarray(v, dtype=np.float64)
        one = v.ndim == 1
        V = v[:, None] if one else v
        Y = np.concatenate([P.forward(V[self.noff[i]:self.noff[i + 1]])
                            for i, P in enumerate(self.patches)], axis=0)
        Z = (stage5 or self.stage5)(Y)
        out = np.concatenate([P.backward(Z[self.toff[i]:self.toff[i + 1]])
                              for i, P in enumerate(self.patches)], axis=0)
        return out[:, 0] if one else out

    def dense_operator(self):
        """A~' assembled column by column from the matrix-free product (small problems)."""
        A = self.apply(np.eye(self.N))
        return 0.5 * (A + A.T)

    def to_coefficients(self, vp):
        """v = L^{-T} v' patch by patch (Sec. 4.1)."""
        vp = np.asarray(vp, dtype=np.float64)
        return np.concatenate([P.to_coefficients(vp[self.noff[i]:self.noff[i + 1]])
                               for i, P in enumerate(self.patches)], axis=0)
