"""Writes tests/golden/cube24_eigs.npz: the oracle's leading eigenpairs of the 3D workload
(sine-perturbed unit cube, 24^3 elements, quadratic splines, exponential kernel with
correlation length 0.5; 17,576 dofs).

Calls only the oracle: ARPACK (scipy eigsh, the implicitly restarted Lanczos family the
paper uses, Sec. 4.4.2) on the literal Algorithm 1 with the C/OpenMP FP64 stage 5, at
tolerance 1e-13.  Stored: the 58 leading eigenvalues (FP64), the 50 leading unit
eigenvectors v' (rounded to FP32: entry errors below 1e-9, far below the 1e-5 bar of the
parity test), their sign fixed by a positive sum, and the oracle's FP64 residual norms.

Usage (repo root): python tests/golden/make_cube24_eigs.py
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import cstage5, operator  # noqa: E402
from oracle import eigs as oeigs  # noqa: E402

K_VALUES, K_VECTORS = 58, 50


def main():
    desc, k, _ = workloads.config("cube24")
    assert k == K_VECTORS
    P = operator.Problem(desc)
    s5 = lambda Y: cstage5.stage5(P, Y)   # noqa: E731
    v0 = np.ones(P.N)
    t = time.time()
    w, V = oeigs.iterative_eigs(P, K_VALUES, tol=1e-13, stage5=s5, v0=v0)
    dt = time.time() - t
    V = V[:, :K_VECTORS]
    V = V * np.where(V.sum(axis=0) < 0, -1.0, 1.0)[None, :]
    r = np.linalg.norm(P.apply(V, stage5=s5) - V * w[None, :K_VECTORS], axis=0)
    out = os.path.join(HERE, "cube24_eigs.npz")
    np.savez_compressed(out, evals=w, evecs=V.astype(np.float32), residuals=r,
                        seconds=dt, source=np.array("oracle ARPACK eigsh tol 1e-13, C stage 5"))
    print("wrote", out, "in %.0f s; max residual / lambda %.2e" % (dt, np.max(r / w[:K_VECTORS])))


if __name__ == "__main__":
    main()
