"""FP64 CPU oracle for the matrix-free isogeometric Galerkin Karhunen-Loeve method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call, link or execute anything in this package.  Only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.

The oracle follows Mika, Hughes, Schillinger, Wriggers and Hiemstra, "A matrix-free
isogeometric Galerkin method for Karhunen-Loeve approximation of random fields using
tensor product splines, tensor contraction and interpolation based quadrature"
(arXiv 2011.13861).  It is deliberately plain and slow: every function states the
passage of the paper it follows, and no blocking, fusion or reordering is done
beyond what that passage states.  It shares no code with the GPU path.

Modules
-------
splines     knot vectors, Cox-de Boor B-splines, Greville abscissae, univariate
            mass / mixed-mass / collocation matrices (Sec. 2.3, Sec. 3.5, Sec. 4.2-4.3)
geometry    geometry maps F and det DF (Sec. 2.4, eq. (integrand))
covariance  covariance kernels Gamma(x, x') (Sec. 3.1, eq. (kernel), Fig. kernels)
kron        mode-k tensor contraction (Sec. 2.2)
operator    Algorithm 1 (matrix-free apply), literal stages 1-9, and the dense
            standard-form operator assembled column by column (Sec. 4.4)
multipatch  several patches with their own spaces and maps, coupled by stage 5 only
            (Sec. 3.6, non-conforming multipatch domains)
kle         truncated KL expansion at the Greville points (Sec. 3.2)
eigs        eigenpairs of the standard-form problem (Sec. 4.1, Sec. 4.4.2)
analytic    closed-form eigenpairs of the 1D exponential kernel (Sec. 6.1 remark)
galerkin    brute-force full Galerkin matrix A (eq. (GalA_mat)) on tiny meshes
mlp         FP64 reference multilayer perceptron (forward, backward, loss)
cstage5     C/OpenMP FP64 stage 5, used only to time the oracle on host cores

Functions without an independent pin say "parity unpinned" in their docstring.
"""

from . import splines, geometry, covariance, kron, operator, eigs, analytic  # noqa: F401
