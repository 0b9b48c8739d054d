"""Learned warm start for the block eigensolver (argument marshalling over kl_mlp_* and
kl_eigs; every computation runs in the HIP library).

The paper starts its Lanczos iteration from a generic vector (Sec. 4.4.2).  Here a
network trained on eigenpairs that the method itself computed maps covariance
parameters (correlation length L, anisotropy ratio a, smoothness flag: 0 = exponential,
1 = squared exponential) to a block of k eigenvector coefficient vectors v' (standard
form, Sec. 4.1), which kl_eigs orthonormalises and uses as its start block.  The plain
random start stays the fallback: a prediction that is not finite is not used.

Network input: (log L, log a, 2 flag - 1).  Output: k N values, eigenvector i at
[i N, (i + 1) N), scaled by sqrt(N) so that the entries are of order one.  Loss: the
sign-invariant squared error per eigenvector (kl_mlp_gradients with group = N) plus, with
weight `subspace`, the part of each predicted eigenvector outside the span of the k
target eigenvectors (kl_mlp_set_subspace), which does not care how eigenvectors of a
cluster are rotated among themselves: near eigenvalue crossings over the parameters the
per-eigenvector targets jump, the span does not.
"""

import math

import numpy as np

from ._binding import KL_ENUMERIC, MLP, KLError


def features(L, a, flag):
    """Network inputs for arrays (or scalars) of parameters: (n, 3) float32."""
    L = np.atleast_1d(np.asarray(L, dtype=np.float64))
    a = np.atleast_1d(np.asarray(a, dtype=np.float64))
    flag = np.atleast_1d(np.asarray(flag, dtype=np.float64))
    return np.stack([np.log(L), np.log(a), 2.0 * flag - 1.0], axis=1).astype(np.float32)


def generate(problem, covs, k, block=16, tol=1e-10, precision="f64"):
    """Eigenvector targets for a list of covariances (kind, sigma2, corr_len) on one
    problem handle (kl_set_cov + kl_eigs per entry).  Returns (targets: CUDA float32
    (n, k N) scaled by sqrt(N), eigenvalues (n, k), reports)."""
    import torch
    N = problem.N
    out = torch.empty((len(covs), k * N), dtype=torch.float32, device="cuda")
    evals = np.zeros((len(covs), k))
    reports = []
    scale = math.sqrt(N)
    for i, (kind, sigma2, ell) in enumerate(covs):
        problem.set_cov(kind, sigma2, ell)
        w, V, rep = problem.eigs(k, precision=precision, block=block, tol=tol)
        out[i] = (V.T * scale).reshape(-1).float()
        evals[i] = w
        reports.append(rep)
    torch.cuda.synchronize()
    return out, evals, reports


class WarmStart:
    """Network (3 -> hidden... -> k N) trained on the GPU; predicts start blocks."""

    def __init__(self, N, k, hidden=(256, 256), seed=0):
        self.N, self.k = int(N), int(k)
        self.net = MLP([3, *hidden, self.k * self.N], seed=seed)

    def fit(self, feats, targets, epochs=200, batch=64, lr0=1e-3, lr1=3e-5, seed=0, subspace=3.0):
        """Trains on (n, 3) inputs and (n, k N) targets; returns the per-epoch loss."""
        import torch
        x = torch.as_tensor(np.ascontiguousarray(feats, dtype=np.float32)).cuda()
        self.net.set_subspace(subspace)
        return self.net.train(x, targets, group=self.N, epochs=epochs, batch=batch, lr0=lr0, lr1=lr1, seed=seed)

    def predict(self, feats):
        """Raw network outputs (n, k N), CUDA float32."""
        import torch
        x = torch.as_tensor(np.ascontiguousarray(feats, dtype=np.float32)).cuda()
        return self.net.forward(x)

    def start_block(self, feat):
        """Start block for one input row: CUDA float64 (N, k), column-major, or None if
        the prediction is not finite."""
        import torch
        y = self.predict(np.asarray(feat, dtype=np.float32).reshape(1, 3))[0]
        if not bool(torch.isfinite(y).all()):
            return None
        return y.view(self.k, self.N).double().T


def solve(problem, k, warm=None, feat=None, **eigs_kwargs):
    """kl_eigs with the predicted start block when one is available and finite, else
    (or if kl_eigs rejects the block as non-finite) the seeded random start."""
    x0 = warm.start_block(feat) if (warm is not None and feat is not None) else None
    if x0 is not None:
        try:
            return problem.eigs(k, x0=x0, **eigs_kwargs)
        except KLError as e:
            if e.status != KL_ENUMERIC:
                raise
    return problem.eigs(k, **eigs_kwargs)
