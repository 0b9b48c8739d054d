"""The learned warm start (network trained on the GPU on eigenpairs the method computed)
against the plain random start, on the 48 x 48 cubic quarter annulus with parameters
drawn as L ~ logU[0.1, 2], a ~ logU[0.5, 2], flag ~ B(1/2).

The prediction's error is measured by the oracle: residuals of the Rayleigh-Ritz
vectors of the predicted block under the oracle operator.  The gain test trains on a
reduced set (300 draws of the training seed) to keep the test short.
"""

import numpy as np
import pytest
import torch

import paper_2011_13861_amd as kl
import workloads
from paper_2011_13861_amd import warmstart
from oracle import cstage5, operator

pytestmark = pytest.mark.gpu

K = 16
N_TRAIN = 300
N_TEST = 8


def _covs(L, a, flag):
    out = []
    for Li, ai, fi in zip(L, a, flag):
        d = workloads.mlp_problem(Li, ai, fi)
        out.append((d["cov"]["kind"], d["cov"]["sigma2"], d["cov"]["corr_len"]))
    return out


@pytest.fixture(scope="module")
def trained():
    L, a, flag = workloads.mlp_parameters(2000, N_TRAIN)
    G = kl.Problem(workloads.mlp_problem(1.0, 1.0, 0))
    T, _, _ = warmstart.generate(G, _covs(L, a, flag), K, block=16, tol=1e-10)
    ws = warmstart.WarmStart(G.N, K, seed=0)
    losses = ws.fit(warmstart.features(L, a, flag), T, epochs=300, batch=32, lr0=1e-3, lr1=3e-5)
    return G, ws, losses


def test_set_cov_matches_fresh_setup():
    """kl_set_cov on an existing handle gives the same operator as a fresh kl_setup."""
    d1 = workloads.mlp_problem(0.3, 1.5, 1)
    G = kl.Problem(workloads.mlp_problem(1.0, 1.0, 0))
    G.set_cov(d1["cov"]["kind"], d1["cov"]["sigma2"], d1["cov"]["corr_len"])
    F = kl.Problem(d1)
    V = kl.to_device_block(workloads.random_block(G.N, 5, seed=1))
    for prec in ("f64", "f32"):
        y1, y2 = kl.new_block(G.N, 5), kl.new_block(G.N, 5)
        G.apply(V, y1, prec)
        F.apply(V, y2, prec)
        torch.cuda.synchronize()
        assert torch.equal(y1, y2), prec


def test_training_converges(trained):
    _, _, losses = trained
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.2 * losses[0], (losses[0], losses[-1])


def test_prediction_error_measured_by_oracle(trained):
    """Rayleigh-Ritz on the predicted block under the oracle operator: relative
    residuals of the leading Ritz pairs are far below those of a random block."""
    G, ws, _ = trained
    L, a, flag = workloads.mlp_parameters(2001, 2)
    for i in range(2):
        desc = workloads.mlp_problem(L[i], a[i], flag[i])
        P = operator.Problem(desc)
        s5 = lambda Y: cstage5.stage5(P, Y)  # noqa: E731
        W = ws.start_block(warmstart.features(L[i], a[i], flag[i])[0]).cpu().numpy()
        R = workloads.random_block(P.N, K, seed=7)

        def ritz_residuals(B):
            Q, _ = np.linalg.qr(B)
            AQ = P.apply(Q, stage5=s5)
            w, S = np.linalg.eigh(Q.T @ AQ)
            order = np.argsort(w)[::-1]
            w, S = w[order], S[:, order]
            res = np.linalg.norm(AQ @ S - (Q @ S) * w, axis=0) / np.abs(w)
            return res[:8]
        r_warm = ritz_residuals(W)
        r_rand = ritz_residuals(R)
        assert np.median(r_warm) < 0.1 * np.median(r_rand), (r_warm, r_rand)


def test_warm_start_gain(trained):
    """Held-out draws: the FP32 solve (with FP64 refinement) from the predicted block
    needs fewer operator applications than from a random block, and both meet the
    criterion under the FP64 operator with the same eigenvalues."""
    G, ws, _ = trained
    L, a, flag = workloads.mlp_parameters(2001, N_TEST)
    n_warm, n_rand = [], []
    for i, cov in enumerate(_covs(L, a, flag)):
        G.set_cov(*cov)
        f = warmstart.features(L[i], a[i], flag[i])[0]
        w1, _, r1 = warmstart.solve(G, K, ws, f, precision="f32", block=16, tol=1e-6)
        w0, _, r0 = G.eigs(K, precision="f32", block=16, tol=1e-6)
        assert r1["converged"] == K and r0["converged"] == K
        assert np.max(np.abs(w1 - w0) / w0) <= 2e-6
        n_warm.append(sum(r1["n_applies"]))
        n_rand.append(sum(r0["n_applies"]))
    assert np.mean(n_warm) < np.mean(n_rand), (n_warm, n_rand)


def test_non_finite_prediction_falls_back():
    G = kl.Problem(workloads.mlp_problem(0.5, 1.0, 1))
    bad = torch.full((K, G.N), float("nan"), dtype=torch.float64, device="cuda").T
    with pytest.raises(kl.KLError):
        G.eigs(K, x0=bad, block=16)

    class Broken:
        def start_block(self, feat):
            return bad
    w, _, rep = warmstart.solve(G, K, Broken(), np.zeros(3, np.float32), block=16, precision="f64")
    assert rep["converged"] == K
