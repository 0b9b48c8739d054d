"""GPU parity of the batched path (kl_setup_batch / kl_apply_batch / kl_eigs_batch): one
graph replay applies every problem of a batch of uneven sizes, kernels and degrees.

References: the oracle's literal Algorithm 1 per problem (small batch; three problems of
the 64-problem batch with the C stage 5), the single-problem apply (all 64), and the
oracle's dense eigensolver (small batch).  Tolerances as for the single-problem apply
(FP64 1e-12 max-norm, FP32 2e-6 Frobenius) and eigenvalues per the parity reading
|lambda - lambda_ref| <= 1e-6 lambda_ref + 1e-12 lambda_1.
"""

import numpy as np
import pytest
import torch

import paper_2011_13861_amd as kl
import workloads
from oracle import cstage5, eigs as oeigs, operator

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-6}

SMALL = [
    workloads.unit_square(5, 2, "exp", 0.7),
    workloads.unit_square(30, 2, "sqexp", 0.3),            # Ntilde = 1024: splits at lchunk 512
    workloads.quarter_annulus(7, 2, "exp", (0.4, 0.9)),
    {"dim": 2, "degree": [4, 2], "nelem": [11, 5], "map": {"kind": "identity"},
     "cov": {"kind": "exp_l1", "sigma2": 1.0, "corr_len": [0.5, 0.3]}},
    workloads.unit_square(13, 4, "sqexp", 1.5),
    {"dim": 2, "degree": [2, 2], "nelem": [6, 6], "map": {"kind": "box", "lo": [0, 0], "hi": [2, 1]},
     "cov": {"kind": "exp", "sigma2": 0.7, "corr_len": [0.8, 0.8]}},
]


def _err(out, ref, prec):
    if prec == "f64":
        return np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    return np.linalg.norm(out - ref) / np.linalg.norm(ref)


def _fill(B, nvec, seed):
    x = B.arena(nvec)
    host = []
    for i in range(B.n):
        V = workloads.random_block(B.N[i], nvec, seed=seed + i)
        B.block(x, i, nvec).copy_(torch.from_numpy(V))
        host.append(V)
    return x, host


@pytest.fixture(scope="module")
def small():
    return kl.Batch(SMALL), [operator.Problem(d) for d in SMALL]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_apply_matches_oracle(small, prec):
    B, P = small
    x, host = _fill(B, 7, 10)
    y = B.arena(7)
    B.apply(x, y, 7, prec)
    torch.cuda.synchronize()
    for i in range(B.n):
        out = B.block(y, i, 7).cpu().numpy()
        assert _err(out, P[i].apply(host[i]), prec) <= TOL[prec], (i, prec)


def test_batch_widths_active_mask_and_replays(small):
    """Replays of the same graph with other column counts and active sets: inactive
    problems keep their output, active ones match the oracle."""
    B, P = small
    for nvec, active in ((1, [1, 0, 1, 1, 0, 1]), (32, [0, 1, 1, 0, 1, 1]), (7, None)):
        x, host = _fill(B, nvec, 20 + nvec)
        y = torch.full((B.Ntot * nvec,), 5.0, dtype=torch.float64, device="cuda")
        B.apply(x, y, nvec, "f64", active=active)
        torch.cuda.synchronize()
        for i in range(B.n):
            out = B.block(y, i, nvec).cpu().numpy()
            if active is not None and not active[i]:
                assert np.all(out == 5.0), (nvec, i)
            else:
                assert _err(out, P[i].apply(host[i]), "f64") <= 1e-12, (nvec, i)


@pytest.mark.parametrize("prec,rb,lchunk", [("f32", 4, 512), ("f32", 2, 512), ("f64", 0, 512), ("f32", 2, 0)])
def test_batch_tile_configs(small, prec, rb, lchunk):
    B, P = small
    grid, items = B.config(prec, rb=rb, lchunk=lchunk)
    assert grid >= 256 and items >= B.n
    x, host = _fill(B, 5, 40)
    y = B.arena(5)
    B.apply(x, y, 5, prec)
    torch.cuda.synchronize()
    for i in range(B.n):
        assert _err(B.block(y, i, 5).cpu().numpy(), P[i].apply(host[i]), prec) <= TOL[prec], (i, prec, rb, lchunk)
    B.config(prec, rb=2, lchunk=0)


def test_batch_eigs_small_matches_dense_oracle(small):
    B, P = small
    k = 6
    ev, V, reps = B.eigs(k, precision="f64", block=8, tol=1e-10)
    for i in range(B.n):
        assert reps[i]["converged"] == k, (i, reps[i])
        w, _ = oeigs.dense_eigs(P[i], k)
        lam1 = w[0]
        assert np.all(np.abs(ev[i] - w) <= 1e-6 * np.abs(w) + 1e-12 * lam1), (i, ev[i], w)
        # eigenvectors: unit norm, residual under the oracle operator
        X = B.block(V, i, k).cpu().numpy()
        R = P[i].apply(X) - X * ev[i]
        assert np.all(np.linalg.norm(R, axis=0) <= 1e-8 * np.abs(ev[i]) + 1e-12 * lam1), i


@pytest.fixture(scope="module")
def batch64():
    descs = workloads.batch_problems(1127)
    return descs, kl.Batch(descs)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch64_batch_apply_matches_single_problem_path(batch64, prec):
    """All 64 problems of the uneven batch against the single-problem apply, and three of
    them (the largest, the smallest and one squared-exponential) against the oracle."""
    descs, B = batch64
    nvec = 32
    x, host = _fill(B, nvec, 100)
    y = B.arena(nvec)
    B.apply(x, y, nvec, prec)
    torch.cuda.synchronize()
    outs = [B.block(y, i, nvec).cpu().numpy() for i in range(B.n)]
    for i, d in enumerate(descs):
        G = kl.Problem(d)
        ys = kl.new_block(G.N, nvec)
        G.apply(B.block(x, i, nvec), ys, prec)
        torch.cuda.synchronize()
        assert _err(outs[i], ys.cpu().numpy(), prec) <= TOL[prec], (i, prec)
    if prec == "f64":
        picks = [int(np.argmax(B.N)), int(np.argmin(B.N)),
                 next(i for i, d in enumerate(descs) if d["cov"]["kind"] == "sqexp")]
        for i in picks:
            P = operator.Problem(descs[i])
            ref = P.apply(host[i], stage5=lambda Y: cstage5.stage5(P, Y))
            assert _err(outs[i], ref, "f64") <= 1e-12, i


def test_batch64_batch_eigs_fp32_refined(batch64):
    """The 64-problem batch: 20 eigenpairs of each of the 64 problems, FP32 applies with FP64
    refinement, against per-problem FP64 solves."""
    descs, B = batch64
    k = 20
    ev, V, reps = B.eigs(k, precision="f32", block=32, tol=1e-6)
    assert all(r["converged"] == k for r in reps)
    for i in (0, 17, 40, 63):
        G = kl.Problem(descs[i])
        w, _, rep = G.eigs(k, precision="f64", block=32, tol=1e-6)
        assert np.all(np.abs(ev[i] - w) <= 1e-6 * np.abs(w) + 1e-12 * w[0]), (i, ev[i], w)


def test_batch64_batch_eigs_match_oracle(batch64):
    """The 64-problem batch (FP32 applies with FP64 refinement, tol 1e-10), sampled problems
    against the oracle's eigenpairs: the smallest (sqexp), an exponential with L near 1.8, a
    fast-decaying squared exponential (L near 1.5, eigenvalues down to the 1e-12 floor), a
    short exponential (L near 0.11), all by dense LAPACK, and the largest problem (8,624
    dofs, sqexp) by ARPACK on the literal Algorithm 1."""
    from test_gpu_eigs import check_pairs
    descs, B = batch64
    k = 20
    ev, V, reps = B.eigs(k, precision="f32", block=32, tol=1e-10)
    assert all(r["converged"] == k for r in reps), [r["converged"] for r in reps]
    for i in (32, 10, 20, 4, 62):
        P = operator.Problem(descs[i])
        if P.N <= 3000:
            w_ref, V_ref = oeigs.dense_eigs(P, k + 8)
        else:
            w_ref, V_ref = oeigs.iterative_eigs(P, k + 8, tol=1e-13, stage5=lambda Y: cstage5.stage5(P, Y))
        X = B.block(V, i, k).cpu().numpy()
        n = check_pairs(ev[i], X, w_ref, V_ref, k)
        print("batch problem", i, "N", P.N, "vectors compared", n)
        assert n >= 4, (i, n)
