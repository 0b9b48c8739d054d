"""GPU parity of the symmetric stage 5 (kl_stage5_symmetric; FP64, BF16x3, BF16): each
kernel value of a pair of point blocks below the diagonal serves both products, and the
partial sums are added in a fixed order.

Same bars as the plain kernels: FP64 relative max-norm error <= 1e-12 against the oracle's
Algorithm 1 (its stage 5 is the dense product Gamma Y, which the symmetric form must
reproduce up to rounding); BF16x3 / BF16 relative Frobenius 5e-5 / 5e-3, every row within
8x that.  Work-item chunk sizes from 1 row tile to the automatic choice
cover items that stop inside, at and across the diagonal block; problem sizes from one
256-point block (no forward partials) to the 24^3 cube (69 blocks).
"""

import ctypes

import numpy as np
import pytest
import torch

import paper_2011_13861_amd as kl
import test_gpu_apply as tga
import test_oracle_multipatch as tom
import workloads
from oracle import cstage5, multipatch, operator

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _apply(G, V):
    return tga._gpu_apply(G, V, "f64")


@pytest.mark.parametrize("chunk", [0, 1, 3])
@pytest.mark.parametrize("name,desc", tga.SMALL, ids=[s[0] for s in tga.SMALL])
def test_symmetric_apply_matches_oracle(name, desc, chunk):
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    assert G.stage5_symmetric(True, chunk) > 0
    V = workloads.random_block(P.N, 7, seed=3)
    tga._check(_apply(G, V), P.apply(V), "f64", name, "sym", chunk)


@pytest.mark.parametrize("precision", ["bf16x3", "bf16"])
@pytest.mark.parametrize("chunk", [0, 3])
@pytest.mark.parametrize("name,desc", tga.SMALL, ids=[s[0] for s in tga.SMALL])
def test_symmetric_low_precision_apply_matches_oracle(name, desc, chunk, precision):
    """The symmetric BF16x3 and BF16 forms at the bars of the plain kernels (relative
    Frobenius 5e-5 / 5e-3 and every row within 8x that)."""
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    assert G.stage5_symmetric(True, chunk, precision=precision) > 0
    V = workloads.random_block(P.N, 7, seed=3)
    tga._check(tga._gpu_apply(G, V, precision), P.apply(V), precision, name, "sym", chunk)


@pytest.mark.parametrize("precision", ["f64", "bf16x3", "bf16"])
@pytest.mark.parametrize("chunk", [0, 1, 2, 5, 7, 1000])
def test_symmetric_stage5_alone_matches_oracle(chunk, precision):
    """Stage 5 alone (no sigma^2 J scaling inside) on 32 and on 3 vectors; 1000 row tiles
    per item puts every column block in one item."""
    desc = workloads.quarter_annulus(20, 2, "exp", (0.3, 0.6))
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    G.stage5_symmetric(True, chunk, precision=precision)
    for nv in (32, 3):
        Y = workloads.random_block(P.Nt, nv, seed=4 + nv)
        y = kl.to_device_block(Y)
        z = kl.new_block(G.Nt, nv)
        G.stage5(y, z, precision)
        torch.cuda.synchronize()
        tga._check(z.cpu().numpy(), P.stage5(Y), precision, "stage5 sym", chunk, nv)


def test_symmetric_and_plain_kernels_agree_and_repeat():
    """The 48x48 cubic annulus (11 blocks): the symmetric and plain FP64 applies agree to
    rounding, and the symmetric one gives the same bits on every call."""
    desc = workloads.config("annulus48")[0]
    G = kl.Problem(desc)
    V = workloads.random_block(G.N, 32, seed=21)
    plain = _apply(G, V)
    G.stage5_symmetric(True)
    a = _apply(G, V)
    b = _apply(G, V)
    assert np.array_equal(a, b)
    assert tga._rel_max(a, plain) <= 1e-13
    G.stage5_symmetric(False)
    assert np.array_equal(_apply(G, V), plain)


def test_full_size_cube24_symmetric_apply():
    """The 24^3 perturbed cube (exp L = 0.5): the symmetric FP64 apply on 32 columns and on
    a ragged 35-column call against the oracle's Algorithm 1 with its C stage 5, and stage 5
    alone on sampled rows recomputed from the kernel definition."""
    from oracle import covariance
    desc = workloads.config("cube24")[0]
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    items = G.stage5_symmetric(True)
    assert items >= G.Nt // 256
    V = workloads.random_block(P.N, 35, seed=13)
    ref = P.apply(V, stage5=lambda Y: cstage5.stage5(P, Y))
    tga._check(_apply(G, V[:, :32]), ref[:, :32], "f64", "cube24 sym 32")
    tga._check(_apply(G, V), ref, "f64", "cube24 sym 35")
    for prec in ("bf16x3", "bf16"):
        G.stage5_symmetric(True, precision=prec)
        tga._check(tga._gpu_apply(G, V[:, :32], prec), ref[:, :32], prec, "cube24 sym 32")
    X, _ = G.points()
    Y = workloads.random_block(G.Nt, 32, seed=6)
    z = kl.new_block(G.Nt, 32)
    G.stage5(kl.to_device_block(Y), z, "f64")
    torch.cuda.synchronize()
    rows = np.concatenate([np.random.default_rng(0).choice(G.Nt, 64, replace=False), [0, G.Nt - 1]])
    tga._check(z.cpu().numpy()[rows], covariance.gamma(desc["cov"], X[rows], X) @ Y, "f64", "cube24 sym rows")


def test_symmetric_eigensolve_matches_oracle():
    """kl_eigs with the symmetric FP64 stage 5 on the 16x16 square: the leading 20
    eigenvalues of the oracle's dense standard-form operator."""
    desc = workloads.config("square16")[0]
    P = operator.Problem(desc)
    lam = np.sort(np.linalg.eigvalsh(P.dense_operator()))[::-1][:20]
    G = kl.Problem(desc)
    G.stage5_symmetric(True)
    w, V, rep = G.eigs(20, precision="f64", tol=1e-10)
    assert rep["status"] == "KL_OK", rep
    assert np.max(np.abs(w - lam) / lam) < 1e-9


def test_symmetric_multipatch_apply_matches_oracle():
    name, descs = tga_mp_case()
    M = multipatch.MultipatchProblem(descs)
    G = kl.Problem(descs)
    G.stage5_symmetric(True, 2)
    V = np.random.default_rng(7).standard_normal((M.N, 37))
    tga._check(_apply(G, V), M.apply(V), "f64", name, "sym")


def tga_mp_case():
    return "l_shape_exp", tom.l_shape("exp", (0.5, 0.3))


def test_symmetric_form_is_skipped_by_noalloc_and_errors():
    desc = workloads.quarter_annulus(11, 2, "sqexp", (0.5, 0.5))
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    G.stage5_symmetric(True)
    V = workloads.random_block(P.N, 9, seed=2)
    x = kl.to_device_block(V)
    out = kl.new_block(G.N, 9)
    st = kl.lib().kl_apply_noalloc(G.handle, kl.PRECISIONS["f64"], 9, ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_int64(G.N), ctypes.c_void_p(out.data_ptr()), ctypes.c_int64(G.N), None)
    assert st == 0, kl.lib().kl_last_error()
    torch.cuda.synchronize()
    tga._check(out.cpu().numpy(), P.apply(V), "f64", "noalloc with sym on")
    for prec, on, chunk in ((0, 2, 0), (0, 1, -1), (1, 1, 0), (7, 1, 0)):
        assert kl.lib().kl_stage5_symmetric(G.handle, prec, on, chunk, None) == -1
    assert G.stage5_symmetric(False) == 0
    # the setting is per precision: FP32 keeps its plain kernel
    G.stage5_symmetric(True)
    G.stage5_symmetric(True, precision="bf16")
    tga._check(tga._gpu_apply(G, V, "f32"), P.apply(V), "f32", "f32 with sym on")
