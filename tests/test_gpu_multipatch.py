"""GPU parity of multipatch problems (kl_setup_patches, Sec. 3.6: non-conforming patches
with their own spaces and maps, coupled by stage 5 over all points) against the oracle's
MultipatchProblem, which is pinned by closed forms in test_oracle_multipatch.py.

Bars as for single problems: FP64 relative max error 1e-12; FP32 / BF16x3 / BF16 relative
Frobenius 2e-6 / 5e-5 / 5e-3 and every row within 8x that; eigenpairs at the solver's
criterion; the truncated expansion at 1e-12.
"""

import ctypes

import numpy as np
import pytest
import torch

import paper_2011_13861_amd as kl
import test_abi_cpu
import test_oracle_multipatch as tom
from oracle import eigs as oeigs
from oracle import kle, multipatch

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-6, "bf16x3": 5e-5, "bf16": 5e-3}
PRECS = ["f64", "f32", "bf16x3", "bf16"]


def _annulus_patch(kind, ell):
    return {"dim": 2, "degree": [3, 2], "nelem": [5, 7], "interp_degree": [2, 2], "interp_nelem": [6, 8],
            "interp_mult": [1, 2], "map": {"kind": "annulus_nurbs", "r0": 3.0, "r1": 4.0},
            "cov": {"kind": kind, "sigma2": 1.0, "corr_len": list(ell)}}


def _kinked(kind, ell):
    """The kinked two-patch square moved to [5, 6] x [0, 1] (control points shifted)."""
    g = test_abi_cpu.kinked_square()
    g = dict(g, ctrl=np.asarray(g["ctrl"]) + np.array([5.0, 0.0]))
    return dict(test_abi_cpu.KINKED_2D, map=g, cov={"kind": kind, "sigma2": 1.0, "corr_len": list(ell)})


def _cube(lo, hi, p, ne, kind="exp", ell=0.5):
    return {"dim": 3, "degree": list(p), "nelem": list(ne), "map": {"kind": "box", "lo": list(lo), "hi": list(hi)},
            "cov": {"kind": kind, "sigma2": 1.0, "corr_len": [ell] * 3}}


CASES = [
    ("l_shape_exp", tom.l_shape("exp", (0.5, 0.3))),
    # an L-shape, an annulus patch away from it and a kinked two-patch square (C^-1 inside
    # a patch as well as between patches), squared exponential
    ("mixed_2d", tom.l_shape("sqexp", (0.6, 0.4)) + [_annulus_patch("sqexp", (0.6, 0.4)),
                                                      _kinked("sqexp", (0.6, 0.4))]),
    ("two_cubes_3d", [_cube((0, 0, 0), (1, 1, 1), (2, 2, 1), (4, 3, 5)),
                      _cube((1, 0, 0), (2, 1, 0.5), (1, 2, 2), (3, 5, 2))]),
]


def _rel_max(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _check(out, ref, precision, name):
    if precision == "f64":
        err = _rel_max(out, ref)
        print("PARITY", name, precision, "max %.3e" % err)
        assert err <= TOL[precision], (name, err)
        return
    err = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    rms = np.linalg.norm(ref) / np.sqrt(ref.shape[0])
    row = float(np.max(np.linalg.norm(out - ref, axis=1)) / rms)
    print("PARITY", name, precision, "fro %.3e row %.3e" % (err, row))
    assert err <= TOL[precision] and row <= 8 * TOL[precision], (name, precision, err, row)


def _apply(G, V, precision):
    x = kl.to_device_block(V)
    y = kl.new_block(G.N, V.shape[1])
    G.apply(x, y, precision)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("name,descs", CASES, ids=[c[0] for c in CASES])
def test_multipatch_apply_matches_oracle(name, descs, precision):
    M = multipatch.MultipatchProblem(descs)
    G = kl.Problem(descs)
    assert G.N == M.N and G.Nt == M.Nt
    assert G.patches() == [(P.N, P.Nt, int(M.noff[i]), int(M.toff[i])) for i, P in enumerate(M.patches)]
    X, J = G.points()
    assert np.max(np.abs(X - M.X)) < 1e-13 * np.abs(M.X).max() and np.max(np.abs(J - M.J)) < 1e-13 * M.J.max()
    V = np.random.default_rng(7).standard_normal((M.N, 37))      # a full block and a ragged one
    _check(_apply(G, V, precision), M.apply(V), precision, name)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_multipatch_fused_and_per_direction_forms_agree(precision):
    name, descs = CASES[1]
    M = multipatch.MultipatchProblem(descs)
    G = kl.Problem(descs)
    V = np.random.default_rng(8).standard_normal((M.N, 9))
    ref = M.apply(V)
    for fuse in (True, False):
        G.apply_config(fuse)
        for ns in (1, 3, 8):
            G.stage5_config(precision, nsplit=ns)
            _check(_apply(G, V, precision), ref, precision, "%s fuse %d ns %d" % (name, fuse, ns))


@pytest.mark.parametrize("precision", ["f64", "bf16x3"])
def test_l_shape_linear_kernel_spectrum_from_the_solver(precision):
    """1 + x . x' on the L-shape: the eigenvalues of the hand-computed Gram matrix of
    (1, x_1, x_2), through the GPU solve (BF16x3 with the FP64 refinement too)."""
    G = kl.Problem(tom.l_shape())
    w, V, rep = G.eigs(3, precision=precision, tol=1e-10)
    assert rep["status"] == "KL_OK" and rep["converged"] == 3, rep
    ref = np.sort(np.linalg.eigvalsh(tom.G_L))[::-1]
    assert np.max(np.abs(w - ref) / ref) < 1e-10, w - ref


def test_multipatch_eigenpairs_and_coefficients_match_oracle():
    name, descs = CASES[0]
    M = multipatch.MultipatchProblem(descs)
    A = M.dense_operator()
    lam, U = np.linalg.eigh(A)
    lam, U = lam[::-1], U[:, ::-1]
    k = 10
    G = kl.Problem(descs)
    w, V, rep = G.eigs(k, precision="f64", tol=1e-10)
    assert rep["status"] == "KL_OK", rep
    assert np.all(np.abs(w - lam[:k]) <= 1e-9 * lam[:k])
    Vh = V.cpu().numpy()
    r = np.linalg.norm(M.apply(Vh) - Vh * w[None, :], axis=0)
    assert np.all(r <= 1e-10 * w + 1e-12 * w[0] + 1e-14)
    # B-spline coefficients v = L^{-T} v' patch by patch
    wc, Vc, _ = G.eigs(k, precision="f64", tol=1e-10, coeffs=True)
    ref = M.to_coefficients(Vh)
    Vc = Vc.cpu().numpy()
    for i in range(k):
        s = np.sign(Vc[:, i] @ ref[:, i])
        assert np.max(np.abs(Vc[:, i] - s * ref[:, i])) <= 1e-7 * np.max(np.abs(ref[:, i])), i


def test_multipatch_kle_field_matches_oracle():
    name, descs = CASES[1]
    M = multipatch.MultipatchProblem(descs)
    lam, V = oeigs.dense_eigs(M, 40)
    lam = np.maximum(lam, 0.0)
    Phi = np.concatenate([kle.eigenfunctions(P, V[M.noff[i]:M.noff[i + 1]]) for i, P in enumerate(M.patches)])
    xi = np.random.default_rng(9).standard_normal((40, 19))
    F_ref = Phi @ (np.sqrt(lam)[:, None] * xi)
    var_ref = (Phi ** 2) @ lam
    G = kl.Problem(descs)
    F, var = G.kle_field(lam, kl.to_device_block(V), kl.to_device_block(xi))
    torch.cuda.synchronize()
    assert _rel_max(F.cpu().numpy(), F_ref) < 1e-12
    assert _rel_max(var.cpu().numpy(), var_ref) < 1e-12


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_multipatch_noalloc_matches_apply(precision):
    name, descs = CASES[2]
    G = kl.Problem(descs)
    x = kl.to_device_block(np.random.default_rng(10).standard_normal((G.N, 33)))
    ref = kl.new_block(G.N, 33)
    G.apply(x, ref, precision)
    out = kl.new_block(G.N, 33)
    st = kl.lib().kl_apply_noalloc(G.handle, kl.PRECISIONS[precision], 33, ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_int64(G.N), ctypes.c_void_p(out.data_ptr()), ctypes.c_int64(G.N), None)
    assert st == 0, kl.lib().kl_last_error()
    torch.cuda.synchronize()
    a, b = out.cpu().numpy(), ref.cpu().numpy()
    err = _rel_max(a, b) if precision == "f64" else float(np.linalg.norm(a - b) / np.linalg.norm(b))
    assert err <= TOL[precision], err


def test_get_factor_rejects_several_patches():
    G = kl.Problem(tom.l_shape())
    out = np.zeros(1000)
    assert kl.lib().kl_get_factor(G.handle, 0, ctypes.c_void_p(out.ctypes.data)) == -1
