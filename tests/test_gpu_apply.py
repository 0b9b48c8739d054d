"""GPU parity of the matrix-free apply (Algorithm 1) and of stage 5 against the oracle.

All calls go through the C ABI (kl_setup / kl_apply / kl_stage5).  Tolerances:
FP64 path: relative max-norm error <= 1e-12 (rounding of FP64 kernels and sums);
FP32 path: relative Frobenius error <= 2e-6 (FP32 kernel evaluation, FP32 MFMA
accumulation of up to ~2e4 terms);
BF16x3 path: <= 5e-5 (hi + lo BF16 split keeps about 16 bits of each operand);
BF16 path: <= 5e-3 (8-bit significands of the kernel values and of the block).
Low-precision paths also bound every row: its error is at most 8 times the tolerance of the
RMS row norm of the reference.
"""

import numpy as np
import pytest
import torch

import paper_2011_13861_amd as kl
import test_abi_cpu
import workloads
from oracle import cstage5, operator

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-6, "bf16x3": 5e-5, "bf16": 5e-3}
ROW_FACTOR = 8.0
PRECS = ["f64", "f32", "bf16x3", "bf16"]


def _rel_max(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def _rel_fro(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _row_err(a, b):
    """Largest error of one row (one point or dof, all columns) relative to the RMS row
    norm of the reference: a single bad row cannot hide in the Frobenius norm."""
    rms = np.linalg.norm(b) / np.sqrt(b.shape[0])
    return np.max(np.linalg.norm(np.atleast_2d((a - b).T).T, axis=1)) / rms


def _check(out, ref, precision, *ctx):
    """FP64: relative max-norm error <= 1e-12.  Low precision: relative Frobenius error <=
    TOL and every row within ROW_FACTOR * TOL of the RMS row norm."""
    if precision == "f64":
        err = _rel_max(out, ref)
        print("PARITY", ctx, precision, "max %.3e" % err)
        assert err <= TOL[precision], (ctx, precision, err)
        return
    err, rerr = _rel_fro(out, ref), _row_err(out, ref)
    print("PARITY", ctx, precision, "fro %.3e row %.3e" % (err, rerr))
    assert err <= TOL[precision], (ctx, precision, err)
    assert rerr <= ROW_FACTOR * TOL[precision], (ctx, precision, rerr)


def _gpu_apply(G, V, precision):
    x = kl.to_device_block(V)
    y = kl.new_block(G.N, V.shape[1])
    G.apply(x, y, precision)
    torch.cuda.synchronize()
    return y.cpu().numpy()


SMALL = [
    ("square16", workloads.config("square16")[0]),
    ("annulus_ragged", workloads.quarter_annulus(13, 3, "sqexp", (0.5, 0.8))),
    ("cube", workloads.sine_cube(6, 2, "exp", 0.5)),
    ("interp_ne_trial", {"dim": 2, "degree": [2, 3], "nelem": [9, 5], "interp_degree": [3, 1],
                         "interp_nelem": [12, 11], "map": {"kind": "annulus_polar", "r0": 1.0, "r1": 2.0},
                         "cov": {"kind": "exp", "sigma2": 1.3, "corr_len": [0.4, 0.9]}}),
    ("interp_c0", {"dim": 2, "degree": [3, 2], "nelem": [10, 7], "interp_degree": [2, 3],
                   "interp_nelem": [9, 6], "interp_mult": [2, 3],
                   "map": {"kind": "annulus_nurbs", "r0": 1.0, "r1": 2.0},
                   "cov": {"kind": "exp", "sigma2": 1.0, "corr_len": [0.5, 0.5]}}),
    ("line", {"dim": 1, "degree": [3], "nelem": [120], "map": {"kind": "box", "lo": [0.0], "hi": [2.0]},
              "cov": {"kind": "sqexp", "sigma2": 1.0, "corr_len": [0.2]}}),
    ("exp_l1", {"dim": 2, "degree": [2, 2], "nelem": [10, 7], "map": {"kind": "identity"},
                "cov": {"kind": "exp_l1", "sigma2": 1.0, "corr_len": [0.5, 0.3]}}),
    ("const", {"dim": 2, "degree": [2, 2], "nelem": [6, 6], "map": {"kind": "box", "lo": [0, 0], "hi": [2, 1]},
               "cov": {"kind": "const", "sigma2": 0.7, "corr_len": [1.0, 1.0]}}),
    ("lin", {"dim": 3, "degree": [1, 2, 1], "nelem": [4, 3, 5], "map": {"kind": "identity"},
             "cov": {"kind": "lin", "sigma2": 1.0, "corr_len": [1.0] * 3}}),
    ("nonuniform_knots", test_abi_cpu.NONUNIFORM),
    ("nurbs_cylinder_shell", test_abi_cpu.CYLINDER),
    # discontinuous spaces: two patches meeting at a kink of the map, and C^-1 interpolation
    # spaces in 3D (coincident Greville points, coincident kernel arguments)
    ("kinked_two_patch", test_abi_cpu.KINKED_2D),
    ("cube_interp_cminus1", test_abi_cpu.CASES[-1]),
]


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("name,desc", SMALL, ids=[s[0] for s in SMALL])
def test_apply_matches_oracle(name, desc, precision):
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    V = workloads.random_block(P.N, 7, seed=3)
    ref = P.apply(V)
    out = _gpu_apply(G, V, precision)
    _check(out, ref, precision, name)


@pytest.mark.parametrize("precision", PRECS)
def test_stage5_alone_matches_oracle(precision):
    desc = workloads.quarter_annulus(20, 2, "exp", (0.3, 0.6))
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    Y = workloads.random_block(P.Nt, 32, seed=4)
    ref = P.stage5(Y)
    y = kl.to_device_block(Y)
    z = kl.new_block(G.Nt, 32)
    G.stage5(y, z, precision)
    torch.cuda.synchronize()
    out = z.cpu().numpy()
    _check(out, ref, precision, "stage5")


@pytest.mark.parametrize("nvec", [1, 31, 32, 33, 70])
def test_block_widths_and_strides(nvec):
    desc = workloads.quarter_annulus(11, 2, "sqexp", (0.5, 0.5))
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    V = workloads.random_block(P.N, nvec, seed=nvec)
    ref = P.apply(V)
    # strided input / output: leading dimension N + 5
    xs = torch.zeros((nvec, P.N + 5), dtype=torch.float64, device="cuda")
    xs[:, :P.N] = torch.from_numpy(np.ascontiguousarray(V.T)).cuda()
    ys = torch.full((nvec, P.N + 5), 7.0, dtype=torch.float64, device="cuda")
    x = xs.T[:P.N]
    y = ys.T[:P.N]
    G.apply(x, y, "f64")
    torch.cuda.synchronize()
    assert _rel_max(y.cpu().numpy(), ref) <= 1e-12
    assert torch.all(ys[:, P.N:] == 7.0)          # padding of the output untouched


def test_full_size_annulus64_apply():
    """The 64x64 cubic quarter annulus (sqexp L = 0.5) at full size, 32 vectors."""
    desc = workloads.config("annulus64")[0]
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    V = workloads.random_block(P.N, 32, seed=5)
    ref = P.apply(V, stage5=lambda Y: cstage5.stage5(P, Y))
    for prec in PRECS:
        out = _gpu_apply(G, V, prec)
        _check(out, ref, prec, "full")


def test_full_size_annulus48_apply():
    """The 48x48 cubic quarter annulus (sqexp L = 0.5, the warm-start workload) at
    full size, 32 vectors, every precision."""
    desc = workloads.config("annulus48")[0]
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    V = workloads.random_block(P.N, 32, seed=6)
    ref = P.apply(V)
    for prec in PRECS:
        out = _gpu_apply(G, V, prec)
        _check(out, ref, prec, "full")


# Correlation lengths far below the point spacing (all but the nearest kernel entries
# underflow: exponents down to about -10^5) and far above the domain (entries within 1e-4
# of 1): both ends of the argument range of the FP64 exponential of the stage-5 kernels.
EXTREME = [
    ("tiny_ell_sqexp", {"dim": 2, "degree": [2, 2], "nelem": [20, 14],
                        "map": {"kind": "annulus_polar", "r0": 1.0, "r1": 2.0},
                        "cov": {"kind": "sqexp", "sigma2": 1.0, "corr_len": [0.01, 0.01]}}),
    ("tiny_ell_exp3d", {"dim": 3, "degree": [1, 1, 1], "nelem": [8, 7, 6], "map": {"kind": "identity"},
                        "cov": {"kind": "exp", "sigma2": 2.0, "corr_len": [0.002, 0.003, 0.002]}}),
    ("huge_ell_exp", {"dim": 2, "degree": [2, 3], "nelem": [11, 9], "map": {"kind": "identity"},
                      "cov": {"kind": "exp", "sigma2": 0.5, "corr_len": [300.0, 150.0]}}),
]


@pytest.mark.parametrize("name,desc", EXTREME, ids=[e[0] for e in EXTREME])
def test_extreme_correlation_lengths(name, desc):
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    V = workloads.random_block(P.N, 32, seed=8)
    ref = P.apply(V)
    for prec in PRECS:
        out = _gpu_apply(G, V, prec)
        assert np.all(np.isfinite(out)), (name, prec)
        _check(out, ref, prec, name)


def test_full_size_cube24_apply():
    """The 24^3 perturbed cube (exp L = 0.5) at full size: the whole apply (fused
    first two directions, third direction, stage 5, backward) on the 32 columns the
    eigensolver applies at a time, and on a ragged 35-column call, against the oracle's
    Algorithm 1 with its C stage 5."""
    desc = workloads.config("cube24")[0]
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    assert G.apply_config(True)
    V = workloads.random_block(P.N, 35, seed=13)
    ref = P.apply(V, stage5=lambda Y: cstage5.stage5(P, Y))
    for prec in PRECS:
        out = _gpu_apply(G, V[:, :32], prec)
        _check(out, ref[:, :32], prec, "cube24 32")
    _check(_gpu_apply(G, V, "f64"), ref, "f64", "cube24 35")


def test_full_size_cube24_stage5_sampled_rows():
    """The 24^3 perturbed cube (exp L = 0.5): stage 5 on 32 vectors, sampled rows
    recomputed one by one by the oracle's kernel definition."""
    from oracle import covariance
    desc = workloads.config("cube24")[0]
    G = kl.Problem(desc)
    X, _ = G.points()
    Y = workloads.random_block(G.Nt, 32, seed=6)
    y = kl.to_device_block(Y)
    for prec in PRECS:
        z = kl.new_block(G.Nt, 32)
        G.stage5(y, z, prec)
        torch.cuda.synchronize()
        out = z.cpu().numpy()
        rows = np.random.default_rng(0).choice(G.Nt, 64, replace=False)
        rows = np.concatenate([rows, [0, G.Nt - 1]])
        ref = covariance.gamma(desc["cov"], X[rows], X) @ Y
        _check(out[rows], ref, prec, "cube24 stage5 rows")


def test_apply_is_symmetric_on_gpu():
    desc = workloads.config("cube24")[0]
    G = kl.Problem(desc)
    rng = np.random.default_rng(7)
    U = rng.standard_normal((G.N, 2))
    for prec, tol in (("f64", 1e-13), ("f32", 1e-6)):
        AU = _gpu_apply(G, U, prec)
        lhs = U[:, 0] @ AU[:, 1]
        rhs = AU[:, 0] @ U[:, 1]
        assert abs(lhs - rhs) <= tol * np.linalg.norm(AU[:, 0]) * np.linalg.norm(U[:, 1]), prec


def test_apply_errors():
    desc = workloads.unit_square(4, 2, "exp", 1.0)
    G = kl.Problem(desc)
    x = kl.new_block(G.N, 2)
    with pytest.raises(kl.KLError):
        G.apply(x, x, "f64")                        # aliasing input and output
    with pytest.raises(KeyError):
        G.apply(x, kl.new_block(G.N, 2), "f16")
    import ctypes
    st = kl.lib().kl_apply(G.handle, 9, 2, ctypes.c_void_p(x.data_ptr()), G.N,
                           ctypes.c_void_p(kl.new_block(G.N, 2).data_ptr()), G.N, None)
    assert st == -1
    # nvec = 0 is a no-op
    assert kl.lib().kl_apply(G.handle, 0, 0, None, G.N, None, G.N, None) == 0



def test_long_direction():
    """A direction with several hundred basis functions (several MFMA chunks of the
    contraction index) against the oracle."""
    desc = {"dim": 1, "degree": [2], "nelem": [400], "map": {"kind": "identity"},
            "cov": {"kind": "exp", "sigma2": 1.0, "corr_len": [0.3]}}
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    V = workloads.random_block(P.N, 3, seed=9)
    assert _rel_max(_gpu_apply(G, V, "f64"), P.apply(V)) <= 1e-12


@pytest.mark.parametrize("prec,rb,ns", [("f32", 1, 0), ("f32", 2, 5), ("f32", 4, 0), ("f32", 8, 0), ("f32", 8, 9),
                                        ("bf16x3", 1, 0), ("bf16x3", 4, 3), ("f64", 0, 7),
                                        # split counts that are multiples of 8: splits placed per XCD
                                        ("f64", 0, 8), ("f64", 0, 16), ("f32", 2, 8), ("f32", 8, 16),
                                        ("bf16x3", 2, 8), ("bf16", 1, 16)])
def test_stage5_tile_settings(prec, rb, ns):
    """Every stage-5 tile setting (32-row blocks per wave, waves per workgroup, l-splits)
    against the oracle on a problem with several row tiles and splits."""
    desc = workloads.quarter_annulus(20, 2, "sqexp", (0.4, 0.7))
    P = operator.Problem(desc)
    G = kl.Problem(desc)
    G.stage5_config(prec, rb=rb, nsplit=ns)
    V = workloads.random_block(P.N, 11, seed=12)
    out = _gpu_apply(G, V, prec)
    ref = P.apply(V)
    _check(out, ref, prec, "tiles", rb, ns)


FUSE_CASES = [s for s in SMALL if s[1]["dim"] >= 2] + [
    # 73 x 19 slab: 8 waves, two leftover tiles of 16 in each phase cut into quarters
    ("wide_2d", {"dim": 2, "degree": [3, 2], "nelem": [70, 17], "map": {"kind": "identity"},
                 "cov": {"kind": "exp", "sigma2": 1.0, "corr_len": [0.3, 0.6]}}),
    # 40 x 40: three leftover tiles per phase (12 quarters, two on some waves)
    ("quarters_r3", {"dim": 2, "degree": [2, 2], "nelem": [38, 38], "map": {"kind": "identity"},
                     "cov": {"kind": "sqexp", "sigma2": 1.0, "corr_len": [0.4, 0.4]}}),
    # 77 x 80: the longest contraction (20 MFMA steps), four whole tiles and one in
    # quarters, slab staged in more than one pass with and without split partials
    ("big_slab", {"dim": 2, "degree": [3, 3], "nelem": [74, 77], "map": {"kind": "annulus_polar", "r0": 1.0, "r1": 2.0},
                  "cov": {"kind": "exp", "sigma2": 1.0, "corr_len": [0.5, 0.5]}}),
]
_FUSE_REF = {}


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("name,desc", FUSE_CASES, ids=[s[0] for s in FUSE_CASES])
def test_fused_directions_match_oracle_and_per_direction_form(name, desc, precision):
    """The fused pair of directions (one launch per side, the backward one adding the
    stage-5 split partials) against the oracle and against the per-direction launches,
    with the split count forced to 1 (stage 5 writes the scaled output), 3 and 9 (more
    partials than the backward launch loads in one group)."""
    G = kl.Problem(desc)
    assert G.apply_config(True), name
    if name not in _FUSE_REF:
        P = operator.Problem(desc)
        V = workloads.random_block(P.N, 33, seed=21)   # a full 32-column block and a ragged one
        _FUSE_REF[name] = (V, P.apply(V))
    V, ref = _FUSE_REF[name]
    tol = TOL[precision]
    for ns in (1, 3, 8, 9):
        G.stage5_config(precision, nsplit=ns)
        G.apply_config(True)
        fused = _gpu_apply(G, V, precision)
        G.apply_config(False)
        per_dir = _gpu_apply(G, V, precision)
        for out in (fused, per_dir):
            _check(out, ref, precision, name, ns)
        assert _rel_max(fused, per_dir) <= (1e-12 if precision == "f64" else 10 * tol), (name, precision, ns)
    G.apply_config(True)
    G.stage5_config(precision, nsplit=0)


def test_fused_directions_fallback_for_large_slabs():
    """A 2-D problem whose slab does not fit the fused kernel's LDS keeps the
    per-direction form (and stays correct)."""
    desc = {"dim": 2, "degree": [2, 2], "nelem": [120, 100], "map": {"kind": "identity"},
            "cov": {"kind": "sqexp", "sigma2": 1.0, "corr_len": [0.3, 0.3]}}
    G = kl.Problem(desc)
    assert not G.apply_config(True)
    P = operator.Problem(desc)
    V = workloads.random_block(P.N, 2, seed=22)
    ref = P.apply(V, stage5=lambda Y: cstage5.stage5(P, Y))
    assert _rel_max(_gpu_apply(G, V, "f64"), ref) <= 1e-12


ULP_CASES = [
    ("exp3d", workloads.sine_cube(6, 2, "exp", 0.5)),
    ("exp2d", workloads.quarter_annulus(14, 2, "exp", (0.5, 0.3))),
    ("sqexp2d", workloads.quarter_annulus(14, 2, "sqexp", (0.5, 0.5))),
    ("expl1", {"dim": 2, "degree": [2, 2], "nelem": [12, 12], "map": {"kind": "identity"},
               "cov": {"kind": "exp_l1", "sigma2": 1.0, "corr_len": [0.3, 0.6]}}),
    ("exp1d_short", {"dim": 1, "degree": [2], "nelem": [300], "map": {"kind": "identity"},
                     "cov": {"kind": "exp", "sigma2": 1.0, "corr_len": [0.05]}}),
]


@pytest.mark.parametrize("name,desc", ULP_CASES, ids=[c[0] for c in ULP_CASES])
def test_fp64_kernel_values_within_a_few_ulp(name, desc):
    """FP64 stage 5 applied to unit vectors returns single kernel values Gamma(x_k, x_j)
    (every other term of the contraction is an exact zero).  Against long-double values
    from the same points: the error stays within a few ulp plus the rounding of the scaled
    coordinates (absolute ~1e-16 |x| / ell in the exponent)."""
    G = kl.Problem(desc)
    X, _ = G.points()
    rng = np.random.default_rng(17)
    cols = rng.choice(G.Nt, 32, replace=False)
    Y = np.zeros((G.Nt, 32))
    Y[cols, np.arange(32)] = 1.0
    y = kl.to_device_block(Y)
    z = kl.new_block(G.Nt, 32)
    G.stage5(y, z, "f64")
    torch.cuda.synchronize()
    out = z.cpu().numpy()
    cov = desc["cov"]
    ell = np.asarray(cov["corr_len"], dtype=np.longdouble)[:G.d]
    Xl = X.astype(np.longdouble)
    diff = (Xl[:, None, :] - Xl[None, cols, :]) / ell
    if cov["kind"] == "exp":
        ref = np.exp(-np.sqrt(np.sum(diff * diff, axis=2)))
    elif cov["kind"] == "sqexp":
        ref = np.exp(-np.sum(diff * diff, axis=2))
    else:
        ref = np.exp(-np.sum(np.abs(diff), axis=2))
    mask = ref > 1e-12
    rel = np.abs(out.astype(np.longdouble) - ref)[mask] / ref[mask]
    scale = float(np.max(np.abs(X) / np.asarray(cov["corr_len"])[:G.d])) * 1.4427
    if cov["kind"] == "sqexp":
        scale = scale * scale
    bar = 2.2e-16 * (4.0 + 2.0 * scale)
    print("ULP", name, "max rel %.3e bar %.3e" % (float(rel.max()), bar))
    assert float(rel.max()) <= bar, (name, float(rel.max()), bar)
