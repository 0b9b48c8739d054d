"""Seeded synthetic workloads shared by the tests, the benchmark and the smoke check.

This module holds problem descriptions (plain dicts) and seeded random inputs only;
it contains none of the method's arithmetic.  Both the HIP path (through its binding)
and the CPU oracle consume the same dicts.

Description dict:
  dim            spatial dimension d (1..3)
  degree, nelem  trial space: degree p_k and element count per direction (open uniform
                 knots with C^{p-1} continuity, n_k = nelem_k + p_k)
  interp_degree, interp_nelem   optional interpolation space (default: trial space)
  interp_mult    optional multiplicity of the interpolation space's interior breakpoints
                 (default 1; interp_mult = interp_degree gives a C^0 space)
  map            {"kind": identity | box | annulus_nurbs | annulus_polar | sine_cube, ...}
  cov            {"kind": exp | sqexp | exp_l1 | const | lin, "sigma2": s2, "corr_len": [...]}

The named configurations are synthetic stand-ins for the paper's 2D and 3D workloads
(its 3D NURBS geometries are not reproducible: their control points are not printed).
"""

import math

import numpy as np


def unit_square(nelem=16, p=2, kind="exp", ell=1.0, d=2):
    return {"dim": d, "degree": [p] * d, "nelem": [nelem] * d,
            "map": {"kind": "identity"},
            "cov": {"kind": kind, "sigma2": 1.0, "corr_len": [ell] * d}}


def quarter_annulus(nelem=64, p=3, kind="sqexp", ell=(0.5, 0.5)):
    return {"dim": 2, "degree": [p, p], "nelem": [nelem, nelem],
            "map": {"kind": "annulus_nurbs", "r0": 1.0, "r1": 2.0},
            "cov": {"kind": kind, "sigma2": 1.0, "corr_len": list(ell)}}


def sine_cube(nelem=24, p=2, kind="exp", ell=0.5):
    return {"dim": 3, "degree": [p] * 3, "nelem": [nelem] * 3,
            "map": {"kind": "sine_cube", "eps": 0.05, "amp": [1.0, 0.5, 0.25]},
            "cov": {"kind": kind, "sigma2": 1.0, "corr_len": [ell] * 3}}


# The named workloads: (description, number of eigenpairs, block size)
def config(name):
    if name == "square16":      # unit square 16x16, quadratic, exponential L = 1, 20 pairs
        return unit_square(16, 2, "exp", 1.0), 20, 32
    if name == "annulus64":      # quarter annulus 64x64, cubic, squared exponential L = 0.5, 40 pairs
        return quarter_annulus(64, 3, "sqexp", (0.5, 0.5)), 40, 32
    if name == "cube24":      # perturbed cube 24^3, quadratic, exponential L = 0.5, 50 pairs
        return sine_cube(24, 2, "exp", 0.5), 50, 32
    if name == "annulus48":      # quarter annulus 48x48, cubic (MLP warm-start problem family)
        return quarter_annulus(48, 3, "sqexp", (0.5, 0.5)), 16, 16
    raise KeyError(name)


def batch_problems(seed=1127, count=64):
    """64 uneven 2D unit-square problems: nelem_x, nelem_y ~ U{16..96}, p ~ U{2,3,4},
    kind exp or sqexp with probability 1/2 each, ell ~ logU[0.1, 2]; drawn in this order."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        nx = int(rng.integers(16, 97))
        ny = int(rng.integers(16, 97))
        p = int(rng.integers(2, 5))
        kind = "exp" if rng.random() < 0.5 else "sqexp"
        ell = float(math.exp(rng.uniform(math.log(0.1), math.log(2.0))))
        out.append({"dim": 2, "degree": [p, p], "nelem": [nx, ny], "map": {"kind": "identity"},
                    "cov": {"kind": kind, "sigma2": 1.0, "corr_len": [ell, ell]}})
    return out


def mlp_parameters(seed, count):
    """Covariance parameters (L, a, flag): L ~ logU[0.1, 2], a ~ logU[0.5, 2], flag ~ B(1/2)."""
    rng = np.random.default_rng(seed)
    L = np.exp(rng.uniform(math.log(0.1), math.log(2.0), size=count))
    a = np.exp(rng.uniform(math.log(0.5), math.log(2.0), size=count))
    flag = (rng.random(count) < 0.5).astype(np.int64)
    return L, a, flag


def mlp_problem(L, a, flag, nelem=48, p=3):
    """Quarter annulus problem with correlation lengths (L, a L) along x1, x2;
    flag 0 = exponential, 1 = squared exponential."""
    return quarter_annulus(nelem, p, "sqexp" if int(flag) == 1 else "exp", (float(L), float(a) * float(L)))


def random_block(n, b, seed=0):
    """Seeded standard normal block of shape (n, b), FP64."""
    return np.random.default_rng(seed).standard_normal((n, b))
