"""Pins of the oracle's geometry, Algorithm 1 and the standard-form operator.

Every test checks the oracle against something other than itself: closed forms,
invariants of the method, brute force, or a second independent evaluation.
Paper passages: Sec. 2.4, Sec. 3.1, Sec. 3.4-3.5, Sec. 4.1-4.4 (Algorithm 1).
"""

import math

import numpy as np
import pytest

import workloads
from oracle import cstage5, eigs, galerkin, geometry, operator


def _desc(d, p, ne, kind, ell, geom, s2=1.0, pt=None, net=None):
    desc = {"dim": d, "degree": [p] * d, "nelem": list(ne) if hasattr(ne, "__len__") else [ne] * d,
            "map": geom, "cov": {"kind": kind, "sigma2": s2,
                                 "corr_len": list(ell) if hasattr(ell, "__len__") else [ell] * d}}
    if pt is not None:
        desc["interp_degree"] = [pt] * d
        desc["interp_nelem"] = list(net) if hasattr(net, "__len__") else [net] * d
    return desc


# ---------------------------------------------------------------- geometry -------
def test_annulus_nurbs_is_exact_circle_and_matches_polar():
    rng = np.random.default_rng(0)
    u = rng.random((200, 2))
    X, det = geometry.map_points({"kind": "annulus_nurbs", "r0": 1.0, "r1": 2.0}, u)
    assert np.max(np.abs(np.linalg.norm(X, axis=1) - (1 + u[:, 0]))) < 1e-14
    assert det.min() > 0
    Xp, _ = geometry.map_points({"kind": "annulus_polar", "r0": 1.0, "r1": 2.0}, u)
    assert np.max(np.abs(np.linalg.norm(Xp, axis=1) - (1 + u[:, 0]))) < 1e-14


@pytest.mark.parametrize("geom,d,measure", [
    ({"kind": "annulus_nurbs", "r0": 1.0, "r1": 2.0}, 2, 0.75 * math.pi),
    ({"kind": "annulus_polar", "r0": 1.0, "r1": 2.0}, 2, 0.75 * math.pi),
    ({"kind": "sine_cube", "eps": 0.05, "amp": [1.0, 0.5, 0.25]}, 3, 1.0),
    ({"kind": "box", "lo": [0.5, -1.0], "hi": [2.0, 1.5]}, 2, 1.5 * 2.5),
])
def test_domain_measure(geom, d, measure):
    assert abs(geometry.domain_measure(geom, d) - measure) < 1e-12


@pytest.mark.parametrize("geom,d", [
    ({"kind": "annulus_nurbs", "r0": 1.0, "r1": 2.0}, 2),
    ({"kind": "sine_cube", "eps": 0.05, "amp": [1.0, 0.5, 0.25]}, 3),
])
def test_jacobian_against_finite_differences(geom, d):
    rng = np.random.default_rng(5)
    u = 0.05 + 0.9 * rng.random((20, d))
    _, det = geometry.map_points(geom, u)
    h = 1e-6
    for r in range(len(u)):
        D = np.zeros((d, d))
        for j in range(d):
            up, um = u[r].copy(), u[r].copy()
            up[j] += h
            um[j] -= h
            D[:, j] = (geometry.map_points(geom, up[None])[0][0] - geometry.map_points(geom, um[None])[0][0]) / (2 * h)
        assert abs(np.linalg.det(D) - det[r]) < 1e-8


def test_sine_cube_is_identity_on_boundary():
    rng = np.random.default_rng(2)
    u = rng.random((30, 3))
    u[:, 0] = 0.0
    X, det = geometry.map_points({"kind": "sine_cube"}, u)
    assert np.max(np.abs(X - u)) < 1e-15


# ---------------------------------------------------------------- operator -------
CASES = [
    _desc(1, 2, 7, "exp", 0.4, {"kind": "identity"}),
    _desc(1, 3, 6, "sqexp", 0.3, {"kind": "box", "lo": [0.0], "hi": [2.0]}, pt=2, net=9),
    _desc(2, 2, (5, 4), "exp", (0.5, 0.8), {"kind": "annulus_nurbs", "r0": 1.0, "r1": 2.0}),
    _desc(2, 3, 4, "sqexp", 0.5, {"kind": "annulus_polar"}, pt=2, net=(6, 3)),
    _desc(3, 2, 3, "exp", 0.5, {"kind": "sine_cube", "eps": 0.05, "amp": [1.0, 0.5, 0.25]}),
]


@pytest.mark.parametrize("desc", CASES)
def test_matrix_free_equals_dense(desc):
    P = operator.Problem(desc)
    A = P.dense_operator()
    V = workloads.random_block(P.N, 5, seed=11)
    Y = P.apply(V)
    assert np.max(np.abs(Y - A @ V)) <= 1e-13 * np.max(np.abs(A @ V))


@pytest.mark.parametrize("desc", CASES[2:4])
def test_symmetric_positive_semidefinite(desc):
    P = operator.Problem(desc)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(P.N)
    v = rng.standard_normal(P.N)
    lhs = u @ P.apply(v)
    rhs = P.apply(u) @ v
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + abs(rhs))
    w = np.linalg.eigvalsh(P.dense_operator())
    assert w.min() >= -1e-12 * w.max()


@pytest.mark.parametrize("kind", ["exp", "sqexp", "exp_l1", "const", "lin"])
@pytest.mark.parametrize("case", [0, 3, 4])
def test_c_stage5_equals_numpy_stage5(kind, case):
    """The C/OpenMP stage 5 and the NumPy one (pinned by the spectral tests) agree for every
    kernel kind, in 1D, 2D and 3D, with unequal correlation lengths per direction."""
    desc = dict(CASES[case])
    d = desc["dim"]
    desc["cov"] = {"kind": kind, "sigma2": 1.3, "corr_len": [0.35, 0.8, 0.55][:d]}
    P = operator.Problem(desc)
    Y = workloads.random_block(P.Nt, 3, seed=2)
    ref = P.stage5(Y)
    assert np.max(np.abs(cstage5.stage5(P, Y) - ref)) < 1e-12 * np.abs(ref).max()


def test_clusters_on_hand_built_spectrum():
    """Runs of consecutive eigenvalues with relative gap below the threshold are grouped;
    the gap is relative to the larger of the two neighbours."""
    w = np.array([1.0, 0.5, 0.4999, 0.49985, 0.3, 0.2999999, 0.1, 0.05, 0.04996])
    assert eigs.clusters(w, rel_gap=1e-3) == [[0], [1, 2, 3], [4, 5], [6], [7, 8]]
    assert eigs.clusters(w, rel_gap=1e-9) == [[i] for i in range(len(w))]
    assert eigs.clusters(w, rel_gap=0.6) == [[0, 1, 2, 3, 4, 5], [6, 7, 8]]
    assert eigs.clusters(w, rel_gap=0.7) == [list(range(len(w)))]
    # exactly repeated and a gap just above the threshold
    assert eigs.clusters(np.array([2.0, 2.0, 2.0 * (1 - 1.001e-3)]), rel_gap=1e-3) == [[0, 1], [2]]
    assert eigs.clusters(np.array([3.0])) == [[0]]


@pytest.mark.parametrize("geom,d,measure", [
    ({"kind": "identity"}, 2, 1.0),
    ({"kind": "box", "lo": [0.0, 0.0, 0.0], "hi": [2.0, 0.5, 1.5]}, 3, 1.5),
    ({"kind": "box", "lo": [1.0], "hi": [3.5]}, 1, 2.5),
])
@pytest.mark.parametrize("p", [1, 3])
def test_constant_kernel_gives_domain_measure(geom, d, measure, p):
    """Gamma = sigma^2: rank one, lambda_1 = sigma^2 |D| exactly, the rest vanish."""
    P = operator.Problem(_desc(d, p, 3, "const", 1.0, geom, s2=1.7))
    w = np.linalg.eigvalsh(P.dense_operator())[::-1]
    assert abs(w[0] - 1.7 * measure) < 1e-13 * 1.7 * measure
    assert np.max(np.abs(w[1:])) < 1e-13 * w[0]


def test_linear_kernel_exact_1d():
    """Gamma = 1 + x x' on [0, 1]: G lies in the interpolation space, so IBQ is exact, and
    range(T) = span{1, x} lies in S_h; lambda = (4 +- sqrt 13) / 6 exactly."""
    for p, pt, ne in [(1, 1, 3), (2, 3, 5), (3, 2, 4)]:
        P = operator.Problem(_desc(1, p, ne, "lin", 1.0, {"kind": "identity"}, pt=pt, net=ne + 1))
        w = np.linalg.eigvalsh(P.dense_operator())[::-1]
        assert np.allclose(w[:2], [(4 + math.sqrt(13)) / 6, (4 - math.sqrt(13)) / 6], rtol=0, atol=1e-13)
        assert np.max(np.abs(w[2:])) < 1e-13


@pytest.mark.parametrize("p,pt,ne,net", [(2, 2, 4, 3), (3, 3, 5, 4), (1, 4, 3, 2)])
def test_linear_kernel_exact_1d_c0_interpolation(p, pt, ne, net):
    """The same closed form through C^0 interpolation spaces (interior breakpoints repeated
    pt times, Sec. 4.2): 1 + x x' still lies in the interpolation space."""
    desc = _desc(1, p, ne, "lin", 1.0, {"kind": "identity"}, pt=pt, net=net)
    desc["interp_mult"] = [pt]
    P = operator.Problem(desc)
    assert P.nt == [net * pt + 1]
    w = np.linalg.eigvalsh(P.dense_operator())[::-1]
    assert np.allclose(w[:2], [(4 + math.sqrt(13)) / 6, (4 - math.sqrt(13)) / 6], rtol=0, atol=1e-13)
    assert np.max(np.abs(w[2:])) < 1e-13


def test_linear_kernel_exact_2d():
    """Gamma = 1 + x . x' on the unit square: lambda = (19 +- sqrt 313)/24 and 1/12."""
    P = operator.Problem(_desc(2, 2, 3, "lin", 1.0, {"kind": "identity"}))
    w = np.linalg.eigvalsh(P.dense_operator())[::-1]
    expect = sorted([(19 + math.sqrt(313)) / 24, 1 / 12, (19 - math.sqrt(313)) / 24], reverse=True)
    assert np.allclose(w[:3], expect, rtol=0, atol=1e-13)
    assert np.max(np.abs(w[3:])) < 1e-13


@pytest.mark.parametrize("kind", ["sqexp", "exp_l1"])
def test_kronecker_separability(kind):
    """Separable kernel on a box with the identity-like map: A~'_2D = A~'_y (x) A~'_x."""
    gx = {"kind": "box", "lo": [0.2], "hi": [1.7]}
    gy = {"kind": "box", "lo": [-0.5], "hi": [0.5]}
    g2 = {"kind": "box", "lo": [0.2, -0.5], "hi": [1.7, 0.5]}
    Px = operator.Problem(_desc(1, 2, 5, kind, 0.7, gx))
    Py = operator.Problem(_desc(1, 3, 3, kind, 0.4, gy))
    d2 = {"dim": 2, "degree": [2, 3], "nelem": [5, 3], "map": g2,
          "cov": {"kind": kind, "sigma2": 1.0, "corr_len": [0.7, 0.4]}}
    P2 = operator.Problem(d2)
    A2 = P2.dense_operator()
    K = np.kron(Py.dense_operator(), Px.dense_operator())
    assert np.max(np.abs(A2 - K)) < 1e-13 * np.max(np.abs(A2))


def test_trace_tends_to_sigma2_measure():
    """sum lambda_i = tr A~' -> sigma^2 |D| (Mercer: int Gamma(x, x) dx) under refinement."""
    gaps = []
    for ne in (4, 8, 16):
        P = operator.Problem(workloads.quarter_annulus(ne, 2, "sqexp", (0.5, 0.5)))
        gaps.append(abs(np.trace(P.dense_operator()) - 0.75 * math.pi))
    assert gaps[0] > gaps[1] > gaps[2]
    assert gaps[2] < 3e-3 and gaps[2] < 0.5 * gaps[0]


def test_rigid_motion_invariance():
    th = 0.7
    Q = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    base = {"kind": "annulus_nurbs", "r0": 1.0, "r1": 2.0}
    moved = dict(base, rotation=Q.tolist(), shift=[3.0, -2.0])
    w1 = np.linalg.eigvalsh(operator.Problem(_desc(2, 2, 5, "exp", 0.6, base)).dense_operator())
    w2 = np.linalg.eigvalsh(operator.Problem(_desc(2, 2, 5, "exp", 0.6, moved)).dense_operator())
    assert np.max(np.abs(w1 - w2)) < 1e-13 * w1.max()


def test_variance_scaling():
    d1 = _desc(2, 2, 5, "sqexp", 0.6, {"kind": "annulus_polar"}, s2=1.0)
    d2 = _desc(2, 2, 5, "sqexp", 0.6, {"kind": "annulus_polar"}, s2=3.5)
    w1 = np.linalg.eigvalsh(operator.Problem(d1).dense_operator())
    w2 = np.linalg.eigvalsh(operator.Problem(d2).dense_operator())
    assert np.max(np.abs(3.5 * w1 - w2)) < 1e-13 * w2.max()


def test_operator_error_decreases_under_interpolation_refinement():
    """|| A - A~ || / || A || shrinks as the interpolation mesh is refined (Sec. 6.2 tables)."""
    errs = []
    for net in (4, 8, 16):
        P = operator.Problem(_desc(1, 2, 4, "sqexp", 0.5, {"kind": "identity"}, pt=2, net=net))
        errs.append(galerkin.relative_operator_errors(P, q=8, nsub=8))
    e2 = [e[0] for e in errs]
    ef = [e[1] for e in errs]
    assert e2[0] > e2[1] > e2[2] and ef[0] > ef[1] > ef[2]
    assert e2[2] < 1e-4


def test_full_galerkin_linear_kernel_matches_ibq():
    """For Gamma = 1 + x x' the IBQ operator equals the exact Galerkin matrix."""
    P = operator.Problem(_desc(1, 2, 4, "lin", 1.0, {"kind": "identity"}))
    A = galerkin.full_galerkin_A(P, q=4, nsub=1)
    assert np.max(np.abs(A - P.dense_A_tilde())) < 1e-14


def test_iterative_equals_dense_eigs():
    desc, k, _ = workloads.config("square16")
    P = operator.Problem(desc)
    w, V = eigs.dense_eigs(P, k)
    wi, Vi = eigs.iterative_eigs(P, k, tol=1e-12)
    assert np.max(np.abs(w - wi)) < 1e-12 * w[0]
    assert np.max(eigs.residual_norms(P, wi, Vi)) < 1e-10 * w[0]
