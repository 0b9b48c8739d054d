"""The FP64 base-2 exponential of the stage-5 kernels: the constants written in
kernels_stage5.hip are the ones exp_poly.py derives (degree-9 Chebyshev interpolant of
2^(f/2) on [-1/2, 1/2], squared by the kernel), and the exact reduction + polynomial +
squaring + scaling, replayed in double on the host, stays within a few ulp of 2^x on
x <= 0."""
import importlib.util
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2011_13861_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("exp_poly", os.path.join(CSRC, "exp_poly.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _kernel_constants():
    src = open(os.path.join(CSRC, "kernels_stage5.hip")).read()
    body = src[src.index("double exp2_nonpos(double x)"):src.index("double sqrt_pos(double a)")]
    first = float(re.search(r"double p = ([0-9.e+-]+);", body).group(1))
    rest = [float(v) for v in re.findall(r"p = fma\(p, f, ([0-9.e+-]+)\);", body)]
    return [first] + rest   # highest degree first


def test_kernel_constants_are_the_generated_ones():
    coef, half = _gen().coefficients(degree=9, base2=True, half=True)
    assert abs(half - 0.5) < 1e-5
    assert _kernel_constants() == list(reversed(coef))
    src = open(os.path.join(CSRC, "kernels_stage5.hip")).read()
    assert "__builtin_ldexp(p * p, int(n))" in src


def test_host_replay_matches_exp2():
    kc = _kernel_constants()
    x = -np.concatenate([np.linspace(0.0, 60.0, 30001), np.geomspace(1e-12, 1000.0, 5000)])
    n = np.rint(x)
    f = x - n                                            # exact
    p = np.full_like(f, kc[0])
    for c in kc[1:]:
        p = p * f + c
    y = np.ldexp(p * p, n.astype(np.int64))
    ref = np.exp2(x.astype(np.longdouble))
    rel = np.abs(y.astype(np.longdouble) - ref) / ref
    assert rel.max() < 5e-16, rel.max()
    assert np.ldexp(kc[-1], 0) == 1.0                    # 2^0 = 1 exactly
