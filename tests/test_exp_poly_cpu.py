"""The FP64 exponential of the stage-5 kernels: the constants written in
kernels_stage5.hip are the ones exp_poly.py derives (Cody-Waite split of ln2, degree-11
Chebyshev interpolant of e^r on [-ln2/2, ln2/2]), and the reduction + polynomial +
scaling, replayed in double on the host, stays within a few ulp of exp on x <= 0."""
import importlib.util
import math
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
    body = src[src.index("double exp_nonpos(double x)"):src.index("double sqrt_nonneg(double a)")]
    hi, lo = re.search(r"kLn2Hi = (0x[0-9a-fp.+-]+), kLn2Lo = (0x[0-9a-fp.+-]+);", body).groups()
    first = float(re.search(r"double p = ([0-9.e+-]+);", body).group(1))
    rest = [float(v) for v in re.findall(r"p = fma\(p, r, ([0-9.e+-]+)\);", body)]
    return float.fromhex(hi), float.fromhex(lo), [first] + rest   # highest degree first


def test_kernel_constants_are_the_generated_ones():
    gen = _gen()
    coef, _ = gen.coefficients()
    hi, lo = gen.ln2_split()
    khi, klo, kc = _kernel_constants()
    assert (khi, klo) == (hi, lo)
    assert kc == list(reversed(coef))
    # n * ln2_hi exact for |n| < 2^21: ln2_hi has at most 32 significant bits
    m, _ = math.frexp(hi)
    assert math.ldexp(m, 32) == int(math.ldexp(m, 32))


def test_host_replay_matches_exp():
    khi, klo, kc = _kernel_constants()
    x = -np.concatenate([np.linspace(0.0, 40.0, 20001), np.geomspace(1e-12, 700.0, 5000)])
    n = np.rint(x * 1.4426950408889634)
    r = (x - n * khi) - n * klo                          # exact first product, as with fma
    p = np.full_like(r, kc[0])
    for c in kc[1:]:
        p = p * r + c
    y = np.ldexp(p, n.astype(np.int64))
    ref = np.exp(x)
    rel = np.abs(y - ref) / ref
    assert rel.max() < 1e-15, rel.max()
    assert np.exp(0.0) == np.ldexp(kc[-1], 0)            # exp(0) = 1 exactly
