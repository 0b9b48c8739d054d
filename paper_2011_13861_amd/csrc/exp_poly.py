"""Coefficients of the FP64 exponentials used by the stage-5 kernels (kernels_stage5.hip):

* `exp2_nonpos`: the degree-9 polynomial in f that interpolates 2^(f/2) at the 10 Chebyshev
  nodes of [-1/2, 1/2] (f the range left by the exact reduction f = x - rint(x) of a base-2
  exponent; the kernels' coordinates absorb log2(e)); the kernel squares it to get 2^f;
* `exp_nonpos` (kept for reference): the degree-11 interpolant of e^r on [-ln2/2, ln2/2]
  after a Cody-Waite reduction, and the split of ln2 into a 32-significant-bit high part
  and the rounded remainder.

Standard library only: the function values at the nodes from 80-digit decimal arithmetic,
the Vandermonde system solved in exact rational arithmetic, the result rounded to double.
Prints the constants and the largest relative error of the rounded polynomials (Horner,
double) on a fine grid.

    python paper_2011_13861_amd/csrc/exp_poly.py
"""
from decimal import Decimal, getcontext
from fractions import Fraction
import math

getcontext().prec = 80
LN2 = Decimal("0.6931471805599453094172321214581765680755001343602552541206800094933936219696947156")
PI = Decimal("3.1415926535897932384626433832795028841971693993751058209749445923078164062862089987")


def dcos(x):
    s, t, k = Decimal(1), Decimal(1), 0
    while True:
        k += 2
        t = -t * x * x / (k * (k - 1))
        if s + t == s:
            return s
        s += t


def coefficients(degree=11, widen=Decimal("1.000001"), base2=False, half=False):
    """Interpolant of e^r on [-a, a], a = ln2 / 2 (base2=False), of 2^f on [-a, a], a = 1/2
    (base2=True), or of 2^(f/2) there (base2=True, half=True), at the Chebyshev nodes;
    coefficients of degree 0 first."""
    a = (Decimal(1) / 2 if base2 else LN2 / 2) * widen
    n = degree + 1
    nodes = [a * dcos((2 * Decimal(i) + 1) * PI / (2 * n)) for i in range(n)]
    A = [[Fraction(x) ** j for j in range(n)] for x in nodes]
    scale = LN2 / 2 if half else LN2
    b = [Fraction((x * scale).exp() if base2 else x.exp()) for x in nodes]
    for c in range(n):                                   # Gaussian elimination, exact
        p = max(range(c, n), key=lambda r: abs(A[r][c]))
        A[c], A[p], b[c], b[p] = A[p], A[c], b[p], b[c]
        for r in range(c + 1, n):
            f = A[r][c] / A[c][c]
            A[r] = [A[r][k] - f * A[c][k] for k in range(n)]
            b[r] -= f * b[c]
    x = [Fraction(0)] * n
    for r in range(n - 1, -1, -1):
        x[r] = (b[r] - sum(A[r][k] * x[k] for k in range(r + 1, n))) / A[r][r]
    return [float(v) for v in x], float(a)


def ln2_split():
    m, e = math.frexp(float(LN2))
    hi = math.ldexp(math.floor(math.ldexp(m, 32)), e - 32)
    return hi, float(LN2 - Decimal(hi))


if __name__ == "__main__":
    cs2, a2 = coefficients(degree=9, base2=True, half=True)
    print("base-2 half-argument coefficients (degree 0 first):", [repr(c) for c in cs2])
    worst = 0.0
    for i in range(4001):
        f = -a2 + 2 * a2 * i / 4000
        p = cs2[-1]
        for c in reversed(cs2[:-1]):
            p = p * f + c
        ref = (Decimal(f) * LN2).exp()
        worst = max(worst, float(abs((Decimal(p * p) - ref) / ref)))
    print("largest relative error of the squared rounded polynomial:", worst)
    cs, a = coefficients()
    hi, lo = ln2_split()
    print("ln2_hi", hi.hex(), "ln2_lo", lo.hex())
    print("coefficients (degree 0 first):", [repr(c) for c in cs])
    worst = 0.0
    for i in range(4001):
        r = -a + 2 * a * i / 4000
        p = cs[-1]
        for c in reversed(cs[:-1]):
            p = p * r + c
        worst = max(worst, float(abs((Decimal(p) - Decimal(r).exp()) / Decimal(r).exp())))
    print("largest relative error of the rounded polynomial:", worst)
