"""Coefficients of the closure kernel's GELU.

GELU(a) = a Phi(a) = max(a, 0) - |a| Phi(-|a|).  The kernel evaluates
Phi(-x) for x = min(|a|, X) as a polynomial in u = 2 x / X - 1 of degree
DEG: the Chebyshev interpolant of Phi(-x) on [0, X] (DEG + 1 Chebyshev
nodes of the first kind), written in powers of u for Horner's rule.  Beyond
X the kernel keeps the correction at X, so the error there is at most
Phi(-X) |a|.  Usage: ``python -m paper_1808_04406_amd.gelu_poly`` prints the
C initialiser and the largest error |GELU_poly(a) - GELU(a)| / |a| of an
FP32 Horner evaluation.
"""
import numpy as np
from numpy.polynomial import chebyshev
from scipy.special import ndtr

X = 4.5
DEG = 11


def coefficients(x_max=X, deg=DEG):
    """Power-basis coefficients c_0..c_deg of the interpolant in u."""
    k = np.arange(deg + 1)
    nodes = np.cos(np.pi * (k + 0.5) / (deg + 1))
    cheb = chebyshev.chebfit(nodes, ndtr(-(nodes + 1.0) * x_max / 2.0), deg)
    return chebyshev.cheb2poly(cheb)


def gelu_poly_f32(a, c, x_max=X):
    """The kernel's evaluation, in FP32 operations."""
    f = np.float32
    a = np.asarray(a, np.float32)
    x = np.minimum(np.abs(a), f(x_max))
    u = (x * f(2.0 / x_max) + f(-1.0)).astype(np.float32)
    p = np.full_like(u, f(c[-1]))
    for ck in c[-2::-1]:
        p = (p * u + f(ck)).astype(np.float32)
    return (np.maximum(a, f(0.0)) - x * p).astype(np.float32)


def max_rel_error(c, lo=-12.0, hi=12.0, n=600001):
    a = np.linspace(lo, hi, n)
    g = gelu_poly_f32(a, c).astype(np.float64)
    return float(np.max(np.abs(g - a * ndtr(a)) / np.maximum(np.abs(a), 1e-30)))


def main():
    c = coefficients()
    print("constexpr float kGeluPoly[%d] = {" % len(c))
    print(",\n".join("    %.9ef" % v for v in c) + "};")
    print("// max |error| / |a| = %.3e" % max_rel_error(c))


if __name__ == "__main__":
    main()
