"""Coefficients of the polynomial behind the FP64 hill-term exponential.

2^r on [-1/2, 1/2] is replaced by its degree-11 Chebyshev interpolant
(nodes cos(pi (j + 1/2) / 12) / 2), written in the monomial basis. All
arithmetic is NumPy's 80-bit long double, so the coefficients are exact to
double rounding; the interpolant's own error is below 1e-17 relative.

`python exp2_poly.py` prints the C++ array that abp_device.h holds.
"""
import numpy as np

DEGREE = 11


def coefficients(degree=DEGREE):
    ld = np.longdouble
    m = degree + 1
    pi = ld("3.14159265358979323846264338327950288")
    theta = pi * (np.arange(m, dtype=ld) + ld(0.5)) / ld(m)
    f = np.exp2(np.cos(theta) / 2)
    a = np.array([ld(2) / m * np.sum(f * np.cos(ld(k) * theta)) for k in range(m)], dtype=ld)
    a[0] /= 2
    # T_k(2r) in powers of r: T_0 = 1, T_1 = 2r, T_k = 4r T_{k-1} - T_{k-2}
    T = [np.zeros(m, dtype=ld) for _ in range(m)]
    T[0][0] = 1
    if m > 1:
        T[1][1] = 2
    for k in range(2, m):
        T[k][1:] = 4 * T[k - 1][:-1]
        T[k] -= T[k - 2]
    return sum(a[k] * T[k] for k in range(m))


def max_rel_error(coef, n=100001):
    """Largest relative error of the polynomial on [-1/2, 1/2], in long double."""
    r = np.linspace(-0.5, 0.5, n).astype(np.longdouble)
    p = np.zeros_like(r) + coef[-1]
    for c in coef[-2::-1]:
        p = p * r + c
    return float(np.max(np.abs(p / np.exp2(r) - 1)))


def cpp_literals(coef):
    return ", ".join(repr(float(c)) for c in coef)


if __name__ == "__main__":
    c = coefficients()
    print("// 2^r on [-1/2, 1/2], degree %d, max relative error %.2e" % (DEGREE, max_rel_error(c)))
    print("constexpr double kExp2Poly[%d] = {%s};" % (DEGREE + 1, cpp_literals(c)))
