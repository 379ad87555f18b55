"""Coefficients of the polynomial behind gelu_exact in cnn_common.h.

GELU(z) = z Phi(z) = max(z, 0) - |z| Q(|z|), with Q(a) = Phi(-a) the upper
tail of the standard normal distribution.  On 0 <= a <= 6 the kernel takes
Q(a) = 2^P(a), where P is the degree-10 polynomial fitted here to log2 Q(a)
by least squares in the Chebyshev basis on 20001 points of [0, 6] (then
written in powers of a for Horner's rule); beyond 6, Q(6) ~ 1e-9 stands in
for the tail.  log2 Q is smooth on the interval (it behaves like
-a^2 / (2 ln 2) - log2(a sqrt(2 pi)) for large a), so one polynomial and one
exp2 replace the reciprocal, the exponential and the polynomial of the
erfc form.  Run this file to print the coefficients and the error of their
float32 Horner evaluation against the double-precision tail.
"""
import numpy as np
from scipy.special import log_ndtr

A_MAX = 6.0
DEGREE = 10


def fit():
    a = np.linspace(0.0, A_MAX, 20001)
    target = log_ndtr(-a) / np.log(2.0)
    cheb = np.polynomial.chebyshev.Chebyshev.fit(a, target, DEGREE, domain=[0.0, A_MAX])
    return cheb.convert(kind=np.polynomial.Polynomial).coef.astype(np.float32)


def horner32(coef, a):
    a = a.astype(np.float32)
    acc = np.full_like(a, coef[-1])
    for c in coef[-2::-1]:
        acc = (acc * a + c).astype(np.float32)
    return acc


if __name__ == "__main__":
    coef = fit()
    a = np.linspace(0.0, A_MAX, 600001)
    q = np.exp(log_ndtr(-a))
    q32 = np.exp2(horner32(coef, a).astype(np.float64))
    rel = np.abs(q32 / q - 1.0)
    print("// log2 Phi(-a) on [0, %g], degree %d, coefficients of a^0 .. a^%d" % (A_MAX, DEGREE, DEGREE))
    for k, c in enumerate(coef):
        print("  %.9ef,  // a^%d" % (c, k))
    print("// max relative error of 2^P(a) in float32: %.2e (a < 3: %.2e)"
          % (rel.max(), rel[a < 3].max()))
    print("// max |GELU error| for z = -a: %.2e" % np.max(a * np.abs(q32 - q)))
