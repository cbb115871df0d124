"""Coefficients of the FP32 erfc used by the FP32-pair kernel.

Form (Hastings 1955, the form of Abramowitz & Stegun 7.1.25-7.1.26):
    erfc(x) = exp(-x^2) * t * Q(t),   t = 1 / (1 + p x),   x >= 0,
with Q a polynomial. p and Q are fitted here by weighted least squares against
scipy.special.erfc, minimising the *relative* error of exp(x^2) erfc(x) on [0, XMAX].
The kernel shares exp(-x^2) with the Ewald force term, so an in-range pair costs one
exp2 and one reciprocal plus the polynomial.

Run: python -m paper_2212_03137_amd.gen_erfc_fit  (prints the C array and the error)
"""
import numpy as np
from scipy.optimize import minimize_scalar
from scipy.special import erfcx

XMAX = 6.0
DEG = 7


def fit(p, deg=DEG, n=4000):
    x = XMAX * (0.5 - 0.5 * np.cos(np.linspace(0, np.pi, n)))      # Chebyshev-spaced
    t = 1.0 / (1.0 + p * x)
    g = erfcx(x)                                                    # exp(x^2) erfc(x)
    A = np.stack([t ** (k + 1) for k in range(deg + 1)], axis=1) / g[:, None]
    c, *_ = np.linalg.lstsq(A, np.ones_like(x), rcond=None)
    approx = (A * g[:, None]) @ c
    return c, np.max(np.abs(approx / g - 1.0))


def best():
    r = minimize_scalar(lambda p: fit(p)[1], bounds=(0.2, 1.2), method="bounded",
                        options={"xatol": 1e-6})
    c, err = fit(r.x)
    return r.x, c, err


if __name__ == "__main__":
    p, c, err = best()
    print(f"// p = {p:.9g}, max relative error of exp(x^2) erfc(x) on [0, {XMAX}]: {err:.2e}")
    print("constexpr float ERFC_P = %.9gf;" % p)
    print("constexpr float ERFC_Q[%d] = {%s};" % (len(c), ", ".join("%.9gf" % v for v in c)))
