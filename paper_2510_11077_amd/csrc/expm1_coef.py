"""Coefficients of the polynomial core of the fast expm1 in k_filter.hip.

With u = x / ln 2 - k (|u| <= 1/2, k an integer),
    expm1(u ln 2) = u (ln 2 + u H(u)),   H(u) = (expm1(u ln 2) - u ln 2) / u^2,
and H is approximated on [-1/2, 1/2] by its 10-term Chebyshev fit (mpmath's
chebyfit, 50 significant digits), printed highest degree first as C++
literals. Run: python expm1_coef.py
"""
import mpmath as mp

mp.mp.dps = 50
LN2 = mp.log(2)


def H(u):
    if abs(u) < mp.mpf("1e-25"):
        return LN2 ** 2 / 2 + LN2 ** 3 * u / 6
    return (mp.expm1(u * LN2) - u * LN2) / u ** 2


if __name__ == "__main__":
    poly, err = mp.chebyfit(H, [-0.5, 0.5], 10, error=True)
    print("// max |H - fit| on [-1/2, 1/2]: %.3e" % float(err))
    print("// expm1 relative error from the fit: <= %.3e" % float(err / 2 / LN2))
    for c in poly:
        print("    %s," % mp.nstr(c, 21, min_fixed=-30, max_fixed=30))
