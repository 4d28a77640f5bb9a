"""Coefficients of the exp/log polynomials in fastmath.hpp.

Each is the Chebyshev interpolant (near-minimax) of the function on the
interval the argument reduction leaves, computed in 50-digit arithmetic and
rounded to double; printed highest degree first, in the order the Horner
schemes use them.  ``python fastmath_coeffs.py`` prints them with the
interpolation error bound.

  exp:  e^r on |r| <= ln2/2 (widened by 0.05 %), degree 11.
  log:  p(t) = (atanh(sqrt t)/sqrt t - 1)/t on 0 <= t <= s_max^2 (widened by
        0.1 %), s_max = 0.1716 > (sqrt 2 - 1)/(sqrt 2 + 1), degree 6, so that
        ln m = 2 s + 2 s^3 p(s^2) with s = (m - 1)/(m + 1).
"""
import mpmath as mp


def coefficients():
    mp.mp.dps = 50
    half = mp.log(2) / 2 * mp.mpf("1.0005")
    pe, ee = mp.chebyfit(mp.exp, [-half, half], 12, error=True)
    tmax = mp.mpf("0.1716") ** 2 * mp.mpf("1.001")

    def atanh_tail(t):
        if t == 0:
            return mp.mpf(1) / 3
        s = mp.sqrt(t)
        return (mp.atanh(s) / s - 1) / t

    pl, el = mp.chebyfit(atanh_tail, [0, tmax], 7, error=True)
    return {"exp": [float(c) for c in pe], "exp_err": float(ee),
            "log": [float(c) for c in pl], "log_err": float(el)}


if __name__ == "__main__":
    c = coefficients()
    for k in ("exp", "log"):
        print(k, "error %.3g" % c[k + "_err"])
        for v in c[k]:
            print("   ", float.hex(v))
