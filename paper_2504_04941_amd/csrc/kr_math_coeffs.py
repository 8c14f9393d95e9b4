"""Writes the polynomial coefficients of kr_math.h (run: python3 kr_math_coeffs.py).

kr_exp2: 2^f on [-1/2, 1/2], degree 10.  kr_log2: log2((1+s)/(1-s)) / s as a
polynomial in u = s^2 on [0, (3 - 2 sqrt 2)^2], degree 7.  Both are Chebyshev
fits in 50-digit arithmetic (near-minimax), rounded to FP64; the script also
reports the largest relative error of the FP64 Horner evaluation on a grid,
each FMA modelled with a single rounding."""
import mpmath as mp

mp.mp.dps = 50


def fit(f, lo, hi, deg):
    poly, err = mp.chebyfit(f, [lo, hi], deg + 1, error=True)
    return [float(c) for c in poly[::-1]], float(err)   # c[0] + c[1] x + ...


def horner(c, x):
    p = c[-1]
    for k in range(len(c) - 2, -1, -1):
        p = float(mp.mpf(p) * mp.mpf(x) + mp.mpf(c[k]))
    return p


def main():
    ce, fe = fit(lambda x: mp.power(2, x), -0.5, 0.5, 10)
    worst = max(abs(float((horner(ce, x) - mp.power(2, x)) / mp.power(2, x)))
                for x in [-0.5 + i / 4000.0 for i in range(4001)])
    print(f"kr_exp2 degree 10: fit error {fe:.2e}, FP64 Horner max rel error {worst:.2e}")
    print("  highest degree first:", ", ".join(c.hex() for c in reversed(ce)))

    smax = (mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)

    def p_exact(u):
        if u == 0:
            return 2 / mp.log(2)
        s = mp.sqrt(u)
        return mp.log((1 + s) / (1 - s)) / mp.log(2) / s

    cl, fl = fit(p_exact, 0, smax ** 2, 7)
    worst = 0.0
    for i in range(4001):
        m = 0.7071067811865476 + i * (1.4142135623730951 - 0.7071067811865476) / 4000
        s = (m - 1.0) / (m + 1.0)
        r = s * horner(cl, s * s)
        ref = mp.log(m) / mp.log(2)
        if abs(ref) > 1e-3:
            worst = max(worst, abs(float((r - ref) / ref)))
    print(f"kr_log2 degree 7 in s^2: fit error {fl:.2e}, FP64 max rel error {worst:.2e}")
    print("  highest degree first:", ", ".join(c.hex() for c in reversed(cl)))


if __name__ == "__main__":
    main()
