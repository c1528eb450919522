"""Coefficients of the FP64 arcsine used for EG2's arc angles (asin_small in af_device.hpp).

asin(x) = x + x^3 g(x^2) on 0 <= x <= 1/sqrt(2), with g(t) = (asin(sqrt t) / sqrt t - 1) / t.
g is analytic on [0, 1/2] (its nearest singularity is the branch point t = 1), so its
interpolant at Chebyshev points converges geometrically; the interpolant of degree N is
computed here in 60-digit arithmetic, converted to monomial coefficients in t and rounded to
double.  The degree is the smallest whose maximum error, with the rounded coefficients and the
polynomial evaluated exactly, is below a quarter of an ulp of asin(x) over the interval.

Run: python asin_coeffs.py  (prints the table for af_device.hpp and the error estimate).
"""
import mpmath as mp

mp.mp.dps = 60
T1 = mp.mpf(1) / 2  # the interval [0, T1] of t = x^2


def g(t):
    if t == 0:
        return mp.mpf(1) / 6
    r = mp.sqrt(t)
    return (mp.asin(r) / r - 1) / t


def interpolant(n):
    """Monomial coefficients (in t) of the degree-n interpolant of g at the Chebyshev points of
    [0, T1]."""
    nodes = [T1 / 2 * (1 + mp.cos(mp.pi * (k + mp.mpf(1) / 2) / (n + 1))) for k in range(n + 1)]
    # Newton divided differences, then expansion into monomials
    c = [g(t) for t in nodes]
    for j in range(1, n + 1):
        for i in range(n, j - 1, -1):
            c[i] = (c[i] - c[i - 1]) / (nodes[i] - nodes[i - j])
    mono = [mp.mpf(0)] * (n + 1)
    for i in range(n, -1, -1):
        # mono = mono * (t - nodes[i]) + c[i]
        nxt = [mp.mpf(0)] * (n + 1)
        for k in range(n, 0, -1):
            nxt[k] = mono[k - 1] - nodes[i] * mono[k]
        nxt[0] = c[i] - nodes[i] * mono[0]
        mono = nxt
    return mono


def max_error_ulps(coef, samples=4000):
    """Largest |x + x^3 p(x^2) - asin(x)| / ulp(asin(x)) over the interval, p with the
    double-rounded coefficients evaluated exactly."""
    cd = [mp.mpf(float(a)) for a in coef]
    worst = mp.mpf(0)
    xmax = mp.sqrt(T1)
    for k in range(1, samples + 1):
        x = xmax * k / samples
        t = x * x
        p = mp.mpf(0)
        for a in reversed(cd):
            p = p * t + a
        y = mp.asin(x)
        ulp = mp.mpf(2) ** (mp.floor(mp.log(y, 2)) - 52)
        worst = max(worst, abs(x + x ** 3 * p - y) / ulp)
    return worst


def main():
    for n in range(12, 30):
        coef = interpolant(n)
        err = max_error_ulps(coef, 800)
        if err < 0.25:
            err = max_error_ulps(coef)
            if err < 0.25:
                break
    print(f"// degree {n} in t = x^2; max error of the polynomial part {float(err):.3f} ulp")
    print(f"constexpr double kAsinC[{n + 1}] = {{")
    for a in coef:
        print(f"    {float(a)!r},")
    print("};")


if __name__ == "__main__":
    main()
