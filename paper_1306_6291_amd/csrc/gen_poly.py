"""Generate ksym_poly.hpp: polynomial coefficients for the device math.

Methods (all arithmetic in mpmath at 60 significant digits, coefficients then
rounded to the target precision):

* sin / cos on [0, pi/3]: Taylor series at 0, sin through x^19 and cos through
  x^20; the first omitted term bounds the truncation error (< 2e-19 on the
  interval).
* asin(x) = x + x z P(z), z = x^2, x in [0, 1/2] (float64): P is the
  polynomial interpolating (asin(sqrt z)/sqrt z - 1)/z at the Chebyshev points
  of [0, 1/4] (near-minimax; the function is analytic on a Bernstein ellipse
  with rho ~ 13.9, so the coefficients of the Chebyshev expansion decay like
  rho^-k).
* atan(x) = x + x t Q(t), t = x^2, x in [0, 1] (float32): Q interpolates
  (atan(sqrt t)/sqrt t - 1)/t at the Chebyshev points of [0, 1].
* atan(t) = t + t u Q64(u), u = t^2, t in [0, tan(pi/8)] (float64): Q64
  interpolates (atan(sqrt u)/sqrt u - 1)/u at the Chebyshev points of
  [0, tan(pi/8)^2] (the float64 atan2, after the reduction
  atan t = pi/4 - atan((1 - t)/(1 + t)) for t > tan(pi/8)).
* asin(x) = x + x z R(z), z = x^2, x in [0, 1/sqrt 2] (float32): R interpolates
  (asin(sqrt z)/sqrt z - 1)/z at the Chebyshev points of [0, 1/2] (the angles
  phi2, phi3 of the float32 path from their squared sines and cosines).
* float32 tails for the cubic stage of the float32 path, where the first two
  terms of the series are formed in float64 and only the remainder (at most
  1.2 % of sin, 0.5 % of asin on their intervals) in float32:
  sin x = x - x^3/6 + x^5 ST(x^2) on [0, pi/3] and asin x = x + x^3/6 +
  x^5 AT(x^2) on [0, 1/2]; each tail is the Chebyshev interpolant of the
  corresponding function of t = x^2, rounded to float, so the combination
  is accurate to a few 1e-10 relative.

The script prints the maximum relative error of each polynomial measured on a
dense grid in mpmath, and writes those figures into the header.
Run: python paper_1306_6291_amd/csrc/gen_poly.py
"""

import os

import mpmath as mp

mp.mp.dps = 60
HERE = os.path.dirname(os.path.abspath(__file__))


def cheb_interp(f, a, b, deg):
    """Monomial coefficients (ascending) of the degree-`deg` polynomial that
    interpolates f at the deg+1 Chebyshev points of the first kind on [a, b]."""
    n = deg + 1
    xs = [(a + b) / 2 + (b - a) / 2 * mp.cos(mp.pi * (2 * k + 1) / (2 * n)) for k in range(n)]
    ys = [f(x) for x in xs]
    # Newton divided differences, then expand to monomials
    coef = list(ys)
    for j in range(1, n):
        for i in range(n - 1, j - 1, -1):
            coef[i] = (coef[i] - coef[i - 1]) / (xs[i] - xs[i - j])
    poly = [mp.mpf(0)] * n
    for i in range(n - 1, -1, -1):
        # poly = poly * (x - xs[i]) + coef[i]
        new = [mp.mpf(0)] * n
        for k in range(n - 1):
            new[k + 1] += poly[k]
        for k in range(n):
            new[k] -= poly[k] * xs[i]
        new[0] += coef[i]
        poly = new
    return poly


def horner(c, x):
    r = mp.mpf(0)
    for v in reversed(c):
        r = r * x + v
    return r


def max_rel_err(approx, exact, a, b, npts=4001):
    m = mp.mpf(0)
    for k in range(npts):
        x = a + (b - a) * k / (npts - 1)
        e = exact(x)
        if e == 0:
            continue
        m = max(m, abs((approx(x) - e) / e))
    return m


def asin_poly(deg):
    def f(z):
        if z == 0:
            return mp.mpf(1) / 6
        s = mp.sqrt(z)
        return (mp.asin(s) / s - 1) / z
    c = cheb_interp(f, mp.mpf(0), mp.mpf(1) / 4, deg)
    cd = [float(v) for v in c]
    err = max_rel_err(lambda x: x + x * x * x * horner([mp.mpf(v) for v in cd], x * x),
                      mp.asin, mp.mpf(0), mp.mpf(1) / 2)
    return cd, err


def atan_poly(deg):
    def f(t):
        if t == 0:
            return mp.mpf(-1) / 3
        s = mp.sqrt(t)
        return (mp.atan(s) / s - 1) / t
    c = cheb_interp(f, mp.mpf(0), mp.mpf(1), deg)
    import struct
    cf = [struct.unpack("f", struct.pack("f", float(v)))[0] for v in c]
    err = max_rel_err(lambda x: x + x * x * x * horner([mp.mpf(v) for v in cf], x * x),
                      mp.atan, mp.mpf(0), mp.mpf(1))
    return cf, err


def tail(kind, deg):
    if kind == "sin":
        f = lambda t: mp.mpf(1) / 120 if t == 0 else (mp.sin(mp.sqrt(t)) / mp.sqrt(t) - 1 + t / 6) / (t * t)
        b, exact = (mp.pi / 3) ** 2, mp.sin
        comb = lambda x, P: x - x ** 3 / 6 + x ** 5 * P(x * x)
    else:
        f = lambda t: mp.mpf(3) / 40 if t == 0 else (mp.asin(mp.sqrt(t)) / mp.sqrt(t) - 1 - t / 6) / (t * t)
        b, exact = mp.mpf(1) / 4, mp.asin
        comb = lambda x, P: x + x ** 3 / 6 + x ** 5 * P(x * x)
    c = [f32(v) for v in cheb_interp(f, mp.mpf(0), b, deg)]
    err = max_rel_err(lambda x: comb(x, lambda t: horner([mp.mpf(v) for v in c], t)), exact,
                      mp.mpf(0), mp.sqrt(b), npts=801)
    return c, err


def atan_f64_poly(deg):
    b = (mp.sqrt(2) - 1) ** 2

    def f(u):
        if u == 0:
            return mp.mpf(-1) / 3
        s = mp.sqrt(u)
        return (mp.atan(s) / s - 1) / u
    c = [float(v) for v in cheb_interp(f, mp.mpf(0), b, deg)]
    err = max_rel_err(lambda x: x + x * x * x * horner([mp.mpf(v) for v in c], x * x),
                      mp.atan, mp.mpf(0), mp.sqrt(b), npts=801)
    return c, err


def asin_f32_poly(deg):
    def f(z):
        if z == 0:
            return mp.mpf(1) / 6
        s = mp.sqrt(z)
        return (mp.asin(s) / s - 1) / z
    c = [f32(v) for v in cheb_interp(f, mp.mpf(0), mp.mpf(1) / 2, deg)]
    err = max_rel_err(lambda x: x + x * x * x * horner([mp.mpf(v) for v in c], x * x),
                      mp.asin, mp.mpf(0), mp.sqrt(mp.mpf(1) / 2), npts=801)
    return c, err


def f32(v):
    import struct
    return struct.unpack("f", struct.pack("f", float(v)))[0]


def taylor_sin_cos():
    sin_c = [mp.mpf((-1) ** k) / mp.factorial(2 * k + 1) for k in range(10)]    # x^1 .. x^19
    cos_c = [mp.mpf((-1) ** k) / mp.factorial(2 * k) for k in range(11)]        # x^0 .. x^20
    x = mp.pi / 3
    bound_s = x ** 21 / mp.factorial(21)
    bound_c = x ** 22 / mp.factorial(22)
    return [float(v) for v in sin_c], [float(v) for v in cos_c], max(bound_s, bound_c)


def main():
    sin_c, cos_c, tb = taylor_sin_cos()
    asin_c, asin_err = asin_poly(11)
    atan_c, atan_err = atan_poly(8)
    asf_c, asf_err = asin_f32_poly(7)
    at64_c, at64_err = atan_f64_poly(10)
    st_c, st_err = tail("sin", 3)
    at_c, at_err = tail("asin", 6)
    out = []
    out.append("// Generated by gen_poly.py (mpmath, 60 digits).  Do not edit by hand.")
    out.append("#pragma once")
    out.append("namespace ksym {")
    out.append("namespace poly {")
    out.append(f"// sin x = x * sum_k S[k] (x^2)^k, Taylor through x^19; truncation < {float(tb):.1e} on [0, pi/3]")
    out.append("constexpr double S[%d] = {%s};" % (len(sin_c), ", ".join(repr(v) for v in sin_c)))
    out.append(f"// cos x = sum_k C[k] (x^2)^k, Taylor through x^20")
    out.append("constexpr double C[%d] = {%s};" % (len(cos_c), ", ".join(repr(v) for v in cos_c)))
    out.append(f"// asin x = x + x z P(z), z = x^2, x in [0, 1/2]; Chebyshev interpolant, "
               f"max relative error {float(asin_err):.2e}")
    out.append("constexpr double ASIN[%d] = {%s};" % (len(asin_c), ", ".join(repr(v) for v in asin_c)))
    out.append(f"// atan x = x + x t Q(t), t = x^2, x in [0, 1]; Chebyshev interpolant rounded to float, "
               f"max relative error {float(atan_err):.2e}")
    out.append("constexpr float ATAN[%d] = {%s};" % (len(atan_c), ", ".join(repr(v) + "f" for v in atan_c)))
    out.append(f"// atan t = t + t u Q64(u), u = t^2, t in [0, tan(pi/8)]; Chebyshev interpolant, "
               f"max relative error {float(at64_err):.2e}")
    out.append("constexpr double ATAN64[%d] = {%s};" % (len(at64_c), ", ".join(repr(v) for v in at64_c)))
    out.append(f"// asin x = x + x z R(z), z = x^2, x in [0, 1/sqrt 2]; Chebyshev interpolant rounded to float, "
               f"max relative error {float(asf_err):.2e}")
    out.append("constexpr float ASINF[%d] = {%s};" % (len(asf_c), ", ".join(repr(v) + "f" for v in asf_c)))
    out.append(f"// float32 tails: sin x = x - x^3/6 + x^5 ST(x^2), max rel err {float(st_err):.1e}; "
               f"asin x = x + x^3/6 + x^5 AT(x^2), {float(at_err):.1e}")
    out.append("constexpr float ST[%d] = {%s};" % (len(st_c), ", ".join(repr(v) + "f" for v in st_c)))
    out.append("constexpr float AT[%d] = {%s};" % (len(at_c), ", ".join(repr(v) + "f" for v in at_c)))
    out.append("}  // namespace poly")
    out.append("}  // namespace ksym")
    path = os.path.join(HERE, "ksym_poly.hpp")
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    print(f"taylor bound {float(tb):.2e}  asin rel err {float(asin_err):.2e}  atan rel err {float(atan_err):.2e}")
    print("wrote", path)


if __name__ == "__main__":
    main()
