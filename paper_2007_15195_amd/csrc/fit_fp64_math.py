"""Fit the rational approximations of the FP64 normal CDF and quantile used by
the FP64 SOV loops and write fp64_math_coeffs.h next to this file.

Phi(-a), a >= 0, is R(a) exp(-a^2/2) with R(a) = Phi(-a) exp(a^2/2) (the scaled
tail, erfcx(a / sqrt 2) / 2), a ratio of degrees (9, 10) in a over [0, 38.5]
with positive coefficients (R decays like 1 / (a sqrt(2 pi)), as the degrees
allow); beyond 38.5, Phi(-a) is below the smallest subnormal.

z = Phi^{-1}(q) is taken in three pieces, on p = min(q, 1 - q) (1 - q is exact
for q >= 1/2):

  central, |q - 1/2| <= 0.425:  z = r P(x) / Q(x), r = q - 1/2, x = 0.425^2 - r^2
      (x runs from 0 at the edges to 0.180625 at the centre, which keeps the
      coefficients of one sign and the evaluation free of cancellation);
  tail 1, s = sqrt(-log p) in [sqrt(-log 0.075), 5]:  |z| = P(s - S1) / Q(s - S1);
  tail 2, s in [5, 27.3] (p down to the smallest subnormal):  |z| = P(s - 5) / Q(s - 5).

This is the classical three-region layout for the normal quantile (the
central rational in r^2, the tails in sqrt(-log p)); the coefficients here
are this file's own fits. Each ratio is fitted by Lawson's iteratively
reweighted least squares on the linearised problem P(x) - f(x) Q(x) = 0 with
relative-error weights, solved in 40-digit arithmetic (mpmath) against
40-digit targets: from erfinv where p > 1e-8, else from a Newton solve of
log Phi(z) = log p.

The CDF's Gaussian factor needs exp(x) for x in [-745, 0]: x = k ln 2 + r with
|r| <= ln 2 / 2 (ln 2 in the same two parts as below), exp(r) = 1 + r + r^2 g(r),
g a degree-10 polynomial in u = r + 0.3466 >= 0 fitted here in relative error
(g is absolutely monotone, so its coefficients in u are positive), and the
result 2^k exp(r).

The quantile's tail needs log p. Its logarithm uses the classical reduction
p = m 2^e, m in [sqrt(1/2), sqrt(2)), log m = 2 atanh(s) with s = (m - 1) / (m + 1),
|s| <= 3 - 2 sqrt 2; the series' remainder (2 atanh(s) - 2 s) / s = z P(z), z = s^2,
takes a degree-6 polynomial P fitted here in relative error, and ln 2 is split
into a head with 42 significant bits (so that e times it is exact) and a tail.

Run: python fit_fp64_math.py   (development-time only; the header is committed)
"""
from __future__ import annotations

import os

import mpmath

mpmath.mp.dps = 40
ONE = mpmath.mpf(1)


def z_of_p(p):
    """Phi^{-1}(p) for p in (0, 1/2], 40 digits."""
    p = mpmath.mpf(p)
    if p > mpmath.mpf("1e-8"):   # 1 - 2p keeps over 30 of p's digits at 40-digit precision
        return -mpmath.sqrt(2) * mpmath.erfinv(1 - 2 * p)
    z = -mpmath.sqrt(-2 * mpmath.log(p))
    for _ in range(200):
        dz = (mpmath.log(mpmath.ncdf(z)) - mpmath.log(p)) / (mpmath.npdf(z) / mpmath.ncdf(z))
        z -= dz
        if abs(dz) < mpmath.mpf(10) ** -36:
            break
    return z


def cheb_nodes(a, b, n):
    a, b = mpmath.mpf(a), mpmath.mpf(b)
    return [(a + b) / 2 + (b - a) / 2 * mpmath.cos(mpmath.pi * (2 * k + 1) / (2 * n)) for k in range(n)]


def lawson(xs, ys, n, m, iters=40):
    """Near-minimax P/Q (degrees n, m; Q(0) = 1) in relative error."""
    N = len(xs)
    w = [ONE / N] * N
    best = None
    for _ in range(iters):
        rows, rhs = [], []
        for x, y, wi in zip(xs, ys, w):
            sw = mpmath.sqrt(wi) / abs(y)
            rows.append([sw * x ** j for j in range(n + 1)] + [-sw * y * x ** j for j in range(1, m + 1)])
            rhs.append(sw * y)
        c, _ = mpmath.qr_solve(mpmath.matrix(rows), mpmath.matrix(rhs))
        p = [c[j] for j in range(n + 1)]
        q = [ONE] + [c[n + 1 + j] for j in range(m)]
        err = []
        for x, y in zip(xs, ys):
            P = mpmath.polyval(p[::-1], x)
            Q = mpmath.polyval(q[::-1], x)
            err.append(abs(P / Q - y) / abs(y))
        e = max(err)
        if best is None or e < best[0]:
            best = (e, p, q)
        tot = sum(wi * ei for wi, ei in zip(w, err))
        w = [max(wi * ei / tot, mpmath.mpf("1e-30")) for wi, ei in zip(w, err)]
    return best


def scaled_tail(a):
    """R(a) = Phi(-a) exp(a^2 / 2), 40 digits."""
    a = mpmath.mpf(a)
    return mpmath.ncdf(-a) * mpmath.exp(a * a / 2)


S1 = mpmath.sqrt(-mpmath.log(mpmath.mpf("0.075")))
S2 = mpmath.mpf(5)
S3 = mpmath.mpf("27.3")
R2MAX = mpmath.mpf("0.425") ** 2

S_MAX = (mpmath.sqrt(2) - 1) / (mpmath.sqrt(2) + 1)


def log_remainder(z):
    """(2 atanh(s) - 2 s) / (s z), s = sqrt(z): the atanh series after its first term, over z."""
    if z == 0:
        return mpmath.mpf(2) / 3
    s = mpmath.sqrt(z)
    return (2 * mpmath.atanh(s) - 2 * s) / (s * z)


EXP_SHIFT = mpmath.mpf("0.3466")


def exp_remainder(r):
    """(exp(r) - 1 - r) / r^2, 40 digits."""
    if r == 0:
        return mpmath.mpf(1) / 2
    return (mpmath.exp(r) - 1 - r) / (r * r)


def ln2_split():
    """ln 2 = hi + lo, hi with 42 significant bits (e * hi exact for |e| < 2^11)."""
    ln2 = mpmath.log(2)
    hi = mpmath.floor(ln2 * 2 ** 42) / 2 ** 42
    return hi, ln2 - hi


PIECES = {
    # name: (degrees, variable nodes, target at a node)
    "phi": ((9, 10), lambda: cheb_nodes(0, 38.5, 160), scaled_tail),
    "central": ((7, 7), lambda: cheb_nodes(0, R2MAX, 120),
                lambda x: z_of_p(mpmath.mpf("0.5") - mpmath.sqrt(R2MAX - x)) / (-mpmath.sqrt(R2MAX - x))
                if x < R2MAX else mpmath.sqrt(2 * mpmath.pi)),
    "tail1": ((7, 7), lambda: cheb_nodes(0, S2 - S1, 120),
              lambda x: -z_of_p(mpmath.exp(-(x + S1) ** 2))),
    "tail2": ((7, 7), lambda: cheb_nodes(0, S3 - S2, 120),
              lambda x: -z_of_p(mpmath.exp(-(x + S2) ** 2))),
}


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    out = ["// Generated by fit_fp64_math.py: rational approximations of the normal CDF's scaled tail and quantile",
           "// for the FP64 loops (coefficients in increasing powers; denominators start at 1).",
           "#pragma once", "", "namespace vecchia {", ""]
    for name, ((n, m), nodes, f) in PIECES.items():
        xs = nodes()
        ys = [f(x) for x in xs]
        e, p, q = lawson(xs, ys, n, m)
        print(f"{name}: degrees ({n},{m}), max relative error of the fit {mpmath.nstr(e, 3)}")
        cname = name.upper()
        out.append(f"// {name}: fitted max relative error {mpmath.nstr(e, 3)}")
        pre = "kPhiR" if name == "phi" else f"kNinv{name.capitalize()}"
        out.append(f"constexpr double {pre}P[{n + 1}] = {{" +
                   ", ".join(mpmath.nstr(c, 20, min_fixed=0, max_fixed=0) for c in p) + "};")
        out.append(f"constexpr double {pre}Q[{m + 1}] = {{" +
                   ", ".join(mpmath.nstr(c, 20, min_fixed=0, max_fixed=0) for c in q) + "};")
    out.append(f"constexpr double kNinvS1 = {mpmath.nstr(S1, 20)};   // sqrt(-log 0.075)")
    xs = cheb_nodes(0, S_MAX ** 2, 100)
    e, p, _ = lawson(xs, [log_remainder(x) for x in xs], 6, 0)
    print(f"log: degree 6, max relative error of the fit {mpmath.nstr(e, 3)}")
    out.append(f"// log: the atanh series' remainder over z = s^2, fitted max relative error {mpmath.nstr(e, 3)}")
    out.append("constexpr double kLogP[7] = {" +
               ", ".join(mpmath.nstr(c, 20, min_fixed=0, max_fixed=0) for c in p) + "};")
    xs = cheb_nodes(0, 2 * EXP_SHIFT, 120)
    e, p, _ = lawson(xs, [exp_remainder(x - EXP_SHIFT) for x in xs], 10, 0)
    print(f"exp: degree 10, max relative error of the fit {mpmath.nstr(e, 3)}")
    out.append(f"// exp: (exp(r) - 1 - r) / r^2 in u = r + kExpShift on |r| <= kExpShift, "
               f"fitted max relative error {mpmath.nstr(e, 3)}")
    out.append(f"constexpr double kExpShift = {mpmath.nstr(EXP_SHIFT, 20)};")
    out.append("constexpr double kExpG[11] = {" +
               ", ".join(mpmath.nstr(c, 20, min_fixed=0, max_fixed=0) for c in p) + "};")
    hi, lo = ln2_split()
    out.append(f"constexpr double kLn2Hi = {mpmath.nstr(hi, 20)};   // 42 significant bits")
    out.append(f"constexpr double kLn2Lo = {mpmath.nstr(lo, 20)};")
    out += ["", "}  // namespace vecchia", ""]
    with open(os.path.join(here, "fp64_math_coeffs.h"), "w") as fh:
        fh.write("\n".join(out))


if __name__ == "__main__":
    main()
