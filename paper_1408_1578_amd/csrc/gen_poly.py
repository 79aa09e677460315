"""Generate hankel_poly.hpp: economized polynomial coefficients for the
device Hankel and sine/cosine evaluations (run from the repository root:
python paper_1408_1578_amd/csrc/gen_poly.py).

All arithmetic is exact (fractions.Fraction); only the final coefficients are
rounded to double.

Hankel asymptotic branch (z >= ZA): with t = 1/z, u = t^2 and the expansion
coefficients a_k(nu) = prod_{m=1..k} (4 nu^2 - (2m - 1)^2)/(8 m),
    H_nu(z) = sqrt(2/(pi z)) e^{i(z - nu pi/2 - pi/4)} (P_nu + i Q_nu),
    P_nu = sum_j (-1)^j a_{2j}(nu) u^j,   Q_nu = t sum_j (-1)^j a_{2j+1}(nu) u^j.
At z >= 25 the terms decrease past k = 40, so the series cut at j = 17 is
exact far below double rounding.  Each of the four polynomials in u is
re-expanded in Chebyshev polynomials on [0, 1/ZA^2] and its highest terms are
dropped while the sum of their magnitudes stays below the tolerance
(Chebyshev economization: |T_k| <= 1 on the interval bounds the error).

Sine/cosine on the reduced range |r| <= pi/4 (v = r^2):
    sin r = r + r v S(v),  S = sum_k (-1)^{k+1} v^k/(2k+3)!
    cos r = 1 + v C(v),    C = sum_k (-1)^{k+1} v^k/(2k+2)!
economized the same way on [0, V], V slightly above (pi/4)^2.

The single-precision evaluation works in quarter turns, w = 2 z / pi, so
that the FP64 reduction is w - rint(w) with no multiple of pi/2 to subtract:
  * the Hankel polynomials become polynomials in s = 1/w^2 = (pi/2)^2 u, i.e.
    P'_k = P_k (2/pi)^{2k} and, with Q multiplied by 1/w instead of t,
    Q'_k = Q_k (2/pi)^{2k+1} (the same functions, so the same error bounds);
  * sine and cosine of (pi/2) f for |f| <= 1/2 (v = f^2), times the
    amplitude constant kappa = (2/pi)/sqrt(2) of the Hankel functions in
    quarter turns (which the sine/cosine pair otherwise needs as an extra
    multiplication):
    kappa sin = f SQ(v), SQ = kappa sum_k (-1)^k (pi/2)^{2k+1} v^k/(2k+1)!,
    kappa cos = CQ(v),   CQ = kappa sum_k (-1)^k (pi/2)^{2k} v^k/(2k)!,
    economized on [0, VQ], VQ slightly above 1/4, to 3e-8: the split FP16
    products downstream carry ~5e-7 relative error anyway.

The script checks every economized polynomial against its full series at
2001 points of its interval in exact arithmetic and fails if the error
exceeds the bound it prints.
"""
from fractions import Fraction as F
import math
import os
import sys

ZA = 25
U = F(1, ZA * ZA)
V = F(617, 1000)  # > (pi/4)^2 = 0.61685...
VQ = F(2501, 10000)  # > (1/2)^2
PI = F("3.14159265358979323846264338327950288419716939937510582097494459")
TWO_OVER_PI = 2 / PI
SQRT2 = F("1.41421356237309504880168872420969807856967187537694807317667974")
KAPPA = SQRT2 / PI  # (2/pi)/sqrt(2)


def a(k, nu):
    p = F(1)
    for m in range(1, k + 1):
        p *= F(4 * nu * nu - (2 * m - 1) ** 2, 8 * m)
    return p


def economize(coef, X, tol):
    """Monomial coefficients (in x on [0, X]) -> economized monomial coefficients."""
    d = len(coef) - 1
    # x = X (1 + s)/2, s in [-1, 1]
    ps = [F(0)] * (d + 1)
    for k, c in enumerate(coef):
        sc = c * (X / 2) ** k
        for i in range(k + 1):
            ps[i] += sc * math.comb(k, i)
    # s^k -> Chebyshev series
    ch = [F(0)] * (d + 1)
    for k, c in enumerate(ps):
        for i in range(k // 2 + 1):
            w = math.comb(k, i) * F(2) ** (1 - k)
            if k == 2 * i:
                w /= 2
            ch[k - 2 * i] += c * w
    keep, dropped = d + 1, F(0)
    while keep > 1 and dropped + abs(ch[keep - 1]) <= tol:
        dropped += abs(ch[keep - 1])
        keep -= 1
    ch = ch[:keep]
    # Chebyshev series -> monomials in s (T_{k+1} = 2 s T_k - T_{k-1})
    T = [[F(1)], [F(0), F(1)]]
    while len(T) < keep:
        t1, t0 = T[-1], T[-2]
        nt = [F(0)] + [2 * c for c in t1]
        for i, c in enumerate(t0):
            nt[i] -= c
        T.append(nt)
    ms = [F(0)] * keep
    for k, c in enumerate(ch):
        for i, tc in enumerate(T[k]):
            ms[i] += c * tc
    # s = 2 x/X - 1 -> monomials in x
    mx = [F(0)] * keep
    for k, c in enumerate(ms):
        for i in range(k + 1):
            mx[i] += c * math.comb(k, i) * (F(2) / X) ** i * (-1) ** (k - i)
    return mx, dropped


def rounded(c, ctype):
    if ctype == "double":
        return float(c)
    import numpy as np
    return float(np.float32(float(c)))


def check(full, econ, X, bound, name, ctype):
    worst = F(0)
    for s in range(2001):
        x = X * s / 2000
        fv = sum(c * x ** k for k, c in enumerate(full))
        # the device evaluates the rounded coefficients
        ev = sum(F(rounded(c, ctype)) * x ** k for k, c in enumerate(econ))
        worst = max(worst, abs(fv - ev))
    if worst > bound:
        sys.exit(f"{name}: error {float(worst):.3e} exceeds {float(bound):.3e}")
    return float(worst)


def emit(name, coefs, ctype):
    vals = ", ".join(repr(rounded(c, ctype)) + ("" if ctype == "double" else "f") for c in coefs)
    return f"constexpr {ctype} {name}[{len(coefs)}] = {{{vals}}};\n"


def main():
    out = []
    report = []
    for prec, tol_p, ctype, sfx in (("fp64", F(2, 10 ** 17), "double", ""), ("fp32", F(1, 10 ** 8), "float", "32")):
        for nu in (0, 1):
            P = [a(2 * j, nu) * (-1) ** j for j in range(18)]
            Q = [a(2 * j + 1, nu) * (-1) ** j for j in range(18)]
            Pe, dP = economize(P, U, tol_p)
            Qe, dQ = economize(Q, U, tol_p * ZA)  # Q is multiplied by t <= 1/ZA
            fl = F(1, 10 ** 7) if ctype == "float" else F(0)  # float rounding of the coefficients
            if ctype == "float":
                # quarter-turn variable s = 1/w^2 = (pi/2)^2 u
                G = TWO_OVER_PI ** 2
                P = [c * G ** k for k, c in enumerate(P)]
                Pe = [c * G ** k for k, c in enumerate(Pe)]
                Q = [c * G ** k * TWO_OVER_PI for k, c in enumerate(Q)]
                Qe = [c * G ** k * TWO_OVER_PI for k, c in enumerate(Qe)]
                X, qb, nm, tmax = U / G, TWO_OVER_PI * 2 * tol_p * ZA + fl, "W", PI / (2 * ZA)
            else:
                X, qb, nm, tmax = U, 2 * tol_p * ZA + fl, "", F(1, ZA)
            eP = check(P, Pe, X, 2 * tol_p + fl, f"P{nu}{nm}{sfx}", ctype)
            eQ = check(Q, Qe, X, qb, f"Q{nu}{nm}{sfx}", ctype)
            out.append(emit(f"kHankP{nu}{nm}{sfx}", Pe, ctype))
            out.append(emit(f"kHankQ{nu}{nm}{sfx}", Qe, ctype))
            report.append(f"// P{nu}{nm}{sfx}: {len(Pe)} terms, max error {eP:.2e}; "
                          f"Q{nu}{nm}{sfx}: {len(Qe)} terms, max error (times {'1/w' if nm else 't'}) "
                          f"{eQ * float(tmax):.2e}\n")
        fl = F(1, 10 ** 7) if ctype == "float" else F(0)
        if ctype == "float":
            tq = F(3, 10 ** 8)
            S = [KAPPA * (-1) ** k * (PI / 2) ** (2 * k + 1) / math.factorial(2 * k + 1) for k in range(14)]
            C = [KAPPA * (-1) ** k * (PI / 2) ** (2 * k) / math.factorial(2 * k) for k in range(14)]
            Se, _ = economize(S, VQ, tq)
            Ce, _ = economize(C, VQ, tq)
            eS = check(S, Se, VQ, 2 * tq + fl, f"SQ{sfx}", ctype)
            eC = check(C, Ce, VQ, 2 * tq + fl, f"CQ{sfx}", ctype)
            names = ("kSinQ", "kCosQ")
        else:
            S = [F((-1) ** (k + 1), math.factorial(2 * k + 3)) for k in range(12)]
            C = [F((-1) ** (k + 1), math.factorial(2 * k + 2)) for k in range(12)]
            Se, _ = economize(S, V, tol_p)
            Ce, _ = economize(C, V, tol_p)
            eS = check(S, Se, V, 2 * tol_p + fl, f"S{sfx}", ctype)
            eC = check(C, Ce, V, 2 * tol_p + fl, f"C{sfx}", ctype)
            names = ("kSinS", "kCosC")
        out.append(emit(f"{names[0]}{sfx}", Se, ctype))
        out.append(emit(f"{names[1]}{sfx}", Ce, ctype))
        report.append(f"// {names[0]}{sfx}: {len(Se)} terms, max error {eS:.2e}; {names[1]}{sfx}: {len(Ce)} terms, "
                      f"max error {eC:.2e}\n")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hankel_poly.hpp")
    with open(path, "w") as f:
        f.write("// Generated by gen_poly.py: economized coefficients (ascending powers of u = 1/z^2\n"
                f"// on [0, 1/{ZA}^2] for the Hankel asymptotic branch, of v = r^2 on [0, {float(V)}] for\n"
                "// sine and cosine; the single-precision W/Q sets in quarter turns w = 2 z / pi:\n"
                f"// s = 1/w^2 and v = f^2 on [0, {float(VQ)}]).  Do not edit.\n")
        f.writelines(report)
        f.write("#pragma once\n\nnamespace dp {\n\n")
        f.write(f"constexpr double kHankelZA = {ZA}.0;\n")
        f.writelines(out)
        f.write("\n}  // namespace dp\n")
    print("".join(report), end="")


if __name__ == "__main__":
    main()
