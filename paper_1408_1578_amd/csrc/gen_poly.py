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
            eP = check(P, Pe, U, 2 * tol_p + fl, f"P{nu}{sfx}", ctype)
            eQ = check(Q, Qe, U, 2 * tol_p * ZA + fl, f"Q{nu}{sfx}", ctype)
            out.append(emit(f"kHankP{nu}{sfx}", Pe, ctype))
            out.append(emit(f"kHankQ{nu}{sfx}", Qe, ctype))
            report.append(f"// P{nu}{sfx}: {len(Pe)} terms, max error {eP:.2e}; "
                          f"Q{nu}{sfx}: {len(Qe)} terms, max error (times t) {eQ / ZA:.2e}\n")
        S = [F((-1) ** (k + 1), math.factorial(2 * k + 3)) for k in range(12)]
        C = [F((-1) ** (k + 1), math.factorial(2 * k + 2)) for k in range(12)]
        Se, _ = economize(S, V, tol_p)
        Ce, _ = economize(C, V, tol_p)
        fl = F(1, 10 ** 7) if ctype == "float" else F(0)
        eS = check(S, Se, V, 2 * tol_p + fl, f"S{sfx}", ctype)
        eC = check(C, Ce, V, 2 * tol_p + fl, f"C{sfx}", ctype)
        out.append(emit(f"kSinS{sfx}", Se, ctype))
        out.append(emit(f"kCosC{sfx}", Ce, ctype))
        report.append(f"// sin S{sfx}: {len(Se)} terms, max error {eS:.2e}; cos C{sfx}: {len(Ce)} terms, "
                      f"max error {eC:.2e}\n")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hankel_poly.hpp")
    with open(path, "w") as f:
        f.write("// Generated by gen_poly.py: economized coefficients (ascending powers of u = 1/z^2\n"
                f"// on [0, 1/{ZA}^2] for the Hankel asymptotic branch, of v = r^2 on [0, {float(V)}] for\n"
                "// sine and cosine).  Do not edit.\n")
        f.writelines(report)
        f.write("#pragma once\n\nnamespace dp {\n\n")
        f.write(f"constexpr double kHankelZA = {ZA}.0;\n")
        f.writelines(out)
        f.write("\n}  // namespace dp\n")
    print("".join(report), end="")


if __name__ == "__main__":
    main()
