"""Writes erf_table.inc: E(z) = erf(z)/z on [0, 6) in 24 pieces of width 1/4,
each a degree-11 polynomial in s = z - c_j about the piece's midpoint
c_j = (j + 1/2)/4.

Each polynomial is the Chebyshev interpolant of E at 12 Chebyshev points of
its piece, computed in 50-digit arithmetic (mpmath) and expanded into powers
of s before rounding the coefficients to doubles.  Beyond z = 6, erf(z) rounds
to 1 in double precision, so erf(z)/z = 1/z there and no piece is needed.

Run from this directory: python gen_erf_table.py (it also prints the largest
error of the rounded table, evaluated by Horner's rule in double precision,
against mpmath's erf on a dense sample, in units of the last place).
"""

import mpmath as mp
import numpy as np

PIECES, WIDTH, DEG = 24, 0.25, 11
mp.mp.dps = 50


def E(z):
    return mp.erf(z) / z if z != 0 else 2 / mp.sqrt(mp.pi)


def piece(j):
    hw = mp.mpf(WIDTH) / 2
    c = (j + mp.mpf(1) / 2) * WIDTH
    n = DEG + 1
    # Chebyshev interpolant at the n Chebyshev points of the first kind
    xs = [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / n) for k in range(n)]
    fx = [E(c + hw * x) for x in xs]
    a = [2 * mp.fsum(fx[k] * mp.cos(mp.pi * i * (k + mp.mpf(1) / 2) / n) for k in range(n)) / n for i in range(n)]
    a[0] /= 2
    # sum_i a_i T_i(s/hw) in powers of s: T_i by the three-term recurrence
    # on coefficient lists in x = s/hw, then x^k = s^k / hw^k
    T = [[mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]]
    for i in range(2, n):
        nxt = [mp.mpf(0)] * (i + 1)
        for k, v in enumerate(T[i - 1]):
            nxt[k + 1] += 2 * v
        for k, v in enumerate(T[i - 2]):
            nxt[k] -= v
        T.append(nxt)
    mono = [mp.mpf(0)] * n
    for i in range(n):
        for k, v in enumerate(T[i]):
            mono[k] += a[i] * v
    return [float(mono[k] / hw ** k) for k in range(n)]


def main():
    table = [piece(j) for j in range(PIECES)]
    worst = 0.0
    for j, coef in enumerate(table):
        c = (j + 0.5) * WIDTH
        for z in np.linspace(j * WIDTH, (j + 1) * WIDTH, 401)[:-1]:
            s = z - c
            r = coef[-1]
            for cf in reversed(coef[:-1]):
                r = r * s + cf
            ref = E(mp.mpf(z))
            err = abs(mp.mpf(r) - ref) / (abs(ref) * mp.mpf(2) ** -52)
            worst = max(worst, float(err))
    with open("erf_table.inc", "w") as f:
        f.write("// Written by gen_erf_table.py: E(z) = erf(z)/z on [0, 6), piece j covers\n")
        f.write("// [j/4, (j+1)/4) as sum_k kErfOverZ[j][k] s^k, s = z - (j + 1/2)/4.\n")
        f.write(f"constexpr int kErfPieces = {PIECES};\n")
        f.write(f"constexpr int kErfTerms = {DEG + 1};\n")
        f.write("constexpr double kErfOverZ[kErfPieces][kErfTerms] = {\n")
        for coef in table:
            f.write("    {" + ", ".join(repr(c) for c in coef) + "},\n")
        f.write("};\n")
    print(f"largest error of the table (Horner in double): {worst:.2f} ulp")


if __name__ == "__main__":
    main()
