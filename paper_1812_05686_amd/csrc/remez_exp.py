"""Coefficients of the polynomial p of degree n that minimises the relative
error max |p(r) / e^r - 1| on [-ln2/(2N), ln2/(2N)], by the Remez exchange
algorithm (equioscillation at n + 2 points), in 80-digit arithmetic; used for
the exponentials in gs_exp.h (N = 1: the plain reduction; N = 64: the
table-driven one).  Prints the coefficients (highest degree first) and the
relative error before and after rounding them to double.

    python remez_exp.py 9        # degree 9 on [-ln2/2, ln2/2]
    python remez_exp.py 5 64     # degree 5 on [-ln2/128, ln2/128]
"""
import sys

import mpmath as mp

mp.mp.dps = 80


def remez(n, a, iters=40):
    # start from Chebyshev extrema
    pts = [a * mp.cos(mp.pi * (n + 1 - i) / (n + 1)) for i in range(n + 2)]
    coef = None
    for _ in range(iters):
        # p(x_i) - e^x_i = (-1)^i E e^x_i  (relative error weight 1/e^x)
        A = mp.matrix(n + 2, n + 2)
        b = mp.matrix(n + 2, 1)
        for i, x in enumerate(pts):
            for j in range(n + 1):
                A[i, j] = x ** j
            A[i, n + 1] = -((-1) ** i) * mp.e ** x
            b[i] = mp.e ** x
        sol = mp.lu_solve(A, b)
        coef = [sol[j] for j in range(n + 1)]
        err = lambda x: (mp.polyval(coef[::-1], x) - mp.e ** x) / mp.e ** x
        # new extrema: one per sign-alternating interval, plus the end points
        grid = [a * (-1 + 2 * mp.mpf(k) / 4000) for k in range(4001)]
        vals = [err(x) for x in grid]
        ext = []
        seg_start = 0
        for k in range(1, len(grid) + 1):
            if k == len(grid) or mp.sign(vals[k]) != mp.sign(vals[seg_start]):
                kk = max(range(seg_start, k), key=lambda q: abs(vals[q]))
                # refine the extremum by golden-section search on |err|
                lo = grid[max(kk - 1, 0)]
                hi = grid[min(kk + 1, len(grid) - 1)]
                f = lambda x: -abs(err(x))
                for _ in range(60):
                    m1 = lo + (hi - lo) * (3 - mp.sqrt(5)) / 2
                    m2 = lo + (hi - lo) * (mp.sqrt(5) - 1) / 2
                    if f(m1) < f(m2):
                        hi = m2
                    else:
                        lo = m1
                ext.append((lo + hi) / 2 if 0 < kk < len(grid) - 1 else grid[kk])
                seg_start = k
        if len(ext) != n + 2:
            break
        pts = ext
    maxerr = max(abs(err(a * (-1 + 2 * mp.mpf(k) / 20000))) for k in range(20001))
    return coef, maxerr


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 10
    N = int(sys.argv[2]) if len(sys.argv) > 2 else 1
    a = mp.log(2) / (2 * N)
    coef, e = remez(n, a)
    cd = [float(c) for c in coef]
    ed = max(abs((mp.polyval([mp.mpf(c) for c in cd[::-1]], x) - mp.e ** x) / mp.e ** x)
             for x in [a * (-1 + 2 * mp.mpf(k) / 20000) for k in range(20001)])
    print("degree", n, "minimax relative error", mp.nstr(e, 3), "after rounding to double", mp.nstr(ed, 3))
    for c in cd[::-1]:
        print(repr(c))
    if N > 1:  # the reduction constants and the table 2^(j/N), rounded to double
        print("N/ln2", repr(float(N / mp.log(2))), "ln2/N", repr(float(mp.log(2) / N)))
        print("table", ", ".join(repr(float(mp.power(2, mp.mpf(j) / N))) for j in range(N)))


if __name__ == "__main__":
    main()
