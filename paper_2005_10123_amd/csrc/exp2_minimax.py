"""Coefficients of the binary64 2^f polynomial in hawkes_device.h (exp2_f64).

Remez exchange for the polynomial p of degree 10 that minimises max |(2^f - p(f)) / 2^f| over
f in [-1/2, 1/2], in 60-digit mpmath arithmetic; prints the coefficients (highest degree first)
rounded to binary64 and the maximal relative error of the rounded polynomial on a fine grid.
Run: python3 exp2_minimax.py [degree]  (needs mpmath; degree 10 by default).
"""
import mpmath as mp

mp.mp.dps = 60


def remez(deg, a=-0.5, b=0.5, iters=30, grid_points=4000):
    f = lambda x: mp.power(2, x)
    n = deg + 2
    xs = [(a + b) / 2 + (b - a) / 2 * mp.cos(mp.pi * (n - 1 - i) / (n - 1)) for i in range(n)]
    for _ in range(iters):
        # p(x_i) + (-1)^i E f(x_i) = f(x_i): equioscillating relative error at the reference points
        A = mp.matrix(n, n)
        rhs = mp.matrix(n, 1)
        for i, x in enumerate(xs):
            for j in range(deg + 1):
                A[i, j] = x ** j
            A[i, deg + 1] = (-1) ** i * f(x)
            rhs[i] = f(x)
        sol = mp.lu_solve(A, rhs)
        c = [sol[j] for j in range(deg + 1)]
        err = lambda x: (f(x) - mp.polyval(c[::-1], x)) / f(x)
        grid = [a + (b - a) * k / grid_points for k in range(grid_points + 1)]
        vals = [err(x) for x in grid]
        ext = [grid[0]] + [grid[k] for k in range(1, grid_points)
                           if (vals[k] - vals[k - 1]) * (vals[k + 1] - vals[k]) <= 0] + [grid[-1]]
        if len(ext) != n:
            ext = sorted(sorted(ext, key=lambda x: -abs(err(x)))[:n])
        xs = ext
    return c


if __name__ == "__main__":
    import sys

    deg = int(sys.argv[1]) if len(sys.argv) > 1 else 10
    c = [mp.mpf(float(v)) for v in remez(deg)]
    pts = [mp.mpf(-0.5) + mp.mpf(k) / 20000 for k in range(20001)]
    worst = max(abs((mp.power(2, x) - mp.polyval(c[::-1], x)) / mp.power(2, x)) for x in pts)
    print(f"degree {deg}, max relative error with binary64 coefficients: {mp.nstr(worst, 5)}")
    for v in c[::-1]:
        print(f"    {float(v):.20e}")
