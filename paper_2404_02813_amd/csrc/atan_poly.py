"""Coefficients of the polynomial in the device Heaviside (rsf_device.hpp).

P(u) of degree 8 with the least maximum relative error against
f(u) = atan(sqrt(u)) / (pi sqrt(u)) on u in [0, 1], by the Remez exchange
algorithm in 40-digit arithmetic (mpmath).  Then atan(t)/pi = t P(t^2) for
t in [0, 1].

    python paper_2404_02813_amd/csrc/atan_poly.py
"""
from mpmath import mp

mp.dps = 40


def f(u):
    u = mp.mpf(u)
    if u == 0:
        return 1 / mp.pi
    s = mp.sqrt(u)
    return mp.atan(s) / (mp.pi * s)


def remez(n, iters=30, grid_n=4000):
    m = n + 2
    xs = [(1 - mp.cos(mp.pi * k / (m - 1))) / 2 for k in range(m)]
    grid = [mp.mpf(k) / grid_n for k in range(grid_n + 1)]
    fg = [f(g) for g in grid]
    for _ in range(iters):
        # P(x_i) + (-1)^i E f(x_i) = f(x_i): equioscillating relative error
        A = mp.matrix(m, m)
        b = mp.matrix(m, 1)
        for i, x in enumerate(xs):
            fx = f(x)
            for j in range(n + 1):
                A[i, j] = x ** j
            A[i, n + 1] = (-1) ** i * fx
            b[i] = fx
        sol = mp.lu_solve(A, b)
        c = [sol[j] for j in range(n + 1)]
        err = [(sum(c[j] * g ** j for j in range(n + 1)) - fv) / fv for g, fv in zip(grid, fg)]
        ext = []
        for k, e in enumerate(err):
            left = err[k - 1] if k > 0 else None
            right = err[k + 1] if k + 1 < len(err) else None
            if (left is None or abs(e) >= abs(left)) and (right is None or abs(e) >= abs(right)):
                ext.append((grid[k], e))
        alt = []
        for x, e in ext:
            if alt and mp.sign(alt[-1][1]) == mp.sign(e):
                if abs(e) > abs(alt[-1][1]):
                    alt[-1] = (x, e)
            else:
                alt.append((x, e))
        if len(alt) < m:
            break
        while len(alt) > m:
            alt.pop(0 if abs(alt[0][1]) < abs(alt[-1][1]) else -1)
        xs = [a[0] for a in alt]
    return c, max(abs(e) for e in err)


if __name__ == "__main__":
    c, e = remez(8)
    print(f"max relative error {float(e):.3e}")
    for j, cj in enumerate(c):
        print(f"c{j} = {float(cj)!r}")
