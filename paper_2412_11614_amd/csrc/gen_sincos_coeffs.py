"""Coefficients of the FP64 sine / cosine in isrs_kernels.hip.

For a phase reduced to |r| <= 1/8 revolution the kernel evaluates
    sin(2 pi r) = r S(r^2),    cos(2 pi r) = 1 + r^2 C(r^2)
with S of degree 6 and C of degree 5 in w = r^2 on [0, 1/64].  This script
finds both by a Remez exchange in 60-digit arithmetic: S minimises the
relative error of the sine, C the error of the cosine.  It prints the
equioscillation error and the coefficients rounded to double, lowest degree
first, then checks the rounded polynomials, evaluated with FP64 rounding and
fused multiply-adds as the kernel does, against 40-digit sin / cos.

    python gen_sincos_coeffs.py
"""
from __future__ import annotations

import random

import mpmath as mp

mp.mp.dps = 60
TWO_PI = 2 * mp.pi
W_MAX = mp.mpf(1) / 64


def remez(f, weight, n, a, b, iters=30, scan=4000):
    """Polynomial P of degree n minimising max |weight(x) (P(x) - f(x))| on [a, b]."""
    m = n + 2
    xs = [(a + b) / 2 - (b - a) / 2 * mp.cos(mp.pi * i / (m - 1)) for i in range(m)]
    coef, level = None, None
    for _ in range(iters):
        A = mp.matrix(m, m)
        rhs = mp.matrix(m, 1)
        for i, x in enumerate(xs):
            for j in range(n + 1):
                A[i, j] = x ** j
            A[i, n + 1] = (-1) ** i / weight(x)
            rhs[i] = f(x)
        sol = mp.lu_solve(A, rhs)
        coef = [sol[j] for j in range(n + 1)]
        level = abs(sol[n + 1])

        def err(x):
            return weight(x) * (mp.polyval(coef[::-1], x) - f(x))

        grid = [a + (b - a) * k / scan for k in range(scan + 1)]
        vals = [err(x) for x in grid]
        idx = [0] + [k for k in range(1, scan) if (vals[k] - vals[k - 1]) * (vals[k + 1] - vals[k]) <= 0] + [scan]
        alt = []
        for k in idx:
            x, v = grid[k], vals[k]
            if alt and mp.sign(alt[-1][1]) == mp.sign(v):
                if abs(v) > abs(alt[-1][1]):
                    alt[-1] = (x, v)
            else:
                alt.append((x, v))
        while len(alt) > m:
            alt.pop(0 if abs(alt[0][1]) < abs(alt[-1][1]) else -1)
        if len(alt) < m:
            break
        xs = [x for x, _ in alt]
    return coef, level


def sine_poly():
    def f(w):
        return mp.sin(TWO_PI * mp.sqrt(w)) / mp.sqrt(w) if w > 0 else TWO_PI

    def weight(w):  # relative error of r S(w)
        return mp.sqrt(w) / mp.sin(TWO_PI * mp.sqrt(w)) if w > 0 else 1 / TWO_PI

    return remez(f, weight, 6, mp.mpf(0), W_MAX)


def cosine_poly():
    def f(w):
        return (mp.cos(TWO_PI * mp.sqrt(w)) - 1) / w

    def weight(w):  # error of 1 + w C(w), relative to the cosine
        return w / mp.cos(TWO_PI * mp.sqrt(w))

    return remez(f, weight, 5, W_MAX * mp.mpf("1e-9"), W_MAX)


def fma(a, b, c):
    with mp.workprec(400):
        v = mp.mpf(a) * mp.mpf(b) + mp.mpf(c)
    return float(v)


def evaluate(t, S, C):
    """The kernel's steps in FP64 for 0 <= t < 1."""
    k = float(round(4.0 * t))
    r = fma(k, -0.25, t)
    w = r * r
    ps = S[-1]
    for c in S[-2::-1]:
        ps = fma(ps, w, c)
    sx = r * ps
    pc = C[-1]
    for c in C[-2::-1]:
        pc = fma(pc, w, c)
    cx = fma(w, pc, 1.0)
    q = int(k) & 3
    s1, c1 = (cx, sx) if q & 1 else (sx, cx)
    return (-s1 if q & 2 else s1), (-c1 if (q + 1) & 2 else c1)


def main():
    S, es = sine_poly()
    C, ec = cosine_poly()
    Sd = [float(x) for x in S]
    Cd = [float(x) for x in C]
    print(f"S: degree 6 in r^2, relative error {mp.nstr(es, 4)}")
    print("  ", ", ".join(repr(x) for x in Sd))
    print(f"C: degree 5 in r^2, error {mp.nstr(ec, 4)}")
    print("  ", ", ".join(repr(x) for x in Cd))
    rng = random.Random(1)
    worst = 0.0
    with mp.workdps(40):
        for i in range(20000):
            t = i / 400.0 if i < 400 else rng.random()
            s, c = evaluate(t, Sd, Cd)
            worst = max(worst, float(abs(mp.mpf(s) - mp.sin(TWO_PI * t))),
                        float(abs(mp.mpf(c) - mp.cos(TWO_PI * t))))
    print(f"largest absolute error over 20000 phases in [0, 1): {worst:.3e}")


if __name__ == "__main__":
    main()
