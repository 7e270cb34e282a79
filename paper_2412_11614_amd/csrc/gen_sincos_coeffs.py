"""Coefficients of the FP64 sine / cosine in isrs_kernels.hip.

For a phase t in revolutions the kernel takes v = t - rint(t) (exact,
|v| <= 1/2) and evaluates the half angle pi v (|pi v| <= pi/2) as
    sin(pi v) = v S(v^2),    cos(pi v) = 1 + v^2 C(v^2)
with S and C of degree 7 in v^2, then doubles it once:
    cos(2 pi v) = 2 cos^2(pi v) - 1,    sin(2 pi v) = 2 cos(pi v) sin(pi v).
This script finds both polynomials by a Remez exchange in 60-digit
arithmetic on r = v / 2 (turns of the half angle, r^2 in [0, 1/16]): S
minimises the relative error of the sine, C the absolute error of the
cosine.  The coefficients are then rescaled to v by powers of two (exact).
It prints the equioscillation errors and the coefficients rounded to
double, lowest degree first, then checks the whole evaluation, in FP64 with
fused multiply-adds as the kernel does, against 40-digit sin / cos.

    python gen_sincos_coeffs.py
"""
from __future__ import annotations

import random

import mpmath as mp

mp.mp.dps = 60
TWO_PI = 2 * mp.pi
W_MAX = mp.mpf(1) / 16
DEG_S, DEG_C = 7, 7


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

    return remez(f, weight, DEG_S, mp.mpf(0), W_MAX)


def cosine_poly():
    def f(w):
        return (mp.cos(TWO_PI * mp.sqrt(w)) - 1) / w

    def weight(w):  # absolute error of 1 + w C(w)
        return w

    return remez(f, weight, DEG_C, W_MAX * mp.mpf("1e-9"), W_MAX)


def fma(a, b, c):
    with mp.workprec(400):
        v = mp.mpf(a) * mp.mpf(b) + mp.mpf(c)
    return float(v)


def evaluate(t, S, C):
    """The kernel's steps in FP64 for a phase t in revolutions."""
    v = t - float(round(t))
    w = v * v
    ps = S[-1]
    for c in S[-2::-1]:
        ps = fma(ps, w, c)
    sh = v * ps
    pc = C[-1]
    for c in C[-2::-1]:
        pc = fma(pc, w, c)
    ch = fma(w, pc, 1.0)
    c2 = ch + ch
    return c2 * sh, fma(c2, ch, -1.0)


def main():
    S, es = sine_poly()
    C, ec = cosine_poly()
    # r = v / 2:  r S(r^2) = v S_j / 2^(2j+1) (v^2)^j,  r^2 C(r^2) = v^2 C_j / 4^(j+1) (v^2)^j
    Sd = [float(x / mp.mpf(2) ** (2 * j + 1)) for j, x in enumerate(S)]
    Cd = [float(x / mp.mpf(4) ** (j + 1)) for j, x in enumerate(C)]
    print(f"S: degree {DEG_S} in v^2, relative error {mp.nstr(es, 4)}")
    print("  ", ", ".join(repr(x) for x in Sd))
    print(f"C: degree {DEG_C} in v^2, absolute error {mp.nstr(ec, 4)}")
    print("  ", ", ".join(repr(x) for x in Cd))
    rng = random.Random(1)
    worst = 0.0
    with mp.workdps(40):
        for i in range(20000):
            t = i / 400.0 if i < 400 else (rng.random() if i % 2 else rng.random() * 1e6)
            s, c = evaluate(t, Sd, Cd)
            tt = mp.mpf(t)
            worst = max(worst, float(abs(mp.mpf(s) - mp.sin(TWO_PI * tt))),
                        float(abs(mp.mpf(c) - mp.cos(TWO_PI * tt))))
    print(f"largest absolute error over 20000 phases: {worst:.3e}")


if __name__ == "__main__":
    main()
