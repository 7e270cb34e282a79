"""The FP64 sine / cosine of the region kernel, checked on the host.

The kernel's `sincos_turns` reduces a phase t (revolutions) to v = t - rint(t),
evaluates the half angle pi v with two degree-7 polynomials in v^2 and doubles
it once.  This test reads the coefficients from the kernel source, repeats
those steps in 80-bit arithmetic (which stands in for the fused multiply-adds)
and compares with the extended-precision sin / cos of 2 pi t.
"""
import os
import re

import numpy as np

PI_LD = np.longdouble("3.14159265358979323846264338327950288")
SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2412_11614_amd", "csrc", "isrs_kernels.hip")


def _coefficients():
    src = open(SRC).read()
    body = src[src.index("void sincos_turns"):]
    body = body[:body.index("\n}\n")]
    num = r"(-?[0-9.]+(?:e-?[0-9]+)?)"
    ps = [float(re.search(r"double ps = " + num, body).group(1))]
    ps += [float(x) for x in re.findall(r"ps = fma\(ps, w, " + num + r"\)", body)]
    pc = [float(re.search(r"double pc = " + num, body).group(1))]
    pc += [float(x) for x in re.findall(r"pc = fma\(pc, w, " + num + r"\)", body)]
    return ps, pc   # highest degree first


def _kernel_steps(t, ps, pc):
    L = np.longdouble
    v = t - np.rint(t)                       # exact in double
    w = L(v * v)                             # rounded to double in the kernel
    w = L(np.float64(w))
    s = L(ps[0])
    for c in ps[1:]:
        s = L(np.float64(s * w + L(c)))
    sh = L(np.float64(L(v) * s))
    cp = L(pc[0])
    for c in pc[1:]:
        cp = L(np.float64(cp * w + L(c)))
    ch = L(np.float64(w * cp + L(1.0)))
    c2 = L(np.float64(ch + ch))
    return np.float64(c2 * sh), np.float64(c2 * ch - L(1.0))


def test_coefficients_are_the_two_degree_seven_polynomials():
    ps, pc = _coefficients()
    assert len(ps) == 8 and len(pc) == 8
    # leading terms of sin(pi v) / v and (cos(pi v) - 1) / v^2
    assert abs(ps[-1] - np.pi) < 1e-15
    assert abs(pc[-1] + np.pi ** 2 / 2) < 1e-14


def test_sine_cosine_of_revolutions_within_1e15():
    ps, pc = _coefficients()
    rng = np.random.default_rng(7)
    t = np.concatenate([rng.random(20000), rng.random(20000) * 1e6, -rng.random(5000) * 1e3,
                        np.arange(-8, 9) / 8.0, np.array([0.25, 0.5, 0.75, 1e7 + 0.125])])
    worst = 0.0
    for x in t:
        s, c = _kernel_steps(np.float64(x), ps, pc)
        ang = 2 * PI_LD * np.longdouble(x - np.rint(x))
        worst = max(worst, abs(float(s - np.sin(ang))), abs(float(c - np.cos(ang))))
    assert worst < 1e-15, worst
