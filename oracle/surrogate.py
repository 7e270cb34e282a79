"""CPU reference of the FWM-efficiency surrogate (FP64 numpy).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the test suite and
the benchmark's CPU-baseline leg are its only users.

Two parts:

* the learning target of one query point: y = ln(|mu_s|^2 / L_eff^2) of the
  segment closed form (Eqs. 7-10, dz = 1 km) for one span with the ISRS
  profile of Eq. 25 over a 10 THz band, and y6 = ln(|eta|^2 / L_eff^2) of the
  same span without ISRS (Eq. 6), both computed by this package's C oracle;
* the network input phi(x): the 9 scaled features and 7 derived from the
  physical values (cos and sin of chi L and of chi Delta, Delta = L / K with
  K = ceil(L / 1 km), ln(1 + |chi| / alpha) / 8 - 1, alpha / |beta| and
  chi / |beta| with |beta| = sqrt(alpha^2 + chi^2), chi of Eq. 24);
* the network, written from its definition: h_1 = silu(phi(x) W1 + b1),
  h_l = silu(h_{l-1} W_l + b_l) for l = 2..4, o = h_4 w5 + b5, loss = mean
  over rows of (o - r)^2, with silu(z) = z / (1 + e^{-z}), and its gradient
  by the chain rule.  The gradient is checked against central differences.

Query points are 16 floats: 9 features scaled linearly from the box below to
[-1, 1] (f1, f2, f in THz from the grid centre; L km; alpha dB/km; beta2
ps^2/km; beta3 ps^3/km; Cr 1/(W km THz); Ptot dBm), then 7 ignored entries.
The network functions below take phi(x), an [n, 16] array.
"""
from __future__ import annotations

import numpy as np

from . import mu as _mu, leff as _leff, alpha_lin as _alpha_lin

NIN = 16
NF = 9
BOX_LO = np.array([-5.0, -5.0, -5.0, 80.0, 0.18, -23.0, 0.10, 0.020, 17.0])
BOX_HI = np.array([5.0, 5.0, 5.0, 100.0, 0.22, -20.0, 0.16, 0.035, 23.0])
B_TOT = 10.0


def layout(hidden=256, nin=NIN):
    """Offsets of the flat parameter vector: W1, b1, W2, b2, W3, b3, W4, b4, w5, b5."""
    shapes = [("W1", (nin, hidden)), ("b1", (hidden,))]
    for l in (2, 3, 4):
        shapes += [(f"W{l}", (hidden, hidden)), (f"b{l}", (hidden,))]
    shapes += [("w5", (hidden,)), ("b5", (1,))]
    out, off = {}, 0
    for name, shp in shapes:
        n = int(np.prod(shp))
        out[name] = (off, shp)
        off += n
    return out, off


def unpack(params, hidden=256, nin=NIN):
    lay, n = layout(hidden, nin)
    p = np.asarray(params, dtype=np.float64)
    assert p.size == n, (p.size, n)
    return {k: p[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in lay.items()}


def pack(d, hidden=256, nin=NIN):
    lay, n = layout(hidden, nin)
    p = np.zeros(n)
    for k, (o, s) in lay.items():
        p[o:o + int(np.prod(s))] = np.asarray(d[k], dtype=np.float64).reshape(-1)
    return p


def silu(z):
    return z / (1.0 + np.exp(-z))


def forward(params, x, hidden=256):
    """Network output o [n] for query points x [n, 16]."""
    P = unpack(params, hidden, x.shape[1])
    h = np.asarray(x, dtype=np.float64)
    for l in (1, 2, 3, 4):
        h = silu(h @ P[f"W{l}"] + P[f"b{l}"])
    return h @ P["w5"] + P["b5"][0]


def loss_and_grad(params, x, r, hidden=256):
    """Mean squared error of o against r, and its gradient (flat, same layout)."""
    P = unpack(params, hidden, x.shape[1])
    x = np.asarray(x, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    n = x.shape[0]
    zs, hs = [], [x]
    for l in (1, 2, 3, 4):
        z = hs[-1] @ P[f"W{l}"] + P[f"b{l}"]
        zs.append(z)
        hs.append(silu(z))
    o = hs[-1] @ P["w5"] + P["b5"][0]
    e = o - r
    loss = float(np.mean(e * e))
    G = {}
    do = 2.0 * e / n                                  # d loss / d o
    G["w5"] = hs[4].T @ do
    G["b5"] = np.array([do.sum()])
    dh = np.outer(do, P["w5"])                        # d loss / d h4
    for l in (4, 3, 2, 1):
        z = zs[l - 1]
        s = 1.0 / (1.0 + np.exp(-z))
        dz = dh * (s * (1.0 + z * (1.0 - s)))         # silu'(z) = s (1 + z (1 - s))
        G[f"W{l}"] = hs[l - 1].T @ dz
        G[f"b{l}"] = dz.sum(axis=0)
        dh = dz @ P[f"W{l}"].T
    return loss, pack(G, hidden, x.shape[1])


def features(x):
    """Network input phi(x) [n, 16] of query points x [n, 16] (FP64)."""
    x = np.asarray(x, dtype=np.float64)
    ph = decode(x)
    a, b, c, L, adb = ph[:, 0], ph[:, 1], ph[:, 2], ph[:, 3], ph[:, 4]
    b2, b3 = ph[:, 5], ph[:, 6]
    alpha = adb * np.log(10.0) / 10.0
    chi = 4.0 * np.pi ** 2 * ((a - c) * (b - c)) * (b2 + np.pi * b3 * (a + b))     # Eq. 24
    K = np.ceil(L / 1.0)
    m = np.sqrt(alpha ** 2 + chi ** 2)
    out = np.zeros((x.shape[0], NIN))
    out[:, :NF] = x[:, :NF]
    out[:, 9] = np.cos(chi * L)
    out[:, 10] = np.sin(chi * L)
    out[:, 11] = np.log1p(np.abs(chi) / alpha) / 8.0 - 1.0
    out[:, 12] = alpha / m
    out[:, 13] = chi / m
    out[:, 14] = np.cos(chi * (L / K))
    out[:, 15] = np.sin(chi * (L / K))
    return out


def decode(x):
    """Physical parameters of query points x [n, 16] (float64 [n, 9])."""
    x = np.asarray(x, dtype=np.float64)[:, :NF]
    return BOX_LO + 0.5 * (x + 1.0) * (BOX_HI - BOX_LO)


def encode(phys):
    phys = np.atleast_2d(np.asarray(phys, dtype=np.float64))
    x = np.zeros((phys.shape[0], NIN))
    x[:, :NF] = 2.0 * (phys - BOX_LO) / (BOX_HI - BOX_LO) - 1.0
    return x


def _span(L, adb, b2, b3, cr):
    # fields: length, alpha (dB/km), beta2, beta3, gamma, Cr
    return np.array([L, adb, b2, b3, 1.3, cr], dtype=np.float64)


def target(phys, cr=None):
    """(y, y6) of one point: segment closed form with ISRS and Eq. 6 without."""
    a, b, c, L, adb, b2, b3, crv, pdbm = [float(v) for v in phys]
    if cr is not None:
        crv = cr
    ptot = 1e-3 * 10.0 ** (pdbm / 10.0)
    alpha = _alpha_lin(adb)
    le = _leff(alpha, L)
    m = _mu(_span(L, adb, b2, b3, crv), ptot, B_TOT, a, b, c, method="segment", dz=1.0)
    e6 = _mu(_span(L, adb, b2, b3, 0.0), ptot, B_TOT, a, b, c, method="maclaurin")
    return np.log(abs(m) ** 2 / le ** 2), np.log(abs(e6) ** 2 / le ** 2)


def init_like(seed, hidden=256, nin=NIN):
    """Seeded He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    lay, n = layout(hidden, nin)
    p = np.zeros(n)
    for name, (o, s) in lay.items():
        if name.startswith("W") or name == "w5":
            fan_in = nin if name == "W1" else hidden
            lim = np.sqrt(6.0 / fan_in)
            w = rng.uniform(-lim, lim, size=s)
            p[o:o + w.size] = w.reshape(-1)
    return p
