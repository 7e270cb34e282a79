"""Pins of the CPU reference of the surrogate: its gradient against central
differences, its target's composition against Eq. 6, the feature box."""
import numpy as np
import pytest

import oracle
from oracle import surrogate as S


def _fd_check(hidden, n_rows, coords, seed, h=1e-6, tol=1e-6):
    rng = np.random.default_rng(seed)
    p = S.init_like(seed, hidden=hidden)
    p += 0.05 * rng.standard_normal(p.size)       # non-zero biases and padding rows too
    x = rng.uniform(-1, 1, size=(n_rows, S.NIN))
    r = rng.standard_normal(n_rows)
    _, g = S.loss_and_grad(p, x, r, hidden)
    for i in coords:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (S.loss_and_grad(pp, x, r, hidden)[0] - S.loss_and_grad(pm, x, r, hidden)[0]) / (2 * h)
        assert abs(fd - g[i]) <= tol * max(1.0, abs(fd)), (i, fd, g[i])


def test_gradient_small_network_all_coordinates():
    _, n = S.layout(hidden=6)
    _fd_check(hidden=6, n_rows=7, coords=range(n), seed=1)


def test_gradient_full_network_sampled_coordinates():
    lay, n = S.layout()
    rng = np.random.default_rng(2)
    coords = []
    for name, (o, s) in lay.items():       # a few coordinates of every tensor
        k = int(np.prod(s))
        coords += list(o + rng.choice(k, size=min(k, 3), replace=False))
    _fd_check(hidden=256, n_rows=5, coords=coords, seed=3, h=1e-5, tol=2e-6)


def test_loss_is_mean_squared_error():
    rng = np.random.default_rng(4)
    p = S.init_like(4, hidden=8)
    x = rng.uniform(-1, 1, size=(9, S.NIN))
    r = rng.standard_normal(9)
    loss, _ = S.loss_and_grad(p, x, r, hidden=8)
    assert np.isclose(loss, np.mean((S.forward(p, x, hidden=8) - r) ** 2), rtol=1e-14)


def test_silu_derivative():
    z = np.linspace(-8, 8, 33)
    s = 1 / (1 + np.exp(-z))
    h = 1e-6
    fd = (S.silu(z + h) - S.silu(z - h)) / (2 * h)
    assert np.allclose(fd, s * (1 + z * (1 - s)), atol=1e-8)


def test_constant_network():
    """Zero weights: every output is b5; the gradient is d/db5 only."""
    p = np.zeros(S.layout(hidden=8)[1])
    p[-1] = 0.75
    x = np.random.default_rng(5).uniform(-1, 1, size=(4, S.NIN))
    r = np.array([0.0, 1.0, 2.0, 3.0])
    assert np.allclose(S.forward(p, x, hidden=8), 0.75)
    loss, g = S.loss_and_grad(p, x, r, hidden=8)
    assert np.isclose(loss, np.mean((0.75 - r) ** 2))
    assert np.isclose(g[-1], 2 * np.mean(0.75 - r))
    # silu(0) = 0 hides every earlier weight from the output except through b_l
    lay, _ = S.layout(hidden=8)
    assert np.all(g[lay["w5"][0]:lay["w5"][0] + 8] == 0)


def test_target_without_raman_is_eq6():
    """With Cr = 0 every segment gain is 1 and the segment sum of Eq. 9 is a
    geometric series equal to Eq. 6, so y = y6."""
    rng = np.random.default_rng(6)
    for _ in range(8):
        x = rng.uniform(-1, 1, size=(1, S.NIN))
        phys = S.decode(x)[0]
        y, y6 = S.target(phys, cr=0.0)
        assert abs(y - y6) <= 1e-9 * max(1.0, abs(y6)), (phys, y, y6)


def test_target_raman_tilt_sign():
    """ISRS moves power to low frequencies: at chi = 0 (f1 = f), a product
    frequency far below the band centre sees more gain than one far above."""
    base = [0.0, 0.0, 0.0, 90.0, 0.2, -21.7, 0.14, 0.028, 21.0]
    lo, hi = list(base), list(base)
    lo[0], lo[1], lo[2] = -4.0, -4.0, -4.0     # f1 + f2 - f = -4 THz
    hi[0], hi[1], hi[2] = 4.0, 4.0, 4.0
    ylo, y6lo = S.target(lo)
    yhi, y6hi = S.target(hi)
    assert abs(y6lo) < 1e-12 and abs(y6hi) < 1e-12     # chi = 0: |eta| = L_eff
    assert ylo > 0.0 > yhi


def test_feature_box_roundtrip():
    rng = np.random.default_rng(7)
    phys = S.BOX_LO + rng.uniform(size=(5, S.NF)) * (S.BOX_HI - S.BOX_LO)
    x = S.encode(phys)
    assert np.all(np.abs(x[:, :S.NF]) <= 1) and np.all(x[:, S.NF:] == 0)
    assert np.allclose(S.decode(x), phys, rtol=0, atol=1e-12)


def test_layout_size_matches_library_constant():
    assert S.layout()[1] == 201_985


def test_features():
    rng = np.random.default_rng(8)
    x = rng.uniform(-1, 1, size=(64, S.NIN)).astype(np.float32)
    f = S.features(x)
    assert np.array_equal(f[:, :S.NF], x[:, :S.NF].astype(np.float64))
    assert np.allclose(f[:, 9] ** 2 + f[:, 10] ** 2, 1.0) and np.allclose(f[:, 14] ** 2 + f[:, 15] ** 2, 1.0)
    assert np.allclose(f[:, 12] ** 2 + f[:, 13] ** 2, 1.0) and np.all(f[:, 12] > 0)
    # f1 = f: chi = 0, so the phases vanish and |beta| = alpha
    phys = S.decode(x[:1])[0]
    phys[0] = phys[2]
    g = S.features(S.encode(phys))[0]
    assert np.allclose(g[9:], [1.0, 0.0, -1.0, 1.0, 0.0, 1.0, 0.0], atol=1e-12)
    # chi is Eq. 24's coefficient, as the oracle forms it
    p = S.decode(x[1:2])[0]
    chi = oracle.phase_coef(p[5], p[6], p[0], p[1], p[2])
    alpha = oracle.alpha_lin(p[4])
    assert np.isclose(f[1, 13], chi / np.hypot(alpha, chi), rtol=1e-12)
