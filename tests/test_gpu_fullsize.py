"""GPU parity at the benchmark sizes, on sampled outputs, against FP64 oracle
values stored by tests/golden/gen_oracle_fullsize.py (which calls only the
oracle):

  * C+L 100 ch, 10 spans, 256 x 256 per square: bare island integrals of
    squares near and far from CUTs 0, 49, 99;
  * S+C+L 150 ch, 40 spans, 1024 x 1024 per square: squares of CUTs 0 and 75;
  * the 512-link batch at 64 x 64 (the launch the benchmark times): eta of
    every CUT of two links.

Bars: FP64 path vs the segment form 1e-9 relative; the integral form
(dz 0.25 km) vs the oracle's integral 1e-6 relative; FP32-integrand path vs the
segment form 1e-3 relative per nonzero integral (0.004 dB); every path vs
the integral form within 0.01 dB on D and on eta.
"""
import json
import os

import numpy as np
import pytest

from paper_2412_11614_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64 = W.PREC_FP64
FP32 = W.PREC_FP32_PHASE64
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_fullsize.json")


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def engine():
    import torch
    assert torch.cuda.is_available()
    from paper_2412_11614_amd import _lib
    e = _lib.Engine(0)
    yield e
    e.close()


def _by_square(entries):
    out = {}
    for e in entries:
        out.setdefault((e["cut"], e["k1"], e["k2"]), {})[e["method"]] = np.array(e["terms"])
    return out


def _check_squares(engine, wl, entries, label):
    engine.load(wl)
    sq = _by_square(entries)
    cuts = sorted({c for c, _, _ in sq})
    for cut in cuts:
        keys = [(k1, k2) for c, k1, k2 in sq if c == cut]
        print(f"{label}: CUT {cut}, squares {keys}", flush=True)
        g64 = engine.eval_islands(wl.numerics, cut, keys, precision=FP64)
        g32 = engine.eval_islands(wl.numerics, cut, keys, precision=FP32)
        gint = engine.eval_islands(wl.numerics, cut, keys, precision=FP64, mu_method=2, dz=0.25)
        for (k1, k2), a64, a32, ai in zip(keys, g64, g32, gint):
            seg = sq[(cut, k1, k2)]["segment"]
            integ = sq[(cut, k1, k2)]["integral"]
            scale = np.abs(seg).max() + 1e-300
            assert np.allclose(a64, seg, rtol=1e-9, atol=1e-12 * scale), (cut, k1, k2, a64, seg)
            # the GPU integral form against the oracle's adaptive integral
            assert np.allclose(ai, integ, rtol=1e-6, atol=1e-9 * scale), (cut, k1, k2, ai, integ)
            nz = np.abs(seg) > 1e-9 * scale
            if not nz.any():                      # no island of this square reaches the CUT
                assert np.all(a32 == 0.0), (cut, k1, k2)
                continue
            rel32 = np.abs(a32[nz] - seg[nz]) / np.abs(seg[nz])
            assert rel32.max() <= 1e-3, (cut, k1, k2, rel32.max())
            # near-CUT squares (which carry the CUT's eta) against the integral form
            # (the model): 0.01 dB on the square's D, and no island off by more than
            # that share of the total.  The segment form's relative error grows with
            # chi, so far squares (D ~1e-11 of the CUT's) and small side islands
            # exceed it, while their share of eta does not; the GPU's parity with
            # the segment form above holds on every square.
            tot = integ[:, 0].sum()
            if tot > 0 and abs(k1 - cut) <= 2 and abs(k2 - cut) <= 2:
                for a in (a64, a32):
                    assert abs(10 * np.log10(a[:, 0].sum() / tot)) <= 0.01, (cut, k1, k2)
                    assert np.all(np.abs(a[:, 0] - integ[:, 0]) <= (10 ** 0.001 - 1) * tot), (cut, k1, k2)


def test_cl_100ch_10span_256_sampled_squares(engine, gold):
    _check_squares(engine, W.cl_100ch_10span(n_grid=256), gold["cl_100ch_10span_256"]["squares"], "C+L")


def test_sclband_150ch_40span_1024_sampled_squares(engine, gold):
    _check_squares(engine, W.sclband_150ch_40span(n_grid=1024), gold["sclband_150ch_40span_1024"]["squares"],
                   "S+C+L")


def test_batch_512_links_sampled_links(engine, gold):
    links = W.batch_links()
    nu = links[0].numerics
    b = engine.batch(links)
    print(f"batch: {b.n_cuts} CUTs", flush=True)
    eta32 = b.eval(nu, precision=FP32)
    off = b.cut_offset
    for rec in gold["batch_links_64"]["links"]:
        i = rec["link"]
        assert list(links[i].cuts) == rec["cuts"]
        ref = np.array(rec["eta"])
        got = eta32[off[i]:off[i + 1]]
        assert np.max(np.abs(10 * np.log10(got / ref))) <= 0.01, i
    b.close()
    # the same links alone through the FP64 path: the method's value to 1e-9 dB
    for rec in gold["batch_links_64"]["links"]:
        w = links[rec["link"]]
        engine.load(w)
        got = engine.eval_eta(nu, w.cuts, precision=FP64)["eta"]
        assert np.max(np.abs(10 * np.log10(got / np.array(rec["eta"])))) <= 1e-9
