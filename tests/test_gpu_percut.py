"""GPU parity per CUT (Eqs. 11 and 15) at the benchmark workloads' sizes,
against FP64 oracle values stored by tests/golden/gen_oracle_percut.py (which
calls only the oracle):

  * C+L 100 ch, 10 spans: every CUT at 64 x 64 (integral form), CUTs 0/49/99
    at 64 x 64 (segment form) and at 256 x 256 (integral form);
  * S+C+L 150 ch, 40 spans: 4 seeded CUTs at 64 x 64 and CUTs 0/75 at
    128 x 128 (integral form), and every near-CUT square of four CUTs at
    1024 x 1024 (island level);
  * the far end of the 512-link batch's cost distribution (the most spans,
    the most channels) at 64 x 64, through the batched launch.

Bars: the FP64 path against the segment form 1e-9 dB per CUT (the same
method, different code); every path (FP64, FP32 integrand with FP64 phase)
against the integral form (the model the closed forms approximate) 0.01 dB
per CUT; at the island level the GPU integral form against the oracle's
adaptive integral 1e-6 relative.
"""
import json
import os

import numpy as np
import pytest

from paper_2412_11614_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64 = W.PREC_FP64
FP32 = W.PREC_FP32_PHASE64
HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def gold(stage):
    path = os.path.join(HERE, f"oracle_percut_{stage}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)


def db(x, ref):
    return 10.0 * np.log10(np.asarray(x) / np.asarray(ref))


@pytest.fixture(scope="module")
def engine():
    import torch
    assert torch.cuda.is_available()
    from paper_2412_11614_amd import _lib
    e = _lib.Engine(0)
    yield e
    e.close()


def _eta_paths(engine, wl, cuts, n_grid):
    engine.load(wl)
    return {prec: engine.eval_eta(wl.numerics, cuts, precision=prec, n=n_grid) for prec in (FP64, FP32)}


@pytest.mark.parametrize("stage,make", [
    ("cl64", lambda: W.cl_100ch_10span(n_grid=64)),
    ("cl256", lambda: W.cl_100ch_10span(n_grid=256)),
    ("scl64", lambda: W.sclband_150ch_40span(n_grid=64)),
    ("scl128", lambda: W.sclband_150ch_40span(n_grid=128)),
])
def test_eta_against_integral_form(engine, stage, make):
    g = gold(stage)
    assert g["method"] == "integral"
    cuts = np.array(g["cuts"], dtype=np.int32)
    ref = np.array(g["eta"])
    out = _eta_paths(engine, make(), cuts, g["n_grid"])
    for prec, r in out.items():
        err = np.abs(db(r["eta"], ref))
        print(f"{stage} precision {prec}: {len(cuts)} CUTs, max |dB| vs the integral form {err.max():.2e} "
              f"(CUT {cuts[err.argmax()]})", flush=True)
        assert err.max() <= 0.01, (prec, cuts[err.argmax()], err.max())
        # the five terms of Eq. 15 add up to sigma^2 on both sides
        assert np.allclose(r["terms"].sum(axis=1), r["sigma2"], rtol=1e-12)
    # the two precisions of the GPU agree more closely than either meets the bar
    assert np.max(np.abs(db(out[FP32]["eta"], out[FP64]["eta"]))) <= 2e-3


def test_eta_against_segment_form_64(engine):
    g = gold("cl64seg")
    assert g["method"] == "segment"
    cuts = np.array(g["cuts"], dtype=np.int32)
    wl = W.cl_100ch_10span(n_grid=64)
    engine.load(wl)
    r = engine.eval_eta(wl.numerics, cuts, precision=FP64, n=64)
    err = np.abs(db(r["eta"], g["eta"]))
    print("C+L 64 x 64 FP64 vs the segment form: max |dB|", err.max(), flush=True)
    assert err.max() <= 1e-9
    ref_terms = np.array(g["terms"])
    s2 = np.array(g["sigma2"])
    assert np.all(np.abs(r["terms"] - ref_terms) <= 1e-9 * s2[:, None]), (r["terms"], ref_terms)


def test_near_cut_squares_1024(engine):
    g = gold("scl1024sq")
    wl = W.sclband_150ch_40span(n_grid=1024)
    engine.load(wl)
    by_cut = {}
    for e in g["squares"]:
        by_cut.setdefault(e["cut"], []).append(e)
    for cut, ents in sorted(by_cut.items()):
        keys = [(e["k1"], e["k2"]) for e in ents]
        ref = np.array([e["terms"] for e in ents])                   # [m][3][5]
        print(f"S+C+L 1024 x 1024: CUT {cut}, {len(keys)} near-CUT squares", flush=True)
        gint = engine.eval_islands(wl.numerics, cut, keys, precision=FP64, mu_method=2, dz=0.25)
        scale = np.abs(ref).max()
        assert np.allclose(gint, ref, rtol=1e-6, atol=1e-9 * scale), cut
        tot = ref[:, :, 0].sum()
        for prec in (FP64, FP32):
            seg = engine.eval_islands(wl.numerics, cut, keys, precision=prec)
            # the CUT's GN sum over its near squares, and no island off by more than that share
            assert abs(db(seg[:, :, 0].sum(), tot)) <= 0.01, (cut, prec)
            assert np.all(np.abs(seg[:, :, 0] - ref[:, :, 0]) <= (10 ** 0.001 - 1) * tot), (cut, prec)


def test_batch_extreme_links(engine):
    g = gold("batchx")
    links = W.batch_links()
    nu = links[0].numerics
    b = engine.batch(links)
    eta32 = b.eval(nu, precision=FP32)
    off = b.cut_offset
    b.close()
    for rec in g["links"]:
        i = rec["link"]
        w = links[i]
        assert len(w.link.spans) == rec["n_spans"] and len(w.cuts) == rec["n_active"]
        pos = np.searchsorted(w.cuts, rec["cuts"])
        assert np.array_equal(w.cuts[pos], rec["cuts"])
        err = np.abs(db(eta32[off[i]:off[i + 1]][pos], rec["eta"]))
        print(f"batch link {i} ({rec['n_active']} ch, {rec['n_spans']} spans): batched FP32 max |dB| {err.max():.2e}",
              flush=True)
        assert err.max() <= 0.01, i
        engine.load(w)
        r64 = engine.eval_eta(nu, np.array(rec["cuts"], dtype=np.int32), precision=FP64)
        assert np.max(np.abs(db(r64["eta"], rec["eta"]))) <= 0.01, i
