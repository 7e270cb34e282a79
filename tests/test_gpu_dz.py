"""Per-CUT sampling step (the segment form's step following the COI) and the
error-model step choice."""
import numpy as np
import pytest

import oracle
from paper_2412_11614_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64 = W.PREC_FP64
FP32 = W.PREC_FP32_PHASE64


@pytest.fixture(scope="module")
def engine():
    import torch
    assert torch.cuda.is_available()
    from paper_2412_11614_amd import _lib
    e = _lib.Engine(0)
    yield e
    e.close()


def test_per_cut_step_matches_single_step_runs(engine):
    wl = W.small_mixed(seed=41, n_ch=7, n_spans=3, n_grid=24)
    engine.load(wl)
    cuts = wl.cuts
    dz = np.array([0.5, 2.0, 1.0, 2.0, 0.5, 3.0, 1.0][:len(cuts)])
    got = engine.eval_eta_dz(wl.numerics, cuts, dz, precision=FP64)
    for q, c in enumerate(cuts):
        one = engine.eval_eta(wl.numerics, [c], precision=FP64, dz=float(dz[q]))
        assert np.allclose(got["eta"][q], one["eta"][0], rtol=1e-13, atol=0), q
        assert np.allclose(got["terms"][q], one["terms"][0], rtol=1e-12, atol=1e-300), q
        nu = W.Numerics(**{**wl.numerics.__dict__, "dz_km": float(dz[q])})
        ref = oracle.eval_cuts(wl, cuts=[c], method="segment", numerics=nu)["eta"][0]
        assert abs(10 * np.log10(got["eta"][q] / ref)) <= 1e-9, q
    # equal steps: the plain path
    same = engine.eval_eta_dz(wl.numerics, cuts, np.full(len(cuts), 1.0), precision=FP64)
    plain = engine.eval_eta(wl.numerics, cuts, precision=FP64, dz=1.0)
    assert np.array_equal(same["eta"], plain["eta"])


def test_per_cut_step_rejects_bad_steps(engine):
    from paper_2412_11614_amd import _lib
    wl = W.small_mixed(seed=42, n_ch=5, n_spans=1, n_grid=16)
    engine.load(wl)
    with pytest.raises(_lib.IsrsError) as ei:
        engine.eval_eta_dz(wl.numerics, wl.cuts[:2], [1.0, -1.0])
    assert ei.value.code == _lib.ISRS_E_ARG and "CUT 1" in str(ei.value)


def test_error_model_step_choice(engine):
    """On the C+L link (coarse grid), the chosen steps meet the target against
    the finest step, grow toward the band centre where the segment form's
    error is least sensitive to the step, and speed up the evaluation."""
    import time
    wl = W.cl_100ch_10span(n_grid=32)
    engine.load(wl)
    cuts = np.arange(0, 100, 3, dtype=np.int32)
    cand = [0.5, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0]
    dz, err = engine.choose_dz(wl.numerics, cuts, cand, 0.005, precision=FP64)
    print("chosen dz", dz, flush=True)
    assert np.all(np.isin(dz, cand))
    got = engine.eval_eta_dz(wl.numerics, cuts, dz, precision=FP64)["eta"]
    ref = engine.eval_eta(wl.numerics, cuts, precision=FP64, dz=0.5)["eta"]
    assert np.max(np.abs(10 * np.log10(got / ref))) <= 0.005
    centre = np.abs(cuts - 49.5) < 15
    edge = np.abs(cuts - 49.5) > 40
    assert dz[centre].mean() >= dz[edge].mean()
