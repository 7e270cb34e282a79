"""GPU: the allocation-free entry point (isrs_eval_eta_dev_noalloc) through the
C-ABI against isrs_eval_eta_dev, the entry point it is a variant of.

Both run the same kernels on the same plan; every square is summed by one
block in a fixed order and the per-CUT assembly is a fixed tree, so the
outputs must agree bit for bit whatever number of persistent blocks the
scratch leaves room for.  Two calls in a row, the second smaller, check that
the shared scratch keeps no state that a later call depends on; a plan too
large for the scratch is refused before any launch.
"""
import numpy as np
import pytest

import oracle
from paper_2412_11614_amd import workloads as W

pytestmark = pytest.mark.gpu


def _cases():
    big = W.small_mixed(n_ch=9, n_spans=3, n_grid=40, precision=W.PREC_FP64)
    small = W.small_mixed(seed=5, n_ch=5, n_spans=2, n_grid=12, precision=W.PREC_FP32_PHASE64)
    return [(big, big.cuts), (small, small.cuts[:2])]


def test_noalloc_matches_eval_eta_dev():
    import torch
    from paper_2412_11614_amd import _lib
    assert torch.cuda.is_available()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st), _lib.Engine(0, stream=st) as eng:
        for wl, cuts in _cases():
            print(f"case {wl.name} n_ch={wl.spectrum.n_ch} grid={wl.numerics.n_grid} cuts={list(cuts)}", flush=True)
            eng.load(wl)
            n = len(cuts)
            outs = []
            for noalloc in (False, True):
                eta = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
                s2 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
                terms = torch.full((n * 5,), float("nan"), dtype=torch.float64, device="cuda")
                eng.eval_eta_dev(wl.numerics, cuts, eta, s2, terms, noalloc=noalloc)
                st.synchronize()
                outs.append((eta.cpu().numpy(), s2.cpu().numpy(), terms.cpu().numpy()))
            for ref, got in zip(outs[0], outs[1]):
                assert np.all(np.isfinite(got))
                assert np.array_equal(ref, got), (ref, got)
            # the E/F/G/H terms are exercised (mixed formats)
            assert np.any(outs[1][2].reshape(n, 5)[:, 1:] != 0.0)
            if wl.numerics.precision == W.PREC_FP64:
                seg = oracle.eval_cuts(wl, cuts=cuts, method="segment")
                err = np.abs(10 * np.log10(outs[1][0] / seg["eta"]))
                print("max |dB| vs the oracle's segment form", err.max(), flush=True)
                assert err.max() <= 1e-9


def test_noalloc_back_to_back_and_too_large():
    import torch
    from paper_2412_11614_amd import _lib
    st = torch.cuda.Stream()
    with torch.cuda.stream(st), _lib.Engine(0, stream=st) as eng:
        (big, cb), (small, cs) = _cases()
        res = {}
        # reference values from the allocating entry point
        for key, wl, cuts in (("big", big, cb), ("small", small, cs)):
            eng.load(wl)
            eta = torch.empty(len(cuts), dtype=torch.float64, device="cuda")
            eng.eval_eta_dev(wl.numerics, cuts, eta)
            st.synchronize()
            res[key] = eta.cpu().numpy()
        # two allocation-free calls queued on the stream with no host wait between
        eng.load(big)
        e1 = torch.empty(len(cb), dtype=torch.float64, device="cuda")
        eng.eval_eta_dev(big.numerics, cb, e1, noalloc=True)
        e2 = torch.empty(len(cb), dtype=torch.float64, device="cuda")
        small_big_link = cb[:3]
        eng.eval_eta_dev(big.numerics, small_big_link, e2[:3], noalloc=True, n=16)
        st.synchronize()
        assert np.array_equal(e1.cpu().numpy(), res["big"])
        eta16 = torch.empty(3, dtype=torch.float64, device="cuda")
        eng.eval_eta_dev(big.numerics, small_big_link, eta16, n=16)
        st.synchronize()
        assert np.array_equal(e2[:3].cpu().numpy(), eta16.cpu().numpy())
        # a plan larger than the scratch array is refused before any launch
        out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        with pytest.raises(_lib.IsrsError) as ei:
            eng.eval_eta_dev(big.numerics, cb[:1], out, noalloc=True, n=8192)
        assert ei.value.code == _lib.ISRS_E_ARG
        assert "bytes of device scratch" in str(ei.value)
        st.synchronize()
        assert out.item() == -1.0
