"""Host-side pieces of bench.py: the roofline arithmetic of a region launch and
the gating of committed counter summaries on the kernel source they were
taken from.  No GPU is used."""
import importlib.util
import os
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _stats(horner_steps, point_spans, region_ms, launches=1):
    # the library's counters: alg_flop prices a segment at 8 FLOP (complex Horner) plus 30 per point-span
    return types.SimpleNamespace(horner_steps=horner_steps, alg_flop=8.0 * horner_steps + 30.0 * point_spans,
                                 region_ms=region_ms, region_launches=launches)


def test_roofline_counts_two_fmas_per_segment(bench, monkeypatch):
    monkeypatch.setattr(bench, "profile_fields", lambda stem: {})
    # 1e12 point-spans of K = 80 segments: (4 * 80 + 30) FLOP each, in 2 launches of 1 s
    st = _stats(horner_steps=80 * 10**12, point_spans=10**12, region_ms=2000.0, launches=2)
    r = bench.kernel_roofline(st, 78.6432, "k", "none")
    assert r["flop_per_launch"] == pytest.approx(350e12 / 2)
    assert r["achieved"] == pytest.approx(175.0)
    assert r["frac"] == pytest.approx(175.0 / 78.6432)
    assert r["traffic"] is None and "frac_counter" not in r
    # the complex-Horner count is the same work priced at 8 FLOP per segment
    assert r["frac_complex_horner_count"] == pytest.approx((8 * 80 + 30) * 1e12 / 2 / 78.6432 / 1e12)


def test_profile_fields_follow_the_kernel_source(bench, tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    good = bench.kernel_source_hash()
    (tmp_path / "k_traffic.md").write_text(f"# t\n\ntraffic_bytes_per_launch: 1.5e+09\nkernel_source_sha256: {good}\n")
    (tmp_path / "k_counters.md").write_text("| a | b |\n\nfma_flop_per_s_frac: 0.5\nkernel_source_sha256: 0000\n")
    f = bench.profile_fields("k")
    assert f["traffic_bytes_per_launch"] == "1.5e+09"
    assert "fma_flop_per_s_frac" not in f          # taken from another kernel source: ignored
    st = _stats(horner_steps=8, point_spans=1, region_ms=1.0)
    r = bench.kernel_roofline(st, 1.0, "k", "k")
    assert r["traffic"] == 1.5e9 and "frac_counter" not in r
