"""Throughput of the ISRS-EGN hot path on one MI355X.

One step = one pass of the whole hot path (segment tables, island work list,
the region kernel over every folded channel-pair square with the coherent
E/F/G/H sums on its tile, the per-CUT assembly of Eq. 15 and eta of Eq. 11)
for one CUT of the S+C+L workload: 150 x 100 GBd channels on a 100 GHz grid
(15 THz), 24 dBm, 40 spans of 80 km with per-span fibre draws, 1024 x 1024
grid per square, everything in FP64.  The timed steps take CUTs spread evenly
over the band (step i: CUT round((i + 1/2) 150 / K - 1/2)); the whole band is
150 such steps, so CUT/s of the sample is the rate of the 150-CUT job.
Inputs are resident on the GPU when the timed region starts; outputs stay on
the GPU.

Prints one JSON line.  The CPU-baseline leg times the FP64 oracle (integral
form of the z-integral) on a bounded sample of the same workload; the
accuracy block compares GPU results with stored oracle values
(tests/golden/, written by scripts that call only the oracle).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Vector ALU peaks of the chip: 256 CU x 4 SIMD x 16 lanes x 2 FLOP (FMA) x 2.4 GHz
# = 78.6 TFLOP/s in FP64, twice that (157.3) in FP32.  gfx950 issues non-packed
# v_fma_f32 at up to ~1.9 wave-instructions per CU per clock (149 TFLOP/s measured
# on independent chains), so 157.3 is also the ceiling of a build without packed
# FP32.
PEAK_FP64_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_FP32_TFLOPS = 2 * PEAK_FP64_TFLOPS
GOLDEN = os.path.join(ROOT, "tests", "golden")
PROFILES = os.path.join(ROOT, "profiles")
HEADLINE_PROFILE = "region_queue_kernel_fp64_scl150ch_40span_1024"
CL_PROFILE = "region_queue_kernel_fp32_cl100ch_10span_256"
BATCH_PROFILE = "region_queue_kernel_fp32_batch512_64"


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("isrs_kernels.hip", "isrs_internal.h"):
        with open(os.path.join(ROOT, "paper_2412_11614_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profile_fields(stem):
    """key: value lines of a committed counter summary, or {} when the kernel
    source has changed since the counters were taken."""
    out = {}
    for kind in ("traffic", "counters"):
        try:
            text = open(os.path.join(PROFILES, f"{stem}_{kind}.md")).read()
        except OSError:
            continue
        fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and
                      line.split(": ", 1)[0].replace("_", "").isalnum() and not line.startswith(("|", "*", "#")))
        if fields.get("kernel_source_sha256", "").strip() != kernel_source_hash():
            continue
        out.update({k: v.strip() for k, v in fields.items()})
    return out


def kernel_roofline(st, peak, name, stem):
    """Roofline of one region launch from the library's counters and HIP-event
    time: algorithmic FLOP of the segment method as evaluated, 4 K_s + 30 per
    live (point, span) (two FMAs per segment of the real-coefficient sum, plus
    the per-point setup: q, I_0, the rotation e^{i Theta}, the accumulation)."""
    per_launch_ms = st.region_ms / max(1, st.region_launches)
    point_spans = (st.alg_flop - 8.0 * st.horner_steps) / 30.0
    flop = (4.0 * st.horner_steps + 30.0 * point_spans) / max(1, st.region_launches)
    achieved = flop / (per_launch_ms * 1e-3) / 1e12
    prof = profile_fields(stem)
    traffic = float(prof["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in prof else None
    r = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
         "traffic": traffic, "kernel": name, "per_launch_ms": per_launch_ms, "flop_per_launch": flop,
         "flop_per_unit": "4 K_s + 30 per live (point, span)",
         # the complex-Horner count (8 K_s + 30) prices each segment at twice what the
         # real-coefficient recurrence needs; as a fraction it can pass 1
         "frac_complex_horner_count": st.alg_flop / max(1, st.region_launches) / (per_launch_ms * 1e-3) / 1e12 / peak}
    if "fma_flop_per_s_frac" in prof:
        r["frac_counter"] = float(prof["fma_flop_per_s_frac"])
    return r


def _plain(o):
    """JSON form of numpy scalars and arrays left in a result."""
    if isinstance(o, np.generic):
        return o.item()
    if isinstance(o, np.ndarray):
        return o.tolist()
    raise TypeError(f"not JSON serializable: {type(o).__name__}")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(wl, n_squares, seed=0):
    """Times the oracle (integral-form FWM factor, FP64) on n_squares randomly
    drawn live channel-pair squares of the middle CUT at the full grid, using
    all host cores (one square per thread), and scales to CUTs per second by
    the CUT's number of live squares (unfolded, as the oracle evaluates them)."""
    import concurrent.futures as cf

    import oracle

    oracle.lib()
    sp = wl.spectrum
    nc = sp.n_ch
    cut = nc // 2
    act = sp.power_w > 0
    live = []
    for k1 in range(nc):
        for k2 in range(nc):
            if not (act[k1] and act[k2]):
                continue
            if any(0 <= k1 + k2 - cut + l < nc and act[k1 + k2 - cut + l] for l in (-1, 0, 1)):
                live.append((k1, k2))
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    n_squares = n_squares or min(cores, 16)
    rng = np.random.default_rng(seed)
    pick = [live[i] for i in rng.choice(len(live), size=n_squares, replace=False)]
    threads = max(1, min(cores, n_squares))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda kk: oracle.square_terms(wl, cut, kk[0], kk[1], method="integral"), pick))
    wall = time.perf_counter() - t0
    cut_seconds = wall / n_squares * len(live)
    return {"value": 1.0 / cut_seconds, "unit": "CUT/s", "cores": threads, "kind": "oracle",
            "sample": (f"{n_squares} random live squares of CUT {cut} (of {len(live)}) at the full "
                       f"{wl.numerics.n_grid}x{wl.numerics.n_grid} grid, {len(wl.link.spans)} spans, "
                       f"integral-form mu; {wall:.1f} s wall on {threads} threads, scaled by squares per CUT")}


def batched_leg(eng, n_links, n_plain, W, torch, tune_links=32):
    """Uneven-link workload in one persistent queue launch, replayed from a
    captured graph, with the launch shape from the project's autotuner (tuned
    on the batch's first tune_links links, whose shape key the full batch
    shares, through the tuning cache), against the default shape and the plain
    one-link-at-a-time path."""
    import tempfile

    links = W.batch_links(n_links=n_links)
    nu = links[0].numerics                       # 64 x 64, FP32 integrand / FP64 phase
    cache = os.path.join(tempfile.mkdtemp(prefix="isrs_tune_"), "autotune.jsonl")
    t0 = time.perf_counter()
    bt = eng.batch(links[:min(tune_links, n_links)])
    bt.autotune(nu, cache)
    bt.close()
    t_tune = time.perf_counter() - t0
    b = eng.batch(links)
    eta_b = torch.empty(b.n_cuts, dtype=torch.float64, device="cuda")

    def timed_replay():
        eng.set_profiling(True)                  # the eager first call reports the work done
        t0 = time.perf_counter()
        b.eval_dev(nu, eta_b)
        torch.cuda.synchronize()
        t_first = time.perf_counter() - t0
        st = eng.stats()
        eng.set_profiling(False)
        b.eval_dev(nu, eta_b)                    # capture the graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.eval_dev(nu, eta_b)                    # timed replay
        torch.cuda.synchronize()
        return time.perf_counter() - t0, t_first, st

    log(f"batched: {n_links} links, {b.n_cuts} CUTs, default launch shape")
    t_default, t_first, st_default = timed_replay()
    shape_default = b.tuning()
    eta_default = eta_b.cpu().numpy().copy()
    b.autotune(nu, cache)                        # cache hit: re-plans with the tuned shape
    log(f"batched: tuned shape {b.tuning()}")
    t_batch, _, st = timed_replay()
    shape_tuned = b.tuning()
    eta_batch = eta_b.cpu().numpy()
    # plain path on the first n_plain links, same numerics
    n_plain = min(n_plain, n_links)
    off = b.cut_offset
    cuts_plain = int(off[n_plain])
    eta_plain = torch.empty(max(1, max(len(w.cuts) for w in links[:n_plain])), dtype=torch.float64, device="cuda")
    agree = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, w in enumerate(links[:n_plain]):
        eng.load(w)
        eng.eval_eta_dev(nu, w.cuts, eta_plain)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for i, w in enumerate(links[:n_plain]):
        eng.load(w)
        eng.eval_eta_dev(nu, w.cuts, eta_plain)
        torch.cuda.synchronize()
        ref = eta_plain[:len(w.cuts)].cpu().numpy()
        agree = max(agree, float(np.max(np.abs(10 * np.log10(eta_batch[off[i]:off[i + 1]] / ref)))))
    b.close()
    per_launch_s = st.region_ms * 1e-3 / max(1, st.region_launches)
    point_spans = (st.alg_flop - 8.0 * st.horner_steps) / 30.0
    flop = 4.0 * st.horner_steps + 30.0 * point_spans
    return {"workload": (f"{n_links} links: 20-100 active of 100 x 96 GBd / 100 GHz slots, P U[-3,3] dBm, "
                         f"1-30 spans U[50,120] km, alpha and Cr per link (seed 3), 64x64 per square, "
                         f"all active channels under test"),
            "n_cut": int(b.n_cuts), "value": b.n_cuts / t_batch, "unit": "CUT/s",
            "ms_per_step": 1e3 * t_batch, "first_call_s": t_first,
            "tuned_shape": shape_tuned, "default_shape": shape_default, "default_ms_per_step": 1e3 * t_default,
            "tuning_s": t_tune, "tuned_on_links": min(tune_links, n_links),
            "max_abs_db_tuned_vs_default": float(np.max(np.abs(10 * np.log10(eta_batch / eta_default)))),
            "region_launches": st.region_launches,
            "plain_path": {"links": n_plain, "n_cut": cuts_plain, "value": cuts_plain / t_plain, "unit": "CUT/s"},
            "speedup_vs_plain": (b.n_cuts / t_batch) / (cuts_plain / t_plain),
            "max_abs_db_batch_vs_plain": agree,
            # FLOP of the segment method as evaluated (4 K + 30 per live point-span) per region
            # launch over its HIP-event time, against the FP32 vector peak
            "tflops": flop / max(1, st.region_launches) / per_launch_s / 1e12,
            "frac": flop / max(1, st.region_launches) / per_launch_s / 1e12 / PEAK_FP32_TFLOPS,
            "region_ms_eager": st.region_ms, "live_points": st.n_points_live,
            "default_region_ms_eager": st_default.region_ms,
            # executed FMA rate and HBM bytes per launch from the committed counter
            # summaries of this launch (absent once the kernel source has changed)
            **{k: float(v) for k, v in profile_fields(BATCH_PROFILE).items()
               if k in ("fma_flop_per_s_frac", "traffic_bytes_per_launch")}}


def integral_form_leg(eng, wl, W, torch, n_cuts=10):
    """The model's integral form (Eq. 23, 4-node product integration per 1 km
    segment, FP64) against the closed forms on the same CUTs: the GPU
    counterpart of the paper's integral vs closed-form time comparison."""
    cuts = np.linspace(0, len(wl.cuts) - 1, n_cuts).astype(np.int32)
    eng.load(wl)
    res = {"workload": f"{n_cuts} CUTs of the benchmark link at {wl.numerics.n_grid}x{wl.numerics.n_grid}"}
    runs = (("integral_fp64", dict(precision=W.PREC_FP64, mu_method=2)),
            ("segment_fp64", dict(precision=W.PREC_FP64)),
            ("segment_fp32", dict(precision=W.PREC_FP32_PHASE64)),
            ("maclaurin_fp32", dict(precision=W.PREC_FP32_PHASE64, mu_method=1)))
    eta = {}
    for name, kw in runs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eta[name] = eng.eval_eta(wl.numerics, cuts, **kw)["eta"]
        res[name + "_s"] = time.perf_counter() - t0
    for name in ("segment_fp64", "segment_fp32", "maclaurin_fp32"):
        res[name + "_max_abs_db_vs_integral"] = float(np.max(np.abs(10 * np.log10(eta[name] / eta["integral_fp64"]))))
    res["segment_fp32_time_saving_vs_integral"] = 1.0 - res["segment_fp32_s"] / res["integral_fp64_s"]
    return res


def mu_accuracy_map_leg(eng, W, torch, crs=(0.0, 0.14, 0.28, 0.56, 0.84, 1.12)):
    """Accuracy of the two closed forms against the integral form (Eq. 23) as
    the ISRS power transfer grows: the paper's Table I link (101 x 10 GBd,
    19 dBm, one 100 km span), every third channel under test, Cr swept; all
    three forms on the GPU in FP64 (the integral form is pinned to the oracle
    by the tests)."""
    cuts = np.arange(0, 101, 3, dtype=np.int32)
    rows = []
    for cr in crs:
        wl = W.table1_1thz(cr=cr, fmt="qpsk", n_grid=10)
        eng.load(wl)
        eta, secs = {}, {}
        for name, mu, kw in (("integral", 2, dict(dz=0.25)), ("segment", 0, {}), ("maclaurin", 1, {})):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eta[name] = eng.eval_eta(wl.numerics, cuts, precision=W.PREC_FP64, mu_method=mu, **kw)["eta"]
            secs[name] = time.perf_counter() - t0
        sp, span = wl.spectrum, wl.link.spans[0]
        alpha = span["alpha_db_km"] / (10.0 / np.log(10.0))
        leff = (1.0 - np.exp(-alpha * span["length_km"])) / alpha
        # Eq. 12: power transfer between the outermost channels
        d_rho = 10.0 / np.log(10.0) * sp.power_w.sum() * cr * leff * sp.n_ch * sp.spacing_thz
        row = {"cr": cr, "delta_rho_db": float(d_rho), "seconds": secs}
        for name in ("segment", "maclaurin"):
            e = 10 * np.log10(eta[name] / eta["integral"])
            row[name + "_max_abs_db"] = float(np.max(np.abs(e)))
            row[name + "_mae_db"] = float(np.mean(np.abs(e)))
        rows.append(row)
    return {"workload": ("Table I link, 1 x 100 km, QPSK, 10 x 10 points per square, CUTs 0, 3, ..., 99; "
                         "closed forms at dz 1 km, integral form at 0.25 km"),
            "rows": rows}


def outer_integral_leg(eng, W, torch, n_f=5, n_cuts=10, grid=1024):
    """The outer f-integral of Eq. 17 with n_f midpoint samples over the CUT's
    band against the CUT-centre sample (n_f = 1), on the benchmark link at a
    grid that resolves the FWM-efficiency ridges (1024 x 1024): time and the
    change of eta, the NLI PSD across the middle CUT, and the convergence of
    the CUT-centre PSD of that CUT with the (f1, f2) grid."""
    wl = W.cl_100ch_10span(n_grid=grid)
    cuts = np.linspace(0, len(wl.cuts) - 1, n_cuts).astype(np.int32)
    mid = int(cuts[n_cuts // 2])
    eng.load(wl)
    res = {"workload": f"{n_cuts} CUTs of the benchmark link at {grid}x{grid}, n_f {n_f}"}
    eta = {}
    for nf in (1, n_f):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eta[nf] = eng.eval_eta(wl.numerics, cuts, precision=W.PREC_FP32_PHASE64, n_f=nf)["eta"]
        res[f"n_f{nf}_s"] = time.perf_counter() - t0
    d = 10 * np.log10(eta[n_f] / eta[1])
    res["eta_change_db"] = {"min": float(d.min()), "max": float(d.max()), "mean": float(d.mean())}
    f, psd = eng.eval_psd(wl.numerics, [mid], precision=W.PREC_FP32_PHASE64, n_f=n_f)
    res["psd_cut_%d" % mid] = {"f_thz": [float(v) for v in f[0]],
                               "rel_to_centre": [float(v) for v in psd[0] / psd[0][n_f // 2]]}
    conv = {}
    for n in (64, 128, 256, 512, 1024):
        w = W.cl_100ch_10span(n_grid=n)
        eng.load(w)
        conv[str(n)] = float(eng.eval_psd(w.numerics, [mid], precision=W.PREC_FP32_PHASE64, n_f=1)[1][0][0])
    res["centre_psd_vs_grid_db_rel_1024"] = {k: float(10 * np.log10(v / conv["1024"])) for k, v in conv.items()}
    return res


def per_cut_dz_leg(eng, wl, eta_dz1, W, torch):
    """The segment form's step chosen per CUT (error model on a 32 x 32 grid,
    0.005 dB against a 0.5 km step), then the full workload with those steps."""
    cuts = wl.cuts
    cand = [0.5, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0]
    eng.load(wl)
    t0 = time.perf_counter()
    dz, _ = eng.choose_dz(wl.numerics, cuts, cand, 0.005, precision=W.PREC_FP64, n=32)
    t_choose = time.perf_counter() - t0
    r = eng.eval_eta_dz(wl.numerics, cuts, dz, precision=W.PREC_FP32_PHASE64)      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = eng.eval_eta_dz(wl.numerics, cuts, dz, precision=W.PREC_FP32_PHASE64)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"choose_s": t_choose, "dz_km_min": float(dz.min()), "dz_km_max": float(dz.max()),
            "dz_km_mean": float(dz.mean()), "value": len(cuts) / dt, "unit": "CUT/s",
            "max_abs_db_vs_dz1": float(np.max(np.abs(10 * np.log10(r["eta"] / eta_dz1))))}


def surrogate_leg(eng, n_points, torch, train_rows=1 << 22, members=4, heldout_links=1024, loop_links=8):
    """Ensemble surrogate of the per-span FWM factor: training time, held-out
    error against the closed form, and throughput of inference with fallback
    (0.01 dB spread threshold) against the closed form on the same points."""
    db = 10.0 / np.log(10.0)

    def data(n, seed):
        x = torch.empty(n, 16, device="cuda")
        r = torch.empty(n, device="cuda")
        y6 = torch.empty(n, device="cuda")
        eng.surrogate_datagen(x, r, seed, y6=y6)
        return x, r, y6

    x, r, _ = data(train_rows, 4)
    s = eng.surrogate(members, seed=4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.train(x, r, steps=1500, batch=1024, lr=1e-3)
    loss = s.train(x, r, steps=500, batch=1024, lr=3e-4)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del x, r
    xh, _, _ = data(8192, 1000)
    ycf = torch.empty(8192, device="cuda")
    eng.closed_form_points(xh, ycf)
    yh = torch.empty(8192, device="cuda")
    res = {}
    for thr in (float("inf"), 0.01):
        nf = s.eval_points(xh, yh, thr)
        err = db * (yh - ycf).double().cpu().numpy()
        res["no_fallback" if thr == float("inf") else "thr_0p01_db"] = {
            "rms_db": float(np.sqrt(np.mean(err ** 2))), "max_abs_db": float(np.abs(err).max()),
            "fallback_fraction": nf / 8192}
    xb, _, y6b = data(n_points, 5)
    yb = torch.empty(n_points, device="cuda")
    times = {}
    nfb = 0
    for name in ("closed_form", "surrogate_thr_0p01_db", "surrogate_no_fallback"):
        def run():
            if name == "closed_form":
                eng.closed_form_points(xb, yb)
                return 0
            return s.eval_points(xb, yb, 0.01 if "0p01" in name else float("inf"))
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            k = run()
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t0) / 3
        if "0p01" in name:
            nfb = k
    flop_pt = 2 * (16 * 256 + 3 * 256 * 256 + 256) * members
    t_sur = times["surrogate_no_fallback"]
    # surrogate in the loop: eta of 3 CUTs of the C+L link at 64^2
    from paper_2412_11614_amd import workloads as W
    wl = W.cl_100ch_10span(n_grid=64)
    cuts = np.array([3, 50, 96], dtype=np.int32)
    eng.load(wl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref = eng.eval_eta(wl.numerics, cuts, precision=W.PREC_FP32_PHASE64)["eta"]
    t_cf = time.perf_counter() - t0
    loop = {"workload": "C+L link (100 x 96 GBd, 10 spans), CUTs 3/50/96, 64x64 per square",
            "closed_form_s": t_cf}
    for name, thr in (("no_fallback", float("inf")), ("thr_0p01_db", 0.01)):
        t0 = time.perf_counter()
        eta, fb = s.eval_eta(wl.numerics, cuts, thr)
        dt = time.perf_counter() - t0
        loop[name] = {"s": dt, "fallback_fraction": fb,
                      "eta_err_db": [float(v) for v in 10 * np.log10(eta / ref)]}
    s.close()
    link_trained = surrogate_link_leg(eng, torch, W, train_rows, members, wl, cuts, ref,
                                      heldout_links=heldout_links, loop_links=loop_links)
    return {"workload": (f"{members}-member 16-256x4-1 SiLU ensemble, BF16 MFMA; trained on {train_rows} "
                         f"closed-form samples (2000 Adam steps of 1024 per member); {n_points} query points "
                         f"(100 x 100 GHz grid squares, 80-100 km spans, 17-23 dBm)"),
            "train_s": t_train, "train_loss_ln2": [float(v) for v in loss], "held_out_8192": res,
            "points_per_s": {k: n_points / v for k, v in times.items()},
            "fallback_fraction_bench": nfb / n_points,
            "speedup_vs_closed_form": times["closed_form"] / times["surrogate_thr_0p01_db"],
            "mlp_tflops": flop_pt * n_points / t_sur / 1e12, "mlp_peak_bf16_tflops": 2500.0,
            "eta_in_the_loop": loop, "link_trained": link_trained}


def surrogate_link_leg(eng, torch, W, train_rows, members, wl, cuts, ref, n_links=64, heldout_links=1024,
                       heldout_points=4096, loop_links=8):
    """The ensemble trained on the query distribution of real links: points
    drawn from the CUTs, channel pairs, grid cells and spans of n_links C+L
    links (the benchmark link's distribution, seeds 100..), its fallback gate
    calibrated on points of n_links other links (seeds 500..) to 0.007 dB per
    point, then tested on heldout_points points of each of heldout_links
    held-out links (seeds 1000..) and in the loop on loop_links links (seeds
    2000..; CUTs 3, 50, 96 at 64 x 64)."""
    db = 10.0 / np.log(10.0)

    def draw(seed0, n_l, n, seed):
        b = eng.batch([W.cl_100ch_10span(seed=seed0 + i, n_grid=wl.numerics.n_grid) for i in range(n_l)])
        x = torch.empty(n, 16, device="cuda")
        r = torch.empty(n, device="cuda")
        rej = eng.surrogate_datagen_batch(b, wl.numerics.n_grid, x, r, seed)
        b.close()
        return x, r, rej

    t0 = time.perf_counter()
    x, r, rej = draw(100, n_links, train_rows, 4)
    t_gen = time.perf_counter() - t0
    s = eng.surrogate(members, seed=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.train(x, r, steps=4000, batch=1024, lr=1e-3)
    s.train(x, r, steps=2000, batch=1024, lr=3e-4)
    loss = s.train(x, r, steps=2000, batch=1024, lr=1e-4)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del x, r
    xc, _, _ = draw(500, n_links, 1 << 20, 5)
    thr, cal_err, cal_frac = s.calibrate(xc, 0.007)
    del xc
    # held-out points: errors without fallback, at the calibrated gate, and the spread -> error map
    nh = heldout_links * heldout_points
    t0 = time.perf_counter()
    xh, _, _ = draw(1000, heldout_links, nh, 1000)
    t_hgen = time.perf_counter() - t0
    log(f"surrogate: {nh} held-out points from {heldout_links} links drawn in {t_hgen:.1f} s")
    ycf = torch.empty(nh, device="cuda")
    eng.closed_form_points(xh, ycf)
    mean = torch.empty(nh, device="cuda")
    spread = torch.empty(nh, device="cuda")
    s.predict(xh, mean, spread)
    yh = torch.empty(nh, device="cuda")
    held = {}
    for name, t in (("no_fallback", float("inf")), ("calibrated_gate", thr)):
        nf = s.eval_points(xh, yh, t)
        err = np.abs(db * (yh - ycf).double().cpu().numpy())
        held[name] = {"rms_db": float(np.sqrt(np.mean(err ** 2))), "max_abs_db": float(err.max()),
                      "fallback_fraction": nf / nh}
    s.eval_points(xh, yh, float("inf"))
    err = np.abs(db * (yh - ycf).double().cpu().numpy())
    spr = db * spread.double().cpu().numpy()
    qs = np.quantile(spr, np.linspace(0, 1, 11))
    smap = []
    for lo, hi in zip(qs[:-1], qs[1:]):
        m = (spr >= lo) & (spr <= hi)
        smap.append({"spread_db": [float(lo), float(hi)], "max_err_db": float(err[m].max()),
                     "p99_err_db": float(np.quantile(err[m], 0.99))})
    del xh, ycf, mean, spread, yh
    # in the loop
    loop_cuts = np.array([3, 50, 96], dtype=np.int32)
    loop = {"links": loop_links, "cuts": loop_cuts.tolist(), "max_abs_db_no_fallback": 0.0,
            "max_abs_db_calibrated_gate": 0.0, "fallback_fraction": [], "s_surrogate": 0.0, "s_closed_form": 0.0}
    for i in range(loop_links):
        w = W.cl_100ch_10span(seed=2000 + i, n_grid=64)
        eng.load(w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ref_i = eng.eval_eta(w.numerics, loop_cuts, precision=W.PREC_FP32_PHASE64)["eta"]
        loop["s_closed_form"] += time.perf_counter() - t0
        eta_n, _ = s.eval_eta(w.numerics, loop_cuts, float("inf"))
        t0 = time.perf_counter()
        eta_g, fb = s.eval_eta(w.numerics, loop_cuts, thr)
        loop["s_surrogate"] += time.perf_counter() - t0
        loop["max_abs_db_no_fallback"] = max(loop["max_abs_db_no_fallback"],
                                             float(np.max(np.abs(10 * np.log10(eta_n / ref_i)))))
        loop["max_abs_db_calibrated_gate"] = max(loop["max_abs_db_calibrated_gate"],
                                                 float(np.max(np.abs(10 * np.log10(eta_g / ref_i)))))
        loop["fallback_fraction"].append(fb)
        if (i + 1) % 32 == 0:
            log(f"surrogate in the loop: {i + 1} of {loop_links} links")
    s.close()
    return {"workload": (f"{train_rows} points from {n_links} C+L links (seeds 100-{99 + n_links}), gate calibrated on "
                         f"1048576 points of {n_links} others (seeds 500-), {heldout_points} held-out points on each of "
                         f"{heldout_links} links (seeds 1000-), in the loop on {loop_links} links (seeds 2000-)"),
            "datagen_s": t_gen, "rejected_draws": rej, "train_s": t_train, "train_steps_per_member": 8000,
            "train_loss_ln2": [float(v) for v in loss],
            "gate": {"target_db": 0.007, "threshold_db": thr, "calibration_max_err_db": cal_err,
                     "calibration_accepted": cal_frac},
            "held_out": held, "held_out_points": nh, "held_out_datagen_s": t_hgen, "spread_to_error_map": smap,
            "eta_in_the_loop": loop}


def _gold(stage):
    path = os.path.join(GOLDEN, f"oracle_percut_{stage}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def headline_accuracy(eng, W):
    """The headline path (FP64, segment form) on the S+C+L workload against
    stored oracle values of the model (integral form, adaptive quadrature):
    per-CUT eta at 64 x 64 (4 seeded CUTs) and 128 x 128 (CUTs 0, 75), and the
    GN sums of every near-CUT square of four CUTs at the full 1024 x 1024 grid
    (an oracle CUT at that grid is out of reach; the near squares carry most of
    its eta)."""
    out = {}
    errs = []
    for stage, n in (("scl64", 64), ("scl128", 128)):
        g = _gold(stage)
        if g is None:
            continue
        wl = W.sclband_150ch_40span(n_grid=n)
        eng.load(wl)
        got = eng.eval_eta(wl.numerics, g["cuts"], precision=W.PREC_FP64, n=n)["eta"]
        e = np.abs(10 * np.log10(got / np.array(g["eta"])))
        out[f"eta_{n}x{n}"] = {"cuts": g["cuts"], "max_abs_db": float(e.max())}
        errs.append(e.max())
    g = _gold("scl1024sq")
    if g is not None:
        wl = W.sclband_150ch_40span(n_grid=1024)
        eng.load(wl)
        by_cut = {}
        for e in g["squares"]:
            by_cut.setdefault(e["cut"], []).append(e)
        worst = 0.0
        for cut, ents in sorted(by_cut.items()):
            keys = [(e["k1"], e["k2"]) for e in ents]
            ref = np.array([e["terms"] for e in ents])
            got = eng.eval_islands(wl.numerics, cut, keys, precision=W.PREC_FP64)
            worst = max(worst, abs(10 * np.log10(got[:, :, 0].sum() / ref[:, :, 0].sum())))
        out["near_cut_squares_1024"] = {"cuts": sorted(by_cut), "squares": len(g["squares"]),
                                        "max_abs_db_of_gn_sum": float(worst)}
        errs.append(worst)
    out["max_abs_db_vs_oracle"] = float(max(errs)) if errs else None
    out["within_0p01_db"] = bool(errs) and bool(max(errs) <= 0.01)
    return out


def cl_leg(eng, W, torch, reps=2):
    """The C+L workload (100 x 96 GBd, 10 spans, 256 x 256 per square): all 100
    CUTs per step in the FP32-integrand / FP64-phase variant and in FP64, with
    both against stored oracle values (CUTs 0/49/99 at 256 x 256, all CUTs at 64 x 64)."""
    wl = W.cl_100ch_10span(n_grid=256)
    cuts = wl.cuts
    n = len(cuts)
    eng.load(wl)
    eta = torch.empty(n, dtype=torch.float64, device="cuda")
    res = {"workload": ("C+L 10 THz: 100 x 96 GBd on 100 GHz, roll-off 0.04, 20 dBm with +-2 dB tilt, 10 spans "
                        "U[80,100] km (seed 2), 16QAM/64QAM alternating, EGN on, 256x256 per square, all 100 CUTs")}
    out_eta = {}
    for name, prec, k in (("fp32_phase64", W.PREC_FP32_PHASE64, reps), ("fp64", W.PREC_FP64, 1)):
        eng.eval_eta_dev(wl.numerics, cuts[:4], eta, precision=prec)        # warm (plan shapes, code)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            eng.eval_eta_dev(wl.numerics, cuts, eta, precision=prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / k
        out_eta[prec] = eta.cpu().numpy().copy()
        eng.set_profiling(True)
        eng.eval_eta_dev(wl.numerics, cuts, eta, precision=prec)
        torch.cuda.synchronize()
        st = eng.stats()
        eng.set_profiling(False)
        fp32 = prec == W.PREC_FP32_PHASE64
        res[name] = {"value": n / dt, "unit": "CUT/s", "ms_per_step": 1e3 * dt,
                     "roofline": kernel_roofline(st, PEAK_FP32_TFLOPS if fp32 else PEAK_FP64_TFLOPS,
                                                 "region_queue_kernel<%s, 0>" % ("float" if fp32 else "double"),
                                                 CL_PROFILE if fp32 else "none"),
                     "region_launches": st.region_launches, "squares": st.n_squares,
                     "delta_squares": st.n_delta_squares}
    acc = {"fp32_vs_fp64_max_abs_db": float(np.max(np.abs(10 * np.log10(out_eta[W.PREC_FP32_PHASE64] /
                                                                          out_eta[W.PREC_FP64]))))}
    g = _gold("cl256")
    if g is not None:
        pos = np.searchsorted(cuts, g["cuts"])
        for prec, name in ((W.PREC_FP32_PHASE64, "fp32_phase64"), (W.PREC_FP64, "fp64")):
            e = np.abs(10 * np.log10(out_eta[prec][pos] / np.array(g["eta"])))
            acc[f"{name}_vs_oracle_256_max_abs_db"] = float(e.max())
        acc["oracle_256_cuts"] = g["cuts"]
    g = _gold("cl64")
    if g is not None:
        for prec, name in ((W.PREC_FP32_PHASE64, "fp32_phase64"), (W.PREC_FP64, "fp64")):
            got = eng.eval_eta(wl.numerics, g["cuts"], precision=prec, n=64)["eta"]
            acc[f"{name}_vs_oracle_64_all_cuts_max_abs_db"] = float(np.max(np.abs(10 * np.log10(got / np.array(g["eta"])))))
    res["accuracy"] = acc
    return res, wl, out_eta[W.PREC_FP32_PHASE64]


def profile_run(args, torch, _lib, W):
    """Timed steps of one other kernel, for its counter runs: the C+L workload
    (region_queue_kernel<float, 0>) or the surrogate's fused inference
    (mlp_fused_kernel).  Prints one JSON line with the HIP-event times."""
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    eng = _lib.Engine(0, stream=stream)
    out = {"workload": args.workload, "steps": args.steps}
    if args.workload == "cl":
        wl = W.cl_100ch_10span(n_grid=256)
        eng.load(wl)
        eta = torch.empty(len(wl.cuts), dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            eng.eval_eta_dev(wl.numerics, wl.cuts, eta, precision=W.PREC_FP32_PHASE64)
        torch.cuda.synchronize()
        eng.set_profiling(True)
        ms = []
        for _ in range(args.steps):
            eng.eval_eta_dev(wl.numerics, wl.cuts, eta, precision=W.PREC_FP32_PHASE64)
            torch.cuda.synchronize()
            st = eng.stats()
            ms.append(st.region_ms)
        out["roofline"] = kernel_roofline(st, PEAK_FP32_TFLOPS, "region_queue_kernel<float, 0>", CL_PROFILE)
        out["region_ms"] = ms
    elif args.workload == "batch":
        links = W.batch_links()
        nu = links[0].numerics
        b = eng.batch(links)
        eta = torch.empty(b.n_cuts, dtype=torch.float64, device="cuda")
        for _ in range(max(2, args.warmup)):      # eager run, then the graph capture
            b.eval_dev(nu, eta)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.eval_dev(nu, eta)
        torch.cuda.synchronize()
        out.update({"n_cut": b.n_cuts, "ms_per_step": 1e3 * (time.perf_counter() - t0) / max(1, args.steps),
                    "shape": b.tuning()})
        b.close()
    else:
        n = 1 << 22
        x = torch.empty(n, 16, device="cuda")
        r = torch.empty(n, device="cuda")
        eng.surrogate_datagen(x, r, 4)
        s = eng.surrogate(4, seed=4)
        s.train(x, r, steps=200, batch=1024, lr=1e-3)
        y = torch.empty(n, device="cuda")
        for _ in range(args.warmup):
            s.eval_points(x, y, float("inf"))
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(args.steps):
            s.eval_points(x, y, float("inf"))
        ev[1].record(stream)
        torch.cuda.synchronize()
        dt = ev[0].elapsed_time(ev[1]) * 1e-3 / max(1, args.steps)
        flop = 2 * (16 * 256 + 3 * 256 * 256 + 256) * 4 * n
        out.update({"points": n, "ms_per_call": 1e3 * dt, "points_per_s": n / dt,
                    "mfma_tflops": flop / dt / 1e12, "frac_bf16_peak": flop / dt / 1e12 / 2500.0})
        s.close()
    eng.close()
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 4 * n
    print(json.dumps(out, default=_plain), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-squares", type=int, default=0,
                    help="oracle squares of the CPU baseline (0: one per host thread, at most 16)")
    ap.add_argument("--only-headline", action="store_true", help="the timed steps only (for counter runs)")
    ap.add_argument("--workload", choices=("scl", "cl", "mlp", "batch"), default="scl",
                    help="timed steps: scl (the headline), or, for profiling the other kernels, cl (the C+L "
                         "workload, all 100 CUTs per step, FP32 integrand), mlp (surrogate inference, 4 M "
                         "points per step, no fallback) or batch (the 512-link batch, graph replays)")
    ap.add_argument("--mu-map", type=int, default=1, help="closed-form accuracy map leg (0 = skip)")
    ap.add_argument("--outer-nf", type=int, default=5, help="outer-integral leg samples (1 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-links", type=int, default=512,
                    help="links of the batched leg (0 = skip)")
    ap.add_argument("--plain-links", type=int, default=48,
                    help="links of the batch evaluated one by one on the plain path for comparison")
    ap.add_argument("--per-cut-dz", type=int, default=1, help="run the per-CUT step leg (0 = skip)")
    ap.add_argument("--integral-cuts", type=int, default=10,
                    help="CUTs of the integral-form comparison leg (0 = skip)")
    ap.add_argument("--surrogate-points", type=int, default=1 << 22,
                    help="query points of the surrogate leg (0 = skip)")
    ap.add_argument("--surrogate-heldout-links", type=int, default=1024,
                    help="held-out links of the link-trained surrogate, 4096 points each (8192 at full scale)")
    ap.add_argument("--surrogate-loop-links", type=int, default=8,
                    help="links of the surrogate-in-the-loop test, 3 CUTs each (256 at full scale)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the steps, copy this many MiB device-to-device (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the path is single-GPU "
              "and shards by (CUT, square) lists without collectives in the compute.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2412_11614_amd import _lib, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload != "scl":
        profile_run(args, torch, _lib, W)
        return
    wl = W.sclband_150ch_40span(n_grid=1024, precision=W.PREC_FP64)
    n_ch = wl.spectrum.n_ch
    K = args.steps
    step_cuts = [int(round((i + 0.5) * n_ch / K - 0.5)) % n_ch for i in range(K)] if K <= n_ch \
        else [i % n_ch for i in range(K)]
    stream = torch.cuda.Stream()          # shared with the library: torch and the kernels stay ordered
    torch.cuda.set_stream(stream)
    eng = _lib.Engine(0, stream=stream)
    eng.load(wl)
    eta = torch.empty(max(K, 1), dtype=torch.float64, device=dev)
    s2 = torch.empty(max(K, 1), dtype=torch.float64, device=dev)
    terms = torch.empty(max(K, 1) * 5, dtype=torch.float64, device=dev)

    def step(i, cut):
        eng.eval_eta_dev(wl.numerics, [cut], eta[i:i + 1], s2[i:i + 1], terms[5 * i:5 * i + 5],
                         precision=W.PREC_FP64)

    mid = n_ch // 2
    log(f"warmup {args.warmup} step(s) on CUT {mid}; {K} timed steps, one CUT each")
    for _ in range(args.warmup):
        step(0, mid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, cut in enumerate(step_cuts):
        step(i, cut)
        log(f"step {i} (CUT {cut}) queued at {time.perf_counter() - t0:.1f} s")   # the host runs a step ahead
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed: {K} CUTs in {elapsed:.2f} s")
    eta_steps = eta[:K].cpu().numpy().copy()
    value = K / elapsed

    # kernel timing with HIP events on the library's stream (one extra step, the middle CUT)
    eng.set_profiling(True)
    step(0, mid)
    torch.cuda.synchronize()
    st = eng.stats()
    eng.set_profiling(False)
    roof = kernel_roofline(st, PEAK_FP64_TFLOPS, "region_queue_kernel<double, 0>", HEADLINE_PROFILE)
    log(f"region kernel {st.region_ms:.1f} ms in {st.region_launches} launch(es); host prep {st.host_prep_ms:.1f} ms; "
        f"{roof['achieved']:.2f} TFLOP/s ({roof['frac']:.3f} of FP64 peak)")

    out = {
        "metric": "CUT NLI coeffs/sec at <=0.01 dB vs FP64 oracle",
        "value": value,
        "unit": "CUT/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / max(K, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("S+C+L 15 THz: 150 x 100 GBd on 100 GHz, roll-off 0, 24 dBm flat, 40 x 80 km spans "
                                "with per-span alpha/beta2/beta3/gamma/Cr draws (seed 5), QPSK/16QAM/64QAM, EGN on, "
                                "1024x1024 points per square, dz 1 km, FP64; one CUT per step, the timed steps "
                                "spread evenly over the 150 CUTs"),
                   "cuts_timed": step_cuts, "grid": 1024, "spans": 40, "channels": n_ch},
        "roofline": roof,
        "detail": {"region_ms": st.region_ms, "assemble_ms": st.assemble_ms, "host_prep_ms": st.host_prep_ms,
                   "region_launches": st.region_launches, "squares": st.n_squares,
                   "delta_squares": st.n_delta_squares, "live_points": st.n_points_live,
                   "horner_steps": st.horner_steps, "eta_timed_cuts": [float(v) for v in eta_steps]},
    }
    if not args.only_headline:
        log("accuracy against the oracle")
        out["accuracy"] = headline_accuracy(eng, W)
        # the host-buffer entry point (CUT list in, eta out through host memory, synchronous)
        eng.load(wl)
        t1 = time.perf_counter()
        eng.eval_eta(wl.numerics, [mid], precision=W.PREC_FP64)
        out["host_buffers"] = {"value": 1.0 / (time.perf_counter() - t1), "unit": "CUT/s", "cut": mid}
        # the same sample with the FP32 integrand (FP64 phases and sums)
        sample = step_cuts[::max(1, K // 5)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r32 = eng.eval_eta(wl.numerics, sample, precision=W.PREC_FP32_PHASE64)
        dt = time.perf_counter() - t1
        pos = [step_cuts.index(c) for c in sample]
        out["fp32_phase64"] = {"value": len(sample) / dt, "unit": "CUT/s", "cuts": sample,
                               "max_abs_db_vs_fp64": float(np.max(np.abs(10 * np.log10(r32["eta"] / eta_steps[pos]))))}
        log("C+L workload")
        out["cl_100ch_10span"], wl2, eta32 = cl_leg(eng, W, torch)
        if args.integral_cuts > 0:
            log("integral form leg")
            out["integral_form"] = integral_form_leg(eng, wl2, W, torch, args.integral_cuts)
        if args.per_cut_dz:
            out["per_cut_dz"] = per_cut_dz_leg(eng, wl2, eta32, W, torch)
        if args.outer_nf > 1:
            log("outer-integral leg")
            out["outer_integral"] = outer_integral_leg(eng, W, torch, n_f=args.outer_nf)
        if args.mu_map:
            log("closed-form accuracy map")
            out["mu_accuracy_map"] = mu_accuracy_map_leg(eng, W, torch)
        if args.batch_links > 0:
            out["batched"] = batched_leg(eng, args.batch_links, args.plain_links, W, torch)
        if args.surrogate_points > 0:
            log("surrogate leg")
            out["surrogate"] = surrogate_leg(eng, args.surrogate_points, torch, heldout_links=args.surrogate_heldout_links,
                                         loop_links=args.surrogate_loop_links)
    eng.close()

    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 4 * n

    if not args.no_cpu_baseline and not args.only_headline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_squares)
    print(json.dumps(out, default=_plain), flush=True)


if __name__ == "__main__":
    main()
