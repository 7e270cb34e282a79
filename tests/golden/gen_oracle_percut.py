"""Writes oracle_percut_<stage>.json: per-CUT NLI coefficients (Eq. 11) of the
benchmark workloads from the FP64 CPU oracle, for the GPU parity tests and the
benchmark's accuracy check.

Only the oracle is called here.  Each stage is one file, so the long ones can
be generated and committed separately:

  cl64       C+L 100 ch, 10 spans, 64 x 64: every CUT, integral form (the model)
  cl64seg    C+L at 64 x 64: CUTs 0, 49, 99, segment form (the method, Eqs. 7-10)
  cl256      C+L at 256 x 256: CUTs 0, 49, 99, integral form
  scl64      S+C+L 150 ch, 40 spans, 64 x 64: 4 seeded CUTs (0, 75, 149 and 1 drawn),
             integral form
  scl128     S+C+L at 128 x 128: CUTs 0 and 75, integral form
  scl1024sq  S+C+L at 1024 x 1024: every near-CUT square (|k1 - CUT|, |k2 - CUT| <= 2,
             k1 <= k2) of CUTs 0, 75, 149 and one drawn CUT, bare island integrals,
             integral form
  batchx     512-link batch at 64 x 64, the far end of its cost distribution: the
             first, middle and last CUT of link 20 (30 spans), of link 343 (97
             channels, 30 spans, the costliest) and of link 91 (100 channels),
             integral form

Run from the repository root:
    python tests/golden/gen_oracle_percut.py <stage> [<stage> ...]
Hours of CPU time in total (on 8 cores: cl64 about 2.5 h, scl128 about 1.2 h,
cl256 about 1 h, scl64 and batchx under 1 h each, scl1024sq 10 min); each
stage prints its own time.
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2412_11614_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def seeded_cuts(fixed, n_ch, seed, n_total=8):
    rng = np.random.default_rng(seed)
    rest = [int(c) for c in rng.permutation(n_ch) if int(c) not in fixed]
    return sorted(list(fixed) + rest[: n_total - len(fixed)])


def cut_record(wl, cuts, method, n_grid):
    # one CUT per oracle call, each announced when done (long stages show progress)
    t0 = time.time()
    eta, s2, terms = [], [], []
    for c in cuts:
        r = oracle.eval_cuts(wl, cuts=[int(c)], method=method, n_grid=n_grid)
        eta.append(float(r["eta"][0]))
        s2.append(float(r["sigma2"][0]))
        terms.append([float(v) for v in r["terms"][0]])
        print(f"  CUT {int(c)}: eta {eta[-1]:.6e} after {time.time() - t0:.0f} s", flush=True)
    return {"cuts": [int(c) for c in cuts], "method": method, "n_grid": n_grid,
            "eta": eta, "sigma2": s2, "terms": terms, "seconds": time.time() - t0}


def stage_cl64():
    wl = W.cl_100ch_10span(n_grid=64)
    return {"workload": "cl_100ch_10span(seed=2, n_grid=64)", **cut_record(wl, wl.cuts, "integral", 64)}


def stage_cl64seg():
    wl = W.cl_100ch_10span(n_grid=64)
    return {"workload": "cl_100ch_10span(seed=2, n_grid=64)", **cut_record(wl, [0, 49, 99], "segment", 64)}


def stage_cl256():
    wl = W.cl_100ch_10span(n_grid=256)
    return {"workload": "cl_100ch_10span(seed=2, n_grid=256)", **cut_record(wl, [0, 49, 99], "integral", 256)}


def stage_scl64():
    wl = W.sclband_150ch_40span(n_grid=64)
    cuts = seeded_cuts([0, 75, 149], 150, seed=55, n_total=4)
    return {"workload": "sclband_150ch_40span(seed=5, n_grid=64)", **cut_record(wl, cuts, "integral", 64)}


def stage_scl128():
    wl = W.sclband_150ch_40span(n_grid=128)
    return {"workload": "sclband_150ch_40span(seed=5, n_grid=128)", **cut_record(wl, [0, 75], "integral", 128)}


def stage_scl1024sq():
    import concurrent.futures as cf
    wl = W.sclband_150ch_40span(n_grid=1024)
    cuts = [0, 75, 149, seeded_cuts([], 150, seed=56, n_total=1)[0]]
    picks = []
    for cut in cuts:
        for k1 in range(max(cut - 2, 0), min(cut + 2, 149) + 1):
            for k2 in range(k1, min(cut + 2, 149) + 1):
                picks.append((cut, k1, k2))

    def one(p):
        cut, k1, k2 = p
        t0 = time.time()
        v = oracle.square_terms(wl, cut, k1, k2, method="integral")
        return {"cut": cut, "k1": k1, "k2": k2, "method": "integral", "terms": v.tolist(),
                "seconds": time.time() - t0}

    threads = int(os.environ.get("GOLDEN_THREADS", os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(threads) as ex:
        squares = list(ex.map(one, picks))
    return {"workload": "sclband_150ch_40span(seed=5, n_grid=1024)", "cuts": cuts, "squares": squares}


def stage_batchx():
    links = W.batch_links()
    out = []
    for li in (20, 343, 91):
        wl = links[li]
        act = wl.cuts
        cuts = act[np.linspace(0, len(act) - 1, 3).round().astype(int)]
        rec = cut_record(wl, cuts, "integral", 64)
        rec.update({"link": li, "n_active": int(len(act)), "n_spans": int(len(wl.link.spans))})
        out.append(rec)
        print(f"  link {li}: {len(cuts)} CUTs in {rec['seconds']:.0f} s", flush=True)
    return {"workload": "batch_links(n_links=512, seed=3, n_grid=64)", "links": out}


STAGES = {k[len("stage_"):]: v for k, v in globals().items() if k.startswith("stage_")}


def main(argv):
    oracle.lib()
    for name in argv:
        if name not in STAGES:
            raise SystemExit(f"unknown stage {name}; stages: {sorted(STAGES)}")
        t0 = time.time()
        rec = STAGES[name]()
        rec.update({"generator": "tests/golden/gen_oracle_percut.py " + name, "oracle": "oracle/isrs_oracle.c (FP64)",
                    "threads": oracle.num_threads(), "host": platform.processor() or platform.machine(),
                    "wall_seconds": time.time() - t0})
        path = os.path.join(HERE, f"oracle_percut_{name}.json")
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        print(f"{name}: {time.time() - t0:.0f} s -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
