"""Writes oracle_fullsize.json: FP64 oracle values at the full sizes of the
benchmark workloads, on sampled outputs, for the GPU parity tests.

Only the oracle is called here.  Sampled outputs:

* C+L 100 x 96 GBd, 10 spans, 256 x 256 per square: bare island integrals
  (D, E, F, G, H for l = -1, 0, 1) of squares near and far from three CUTs,
  segment form (the method) and integral form (the model);
* S+C+L 150 x 100 GBd, 40 spans, 1024 x 1024 per square: bare island
  integrals of squares of two CUTs, segment and integral forms;
* the 512-link batch at 64 x 64: eta of every CUT of two links, segment form.

Run from the repository root:  python tests/golden/gen_oracle_fullsize.py
(about 10 minutes on 8 cores).
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2412_11614_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_fullsize.json")


def squares_job(wl, picks, methods, threads):
    def one(p):
        cut, k1, k2, m = p
        t0 = time.time()
        v = oracle.square_terms(wl, cut, k1, k2, method=m)
        return {"cut": cut, "k1": k1, "k2": k2, "method": m, "terms": v.tolist(), "seconds": time.time() - t0}

    jobs = [(c, a, b, m) for (c, a, b) in picks for m in methods]
    with cf.ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, jobs))


def main():
    oracle.lib()
    threads = os.cpu_count() or 1
    out = {"generator": "tests/golden/gen_oracle_fullsize.py", "oracle": "oracle/isrs_oracle.c (FP64)"}

    wl = W.cl_100ch_10span(n_grid=256)
    rng = np.random.default_rng(20)
    picks = []
    for cut in (0, 49, 99):
        near = [(cut, cut), (max(cut - 1, 0), min(cut + 1, 99)), (cut, min(cut + 1, 99)),
                (max(cut - 2, 0), cut)]
        far = [tuple(sorted(rng.integers(0, 100, size=2).tolist())) for _ in range(2)]
        for k1, k2 in near + far:
            picks.append((cut, int(min(k1, k2)), int(max(k1, k2))))
    t0 = time.time()
    out["cl_100ch_10span_256"] = {"workload": "cl_100ch_10span(n_grid=256)",
                                   "squares": squares_job(wl, picks, ("segment", "integral"), threads)}
    print(f"C+L squares: {len(picks)} in {time.time() - t0:.0f} s", flush=True)

    wl5 = W.sclband_150ch_40span(n_grid=1024)
    rng = np.random.default_rng(21)
    picks = []
    for cut in (0, 75):
        far = tuple(sorted(rng.integers(0, 150, size=2).tolist()))
        for k1, k2 in [(cut, cut), (max(cut - 1, 0), min(cut + 1, 149)), far]:
            picks.append((cut, int(min(k1, k2)), int(max(k1, k2))))
    t0 = time.time()
    out["sclband_150ch_40span_1024"] = {"workload": "sclband_150ch_40span(n_grid=1024)",
                                         "squares": squares_job(wl5, picks, ("segment", "integral"), threads)}
    print(f"S+C+L squares: {len(picks)} in {time.time() - t0:.0f} s", flush=True)

    links = W.batch_links()
    cost = [len(w.cuts) ** 3 * len(w.link.spans) * float(np.mean(w.link.spans["length_km"])) for w in links]
    chosen = [int(i) for i in np.argsort(cost)[:2]]
    t0 = time.time()
    res = []
    for i in chosen:
        r = oracle.eval_cuts(links[i], method="segment")
        res.append({"link": i, "cuts": links[i].cuts.tolist(), "eta": r["eta"].tolist()})
    out["batch_links_64"] = {"workload": "batch_links(n_links=512, seed=3, n_grid=64)", "links": res}
    print(f"batch links {chosen} in {time.time() - t0:.0f} s", flush=True)

    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
