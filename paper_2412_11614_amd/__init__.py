"""MI355X (gfx950) implementation of the ISRS-aware EGN hot path of
arXiv 2412.11614: per-CUT NLI coefficients from the island integrals of the
EGN model with the closed-form (segment) FWM efficiency factor.

    from paper_2412_11614_amd import Engine, workloads
    wl = workloads.cl_100ch_10span()
    with Engine(0) as e:
        e.load(wl)
        out = e.eval_eta(wl.numerics, wl.cuts)

The compute runs in libisrs_egn.so (HIP, built by paper_2412_11614_amd.build);
importing this package does not load it.
"""
from . import workloads  # noqa: F401


def __getattr__(name):
    if name in ("Engine", "IsrsError", "lib"):
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)
