"""Seeded synthetic workloads shaped like the paper's WDM links.

This module only draws and packs input parameters (channel grids, launch
powers, span parameters, numerics).  It holds none of the model's arithmetic:
both the HIP path and the CPU oracle receive the same arrays from here and
compute everything else on their own.

Units are the ones the C-ABI takes: THz, W, km, dB/km, ps^2/km, ps^3/km,
1/(W km), 1/(W km THz).

Workload shapes follow the paper's Table I (1 THz, 101 channels, 100 km spans)
and Table II (10 THz partial validation), widened to C+L and S+C+L grids with
uneven span lengths, tilted power profiles and mixed modulation formats.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np

# Format constants (Phi, Psi) of the EGN model's modulation-format correction
# terms.  Phi = mu4/mu2^2 - 2 and Psi = mu6/mu2^3 - 9 mu4/mu2^2 + 12 over the
# constellation's moments (EGN model, the paper's reference [17]); the values
# are plain inputs here.  The oracle derives them independently from the
# constellation points and a CPU test checks this table against it.
FORMATS = {
    "gaussian": (0.0, 0.0),
    "qpsk": (-1.0, 4.0),
    "16qam": (-0.68, 2.08),
    "64qam": (-13.0 / 21.0, 5548.0 / 3087.0),
}

GAIN_EQUALIZED = 0
GAIN_LOSS_ONLY = 1

PREC_FP64 = 0
PREC_FP32_PHASE64 = 1

MU_SEGMENT = 0     # the paper's segment closed form (Eqs. 7-10): the hot path
MU_MACLAURIN = 1   # the Maclaurin closed form (Eqs. 2-6)


def dbm_to_w(dbm):
    return 1e-3 * 10.0 ** (np.asarray(dbm, dtype=np.float64) / 10.0)


@dataclass
class Spectrum:
    """A WDM grid: n_ch slots at offsets (k - (n_ch-1)/2) * spacing from the grid centre."""
    n_ch: int
    spacing_thz: float
    symbol_rate_thz: float
    rolloff: float
    power_w: np.ndarray          # [n_ch], 0 = inactive slot
    phi: np.ndarray              # [n_ch]
    psi: np.ndarray              # [n_ch]
    f_center_thz: float = 193.4
    formats: Optional[List[str]] = None

    def active(self):
        return np.nonzero(self.power_w > 0)[0].astype(np.int32)


SPAN_DTYPE = np.dtype([
    ("length_km", np.float64),
    ("alpha_db_km", np.float64),
    ("beta2_ps2_km", np.float64),
    ("beta3_ps3_km", np.float64),
    ("gamma_w_km", np.float64),
    ("cr_w_km_thz", np.float64),
])


def make_spans(lengths, alpha=0.2, beta2=-21.7, beta3=0.14, gamma=1.3, cr=0.028):
    n = len(lengths)
    spans = np.zeros(n, dtype=SPAN_DTYPE)
    spans["length_km"] = lengths
    spans["alpha_db_km"] = np.broadcast_to(alpha, (n,))
    spans["beta2_ps2_km"] = np.broadcast_to(beta2, (n,))
    spans["beta3_ps3_km"] = np.broadcast_to(beta3, (n,))
    spans["gamma_w_km"] = np.broadcast_to(gamma, (n,))
    spans["cr_w_km_thz"] = np.broadcast_to(cr, (n,))
    return spans


@dataclass
class Link:
    spans: np.ndarray                  # structured array of SPAN_DTYPE
    gain_mode: int = GAIN_EQUALIZED
    ptot_override_w: float = 0.0       # > 0 freezes the ISRS total power


@dataclass
class Numerics:
    n_grid: int = 64                   # N x N midpoint grid per channel-pair square
    n_f: int = 1                       # outer f samples per CUT (1 = CUT centre)
    dz_km: float = 1.0                 # segment length target; K = ceil(L / dz)
    egn: int = 1                       # 1 = add the E, F, G, H format terms
    precision: int = PREC_FP64
    mu_method: int = MU_SEGMENT


@dataclass
class Workload:
    name: str
    spectrum: Spectrum
    link: Link
    numerics: Numerics
    cuts: np.ndarray                   # int32 channel indices under test

    def with_numerics(self, **kw):
        return replace(self, numerics=replace(self.numerics, **kw))


def _fmt_arrays(names: Sequence[str]):
    phi = np.array([FORMATS[n][0] for n in names], dtype=np.float64)
    psi = np.array([FORMATS[n][1] for n in names], dtype=np.float64)
    return phi, psi


def spectrum_from(n_ch, spacing, rs, rolloff, power_w, formats, f_center=193.4):
    phi, psi = _fmt_arrays(formats)
    return Spectrum(n_ch=int(n_ch), spacing_thz=float(spacing), symbol_rate_thz=float(rs),
                    rolloff=float(rolloff), power_w=np.asarray(power_w, dtype=np.float64).copy(),
                    phi=phi, psi=psi, f_center_thz=f_center, formats=list(formats))


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def single_span_11ch(n_grid=64):
    """11 x 64 GBd on 75 GHz, roll-off 0.1, 0 dBm/ch, one 80 km SSMF span, GN only,
    centre channel (index 5) under test."""
    sp = spectrum_from(11, 0.075, 0.064, 0.1, np.full(11, 1e-3), ["gaussian"] * 11)
    link = Link(make_spans([80.0]))
    return Workload("single_span_11ch", sp, link,
                    Numerics(n_grid=n_grid, egn=0, precision=PREC_FP64),
                    np.array([5], dtype=np.int32))


def cl_100ch_10span(seed=2, n_grid=256, precision=PREC_FP32_PHASE64):
    """C+L, 10 THz: 100 x 96 GBd on 100 GHz (roll-off 0.04), 20 dBm total with a
    linear +-2 dB tilt across the band, 10 spans of U[80,100] km, channels
    alternating 16QAM / 64QAM, every channel under test."""
    rng = np.random.default_rng(seed)
    n = 100
    tilt_db = np.linspace(-2.0, 2.0, n)
    p = 10.0 ** (tilt_db / 10.0)
    p *= dbm_to_w(20.0) / p.sum()
    fmts = ["16qam" if k % 2 == 0 else "64qam" for k in range(n)]
    sp = spectrum_from(n, 0.1, 0.096, 0.04, p, fmts)
    lengths = rng.uniform(80.0, 100.0, size=10)
    link = Link(make_spans(lengths))
    return Workload("cl_100ch_10span", sp, link,
                    Numerics(n_grid=n_grid, egn=1, precision=precision),
                    np.arange(n, dtype=np.int32))


def batch_links(n_links=512, seed=3, n_grid=64):
    """Uneven links for batched evaluation: per link 20..100 active slots of a
    100 x 96 GBd / 100 GHz grid, powers U[-3,3] dBm, 1..30 spans of U[50,120] km,
    alpha U[0.17,0.22] dB/km and Cr U[0.025,0.032] per link, formats drawn from
    {QPSK, 16QAM, 64QAM}; every active channel is under test."""
    rng = np.random.default_rng(seed)
    out = []
    names = ["qpsk", "16qam", "64qam"]
    for li in range(n_links):
        n_act = int(rng.integers(20, 101))
        act = np.sort(rng.choice(100, size=n_act, replace=False))
        p = np.zeros(100)
        p[act] = dbm_to_w(rng.uniform(-3.0, 3.0, size=n_act))
        fmts = [names[int(x)] for x in rng.integers(0, 3, size=100)]
        sp = spectrum_from(100, 0.1, 0.096, 0.04, p, fmts)
        n_sp = int(rng.integers(1, 31))
        lengths = rng.uniform(50.0, 120.0, size=n_sp)
        alpha = float(rng.uniform(0.17, 0.22))
        cr = float(rng.uniform(0.025, 0.032))
        link = Link(make_spans(lengths, alpha=alpha, cr=cr))
        out.append(Workload(f"batch_link_{li}", sp, link,
                            Numerics(n_grid=n_grid, egn=1, precision=PREC_FP32_PHASE64),
                            act.astype(np.int32)))
    return out


def sclband_150ch_40span(seed=5, n_grid=1024, precision=PREC_FP32_PHASE64):
    """S+C+L, 15 THz: 150 x 100 GBd on 100 GHz (roll-off 0), 24 dBm flat total,
    40 x 80 km spans with per-span fibre draws, dispersion slope on, formats
    cycling QPSK / 16QAM / 64QAM, every channel under test."""
    rng = np.random.default_rng(seed)
    n = 150
    p = np.full(n, dbm_to_w(24.0) / n)
    names = ["qpsk", "16qam", "64qam"]
    fmts = [names[k % 3] for k in range(n)]
    sp = spectrum_from(n, 0.1, 0.1, 0.0, p, fmts)
    ns = 40
    spans = make_spans(np.full(ns, 80.0),
                       alpha=rng.uniform(0.17, 0.22, ns),
                       beta2=rng.uniform(-23.0, -20.0, ns),
                       beta3=rng.uniform(0.12, 0.16, ns),
                       gamma=rng.uniform(1.2, 1.4, ns),
                       cr=rng.uniform(0.025, 0.032, ns))
    return Workload("sclband_150ch_40span", sp, Link(spans),
                    Numerics(n_grid=n_grid, egn=1, precision=precision),
                    np.arange(n, dtype=np.int32))


def table1_1thz(cr=1.12, n_spans=1, fmt="qpsk", n_grid=10):
    """The paper's Table I: 101 x 10 GBd on 10.1 GHz, 19 dBm total, 100 km spans,
    alpha 0.2 dB/km, D = 17 ps/nm/km (beta2 = -21.68 ps^2/km at 1550 nm), no
    slope, gamma 1.2, Cr 0.28 or 1.12.  Roll-off is not stated: 0 is used.
    n_grid = 10 gives the paper's 1 GHz integration resolution."""
    n = 101
    p = np.full(n, dbm_to_w(19.0) / n)
    sp = spectrum_from(n, 0.0101, 0.010, 0.0, p, [fmt] * n)
    beta2 = -17.0 * 1550.0 ** 2 / (2 * np.pi * 299792.458)  # ps^2/km (lambda nm, c nm/ps)
    link = Link(make_spans(np.full(n_spans, 100.0), alpha=0.2, beta2=beta2, beta3=0.0,
                           gamma=1.2, cr=cr))
    return Workload("table1_1thz", sp, link, Numerics(n_grid=n_grid, egn=1),
                    np.array([50], dtype=np.int32))


def table2_10thz(n_grid=16):
    """The paper's Table II: 101 x 100 GBd on 101 GHz, 25 dBm total, one 100 km span,
    Cr 0.028, D 17 ps/nm/km, S 0.067 ps/nm^2/km, gamma 1.2."""
    n = 101
    p = np.full(n, dbm_to_w(25.0) / n)
    sp = spectrum_from(n, 0.101, 0.100, 0.0, p, ["qpsk"] * n)
    lam = 1550.0
    c = 299792.458
    beta2 = -17.0 * lam ** 2 / (2 * np.pi * c)
    # beta3 = S lam^4 / (2 pi c)^2 + D lam^3 / (2 pi^2 c^2): ps^3/km
    beta3 = 0.067 * lam ** 4 / (2 * np.pi * c) ** 2 + 17.0 * lam ** 3 / (2 * np.pi ** 2 * c ** 2)
    link = Link(make_spans([100.0], alpha=0.2, beta2=beta2, beta3=beta3, gamma=1.2, cr=0.028))
    return Workload("table2_10thz", sp, link, Numerics(n_grid=n_grid, egn=1),
                    np.array([50], dtype=np.int32))


def small_mixed(seed=11, n_ch=7, n_spans=3, n_grid=40, rolloff=0.04, egn=1,
                precision=PREC_FP64, gain_mode=GAIN_EQUALIZED, rs=0.096):
    """A cheap stand-in with the C+L workload's structure (tilted powers, uneven
    spans, mixed formats, one inactive slot) for parity tests."""
    rng = np.random.default_rng(seed)
    p = dbm_to_w(rng.uniform(-2.0, 2.0, size=n_ch) + 10.0 * np.log10(100.0 / n_ch))
    if n_ch >= 6:
        p[n_ch - 2] = 0.0
    names = ["qpsk", "16qam", "64qam"]
    fmts = [names[k % 3] for k in range(n_ch)]
    sp = spectrum_from(n_ch, 0.1, rs, rolloff, p, fmts)
    spans = make_spans(rng.uniform(50.0, 100.0, n_spans),
                       alpha=rng.uniform(0.17, 0.22, n_spans),
                       beta2=rng.uniform(-23.0, -20.0, n_spans),
                       beta3=rng.uniform(0.12, 0.16, n_spans),
                       gamma=rng.uniform(1.2, 1.4, n_spans),
                       cr=rng.uniform(0.025, 0.032, n_spans))
    cuts = np.nonzero(p > 0)[0].astype(np.int32)
    return Workload("small_mixed", sp, Link(spans, gain_mode=gain_mode),
                    Numerics(n_grid=n_grid, egn=egn, precision=precision), cuts)
