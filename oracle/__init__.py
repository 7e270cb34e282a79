"""CPU oracle of the ISRS-aware EGN model (FP64, plain C, OpenMP over squares).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The GPU library never imports, links or
calls anything here, and nothing here imports the GPU library.

The arithmetic lives in ``isrs_oracle.c``; this module compiles it with gcc
and marshals numpy arrays through ctypes.  See the C file's header for the
equations it follows and the readings it takes where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "isrs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

MU_INTEGRAL = 0
MU_SEGMENT = 1
MU_MACLAURIN = 2
_METHODS = {"integral": MU_INTEGRAL, "segment": MU_SEGMENT, "maclaurin": MU_MACLAURIN}

GAIN_EQUALIZED = 0
GAIN_LOSS_ONLY = 1


class _Spectrum(C.Structure):
    _fields_ = [("n_ch", C.c_int), ("spacing", C.c_double), ("rs", C.c_double),
                ("rolloff", C.c_double), ("power", C.POINTER(C.c_double)),
                ("phi", C.POINTER(C.c_double)), ("psi", C.POINTER(C.c_double))]


class _Numerics(C.Structure):
    _fields_ = [("n_grid", C.c_int), ("n_f", C.c_int), ("dz", C.c_double), ("egn", C.c_int),
                ("mu_method", C.c_int), ("gain_mode", C.c_int), ("ptot_override", C.c_double)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = C.CDLL(_LIB)
            dp = C.POINTER(C.c_double)
            L.orc_eval_cut.argtypes = [C.POINTER(_Spectrum), dp, C.c_int, C.POINTER(_Numerics), C.c_int,
                                       dp, dp, dp, dp]
            L.orc_eval_cut.restype = C.c_int
            L.orc_square_terms.argtypes = [C.POINTER(_Spectrum), dp, C.c_int, C.POINTER(_Numerics),
                                           C.c_int, C.c_int, C.c_int, C.c_double, dp]
            L.orc_square_terms.restype = C.c_int
            L.orc_mu.argtypes = [dp, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double,
                                 C.c_double, C.c_double, dp]
            L.orc_mu.restype = None
            L.orc_upsilon.argtypes = [dp, C.c_int, C.c_double, C.c_double, C.c_int, C.c_double,
                                      C.c_int, C.c_double, C.c_double, C.c_double, dp]
            L.orc_upsilon.restype = None
            for name in ("orc_alpha_lin",):
                getattr(L, name).argtypes = [C.c_double]
                getattr(L, name).restype = C.c_double
            L.orc_leff.argtypes = [C.c_double, C.c_double]
            L.orc_leff.restype = C.c_double
            L.orc_srs_gain.argtypes = [C.c_double, C.c_double, C.c_double]
            L.orc_srs_gain.restype = C.c_double
            L.orc_rho.argtypes = [C.c_double] * 6
            L.orc_rho.restype = C.c_double
            L.orc_delta_rho_db.argtypes = [C.c_double] * 5
            L.orc_delta_rho_db.restype = C.c_double
            L.orc_S.argtypes = [C.c_double] * 3
            L.orc_S.restype = C.c_double
            L.orc_moments.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, dp]
            L.orc_moments.restype = None
            L.orc_gl_rule.argtypes = [dp, dp]
            L.orc_gl_rule.restype = None
            L.orc_format_constants.argtypes = [dp, dp, C.c_int, dp, dp]
            L.orc_format_constants.restype = None
            L.orc_domain_max_d1d2.argtypes = [C.POINTER(_Spectrum), C.c_int, C.c_int]
            L.orc_domain_max_d1d2.restype = C.c_double
            L.orc_phase_coef.argtypes = [C.c_double] * 5
            L.orc_phase_coef.restype = C.c_double
            L.orc_num_threads.argtypes = []
            L.orc_num_threads.restype = C.c_int
            _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class _Inputs:
    """Keeps the numpy buffers alive while C structs point into them."""

    def __init__(self, spectrum, link, numerics, method, n_grid=None):
        self.power = _f64(spectrum.power_w)
        self.phi = _f64(spectrum.phi)
        self.psi = _f64(spectrum.psi)
        self.spec = _Spectrum(int(spectrum.n_ch), float(spectrum.spacing_thz),
                              float(spectrum.symbol_rate_thz), float(spectrum.rolloff),
                              _dp(self.power), _dp(self.phi), _dp(self.psi))
        self.spans = span_array(link.spans)
        self.n_sp = self.spans.shape[0]
        self.nu = _Numerics(int(n_grid if n_grid is not None else numerics.n_grid), int(numerics.n_f),
                            float(numerics.dz_km), int(numerics.egn), _METHODS[method],
                            int(link.gain_mode), float(link.ptot_override_w))


def span_array(spans):
    """Structured span records -> contiguous [n, 6] float64
    (length, alpha_dB, beta2, beta3, gamma, Cr)."""
    if spans.dtype.names:
        cols = ["length_km", "alpha_db_km", "beta2_ps2_km", "beta3_ps3_km", "gamma_w_km", "cr_w_km_thz"]
        return np.ascontiguousarray(np.stack([np.asarray(spans[c], np.float64) for c in cols], axis=1))
    return _f64(spans).reshape(-1, 6)


def eval_cuts(workload, cuts=None, method="integral", n_grid=None, numerics=None):
    """sigma^2 [W], eta [1/W^2], per-term contributions [n_cut, 5] (D,E,F,G,H) and
    PSD samples [n_cut, n_f] for the CUTs of a workload."""
    nu = numerics if numerics is not None else workload.numerics
    inp = _Inputs(workload.spectrum, workload.link, nu, method, n_grid)
    cuts = np.asarray(workload.cuts if cuts is None else cuts, dtype=np.int64)
    n = len(cuts)
    s2 = np.zeros(n)
    eta = np.zeros(n)
    terms = np.zeros((n, 5))
    psd = np.zeros((n, inp.nu.n_f))
    L = lib()
    for q, c in enumerate(cuts):
        o_s2 = C.c_double()
        o_eta = C.c_double()
        t5 = np.zeros(5)
        ps = np.zeros(inp.nu.n_f)
        rc = L.orc_eval_cut(C.byref(inp.spec), _dp(inp.spans), inp.n_sp, C.byref(inp.nu), int(c),
                            C.byref(o_s2), C.byref(o_eta), _dp(t5), _dp(ps))
        if rc != 0:
            raise ValueError(f"oracle rejected inputs (cut {c})")
        s2[q], eta[q], terms[q], psd[q] = o_s2.value, o_eta.value, t5, ps
    return {"sigma2": s2, "eta": eta, "terms": terms, "psd": psd}


def square_terms(workload, cut, k1, k2, f=0.0, method="integral", n_grid=None, numerics=None):
    """Bare island integrals [3 (l=-1,0,1), 5 (D,E,F,G,H)] of one square."""
    nu = numerics if numerics is not None else workload.numerics
    inp = _Inputs(workload.spectrum, workload.link, nu, method, n_grid)
    out = np.zeros(15)
    rc = lib().orc_square_terms(C.byref(inp.spec), _dp(inp.spans), inp.n_sp, C.byref(inp.nu),
                                int(cut), int(k1), int(k2), float(f), _dp(out))
    if rc != 0:
        raise ValueError("oracle rejected inputs")
    return out.reshape(3, 5)


def mu(span, ptot, B, a, b, c, method="integral", dz=1.0):
    """FWM efficiency factor mu_s(a, b, c) of one span (Eq. 23 / Eqs. 8-10 / Eq. 4)."""
    sp = span_array(np.asarray(span).reshape(-1))[0] if hasattr(span, "dtype") else _f64(span)
    out = np.zeros(2)
    lib().orc_mu(_dp(sp), float(ptot), float(B), _METHODS[method], float(dz), float(a), float(b),
                 float(c), _dp(out))
    return complex(out[0], out[1])


def upsilon(spans, ptot, B, a, b, c, method="integral", dz=1.0, gain_mode=GAIN_EQUALIZED):
    """Link function Upsilon(a, b, c), Eq. 22."""
    sp = span_array(spans)
    out = np.zeros(2)
    lib().orc_upsilon(_dp(sp), sp.shape[0], float(ptot), float(B), _METHODS[method], float(dz),
                      int(gain_mode), float(a), float(b), float(c), _dp(out))
    return complex(out[0], out[1])


def alpha_lin(alpha_db):
    return lib().orc_alpha_lin(float(alpha_db))


def leff(alpha, z):
    return lib().orc_leff(float(alpha), float(z))


def srs_gain(X, f, B):
    return lib().orc_srs_gain(float(X), float(f), float(B))


def rho(alpha, cr, ptot, B, z, f):
    return lib().orc_rho(float(alpha), float(cr), float(ptot), float(B), float(z), float(f))


def delta_rho_db(ptot, cr, alpha, L, B):
    return lib().orc_delta_rho_db(float(ptot), float(cr), float(alpha), float(L), float(B))


def S(x, rs, rolloff):
    return lib().orc_S(float(x), float(rs), float(rolloff))


def moments(w, n=16, method="auto"):
    """Chebyshev moments int_{-1}^{1} T_k(t) exp(w t) dt, k = 0..n."""
    out = np.zeros(2 * (n + 1))
    m = {"gl": 0, "rec": 1}[method] if method != "auto" else (0 if abs(w) <= 20.0 else 1)
    lib().orc_moments(float(np.real(w)), float(np.imag(w)), int(n), m, _dp(out))
    return out[0::2] + 1j * out[1::2]


def gl_rule():
    x = np.zeros(64)
    w = np.zeros(64)
    lib().orc_gl_rule(_dp(x), _dp(w))
    return x, w


def format_constants(points):
    """(Phi, Psi) of a constellation given as complex points."""
    p = np.asarray(points, dtype=np.complex128)
    re, im = _f64(p.real), _f64(p.imag)
    phi, psi = C.c_double(), C.c_double()
    lib().orc_format_constants(_dp(re), _dp(im), len(p), C.byref(phi), C.byref(psi))
    return phi.value, psi.value


def domain_max_d1d2(spectrum, n_grid, cut):
    """max |(f1 - f)(f2 - f)| over the grid points of CUT `cut`'s islands (f = 0)."""
    inp = _Inputs(spectrum, _DummyLink(), _DummyNum(n_grid), "segment")
    return lib().orc_domain_max_d1d2(C.byref(inp.spec), int(n_grid), int(cut))


def phase_coef(beta2, beta3, a, b, c):
    """Phase-mismatch coefficient chi of Eqs. 5 / 24 in rad/km."""
    return lib().orc_phase_coef(float(beta2), float(beta3), float(a), float(b), float(c))


class _DummyLink:
    spans = np.array([[1.0, 0.2, -20.0, 0.0, 1.0, 0.0]])
    gain_mode = 0
    ptot_override_w = 0.0


class _DummyNum:
    def __init__(self, n):
        self.n_grid, self.n_f, self.dz_km, self.egn = n, 1, 1.0, 0


def num_threads():
    return lib().orc_num_threads()
