"""ctypes binding of libisrs_egn.so (argument marshalling only).

Every step of the computation runs in the HIP library; this module converts
numpy arrays and torch device tensors into the plain pointers and structs of
include/isrs_egn.h.  It raises when the library is missing: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisrs_egn.so")

ISRS_OK = 0
ISRS_E_ARG = -1
ISRS_E_SPECTRUM = -2
ISRS_E_LINK = -3
ISRS_E_STATE = -4
ISRS_E_DEVICE = -5
ISRS_E_NOMEM = -6
ISRS_E_NUMERIC = -7

STATUS_NAMES = {0: "ISRS_OK", -1: "ISRS_E_ARG", -2: "ISRS_E_SPECTRUM", -3: "ISRS_E_LINK",
                -4: "ISRS_E_STATE", -5: "ISRS_E_DEVICE", -6: "ISRS_E_NOMEM", -7: "ISRS_E_NUMERIC"}

EXPORTED = [
    "isrs_create", "isrs_destroy", "isrs_last_error", "isrs_set_spectrum", "isrs_set_link",
    "isrs_set_ptot_override", "isrs_eval_eta", "isrs_eval_eta_dev", "isrs_eval_psd",
    "isrs_eval_islands", "isrs_set_profiling", "isrs_get_stats", "isrs_validate_spectrum",
    "isrs_validate_link", "isrs_validate_numerics", "isrs_version",
    "isrs_batch_create", "isrs_batch_destroy", "isrs_batch_num_cuts", "isrs_batch_eval",
    "isrs_batch_eval_dev", "isrs_autotune", "isrs_batch_get_tuning",
    "isrs_surrogate_create", "isrs_surrogate_destroy", "isrs_surrogate_datagen", "isrs_surrogate_train",
    "isrs_surrogate_predict", "isrs_surrogate_eval_points", "isrs_closed_form_points",
    "isrs_surrogate_num_params", "isrs_surrogate_get_params", "isrs_surrogate_set_params",
    "isrs_surrogate_grad", "isrs_surrogate_save", "isrs_surrogate_load", "isrs_surrogate_get_target_scale",
    "isrs_eval_eta_surrogate", "isrs_eval_eta_dz", "isrs_choose_dz", "isrs_surrogate_datagen_batch",
    "isrs_eval_eta_dev_noalloc", "isrs_surrogate_calibrate",
]

SUR_FEATURES = 16
SUR_HIDDEN = 256


class IsrsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Spectrum_c(C.Structure):
    _fields_ = [("n_ch", C.c_int32), ("f_center_thz", C.c_double), ("spacing_thz", C.c_double),
                ("symbol_rate_thz", C.c_double), ("rolloff", C.c_double),
                ("power_w", C.POINTER(C.c_double)), ("phi", C.POINTER(C.c_double)),
                ("psi", C.POINTER(C.c_double))]


class Span_c(C.Structure):
    _fields_ = [("length_km", C.c_double), ("alpha_db_km", C.c_double), ("beta2_ps2_km", C.c_double),
                ("beta3_ps3_km", C.c_double), ("gamma_w_km", C.c_double), ("cr_w_km_thz", C.c_double)]


class Numerics_c(C.Structure):
    _fields_ = [("dz_km", C.c_double), ("n1", C.c_int32), ("n2", C.c_int32), ("n_f", C.c_int32),
                ("egn", C.c_int32), ("precision", C.c_int32), ("mu_method", C.c_int32)]


class LinkBatch_c(C.Structure):
    _fields_ = [("n_links", C.c_int32), ("ch_offset", C.POINTER(C.c_int32)),
                ("span_offset", C.POINTER(C.c_int32)), ("cut_offset", C.POINTER(C.c_int32)),
                ("cuts", C.POINTER(C.c_int32)), ("spacing_thz", C.POINTER(C.c_double)),
                ("symbol_rate_thz", C.POINTER(C.c_double)), ("rolloff", C.POINTER(C.c_double)),
                ("gain_mode", C.POINTER(C.c_int32)), ("power_w", C.POINTER(C.c_double)),
                ("phi", C.POINTER(C.c_double)), ("psi", C.POINTER(C.c_double)),
                ("spans", C.c_void_p)]


class TrainOpts_c(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("member", C.c_int32)]


class Stats_c(C.Structure):
    _fields_ = [("region_ms", C.c_double), ("egn_ms", C.c_double), ("assemble_ms", C.c_double),
                ("host_prep_ms", C.c_double), ("region_launches", C.c_int64), ("n_squares", C.c_int64),
                ("n_delta_squares", C.c_int64), ("n_points_live", C.c_int64), ("horner_steps", C.c_int64),
                ("alg_flop", C.c_double)]


_lib = None


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2412_11614_amd.build "
                           "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    L.isrs_create.argtypes = [C.POINTER(vp), C.c_int32, vp]
    L.isrs_destroy.argtypes = [vp]
    L.isrs_last_error.argtypes = [vp]
    L.isrs_last_error.restype = C.c_char_p
    L.isrs_set_spectrum.argtypes = [vp, C.POINTER(Spectrum_c)]
    L.isrs_set_link.argtypes = [vp, C.POINTER(Span_c), C.c_int32, C.c_int32]
    L.isrs_set_ptot_override.argtypes = [vp, C.c_double]
    L.isrs_eval_eta.argtypes = [vp, C.POINTER(Numerics_c), ip, C.c_int32, dp, dp, dp]
    L.isrs_eval_eta_dev.argtypes = [vp, C.POINTER(Numerics_c), ip, C.c_int32, vp, vp, vp]
    L.isrs_eval_eta_dev_noalloc.argtypes = [vp, C.POINTER(Numerics_c), ip, C.c_int32, vp, vp, vp]
    L.isrs_eval_psd.argtypes = [vp, C.POINTER(Numerics_c), ip, C.c_int32, dp, dp]
    L.isrs_eval_islands.argtypes = [vp, C.POINTER(Numerics_c), C.c_int32, ip, C.c_int32, dp]
    L.isrs_set_profiling.argtypes = [vp, C.c_int32]
    L.isrs_get_stats.argtypes = [vp, C.POINTER(Stats_c)]
    L.isrs_validate_spectrum.argtypes = [C.POINTER(Spectrum_c)]
    L.isrs_validate_link.argtypes = [C.POINTER(Span_c), C.c_int32, C.c_int32]
    L.isrs_validate_numerics.argtypes = [C.POINTER(Numerics_c)]
    L.isrs_version.argtypes = []
    L.isrs_version.restype = C.c_char_p
    L.isrs_batch_create.argtypes = [vp, C.POINTER(LinkBatch_c), C.POINTER(vp)]
    L.isrs_batch_destroy.argtypes = [vp]
    L.isrs_batch_num_cuts.argtypes = [vp, C.POINTER(C.c_int64)]
    L.isrs_batch_eval.argtypes = [vp, vp, C.POINTER(Numerics_c), dp]
    L.isrs_batch_eval_dev.argtypes = [vp, vp, C.POINTER(Numerics_c), vp]
    L.isrs_autotune.argtypes = [vp, vp, C.POINTER(Numerics_c), C.c_char_p]
    L.isrs_batch_get_tuning.argtypes = [vp, ip, ip, ip, ip, ip]
    fp = C.POINTER(C.c_float)
    L.isrs_surrogate_create.argtypes = [vp, C.c_int32, C.c_uint64, C.POINTER(vp)]
    L.isrs_surrogate_destroy.argtypes = [vp]
    L.isrs_surrogate_datagen.argtypes = [vp, C.c_int64, C.c_uint64, vp, vp, vp]
    L.isrs_surrogate_train.argtypes = [vp, vp, vp, vp, C.c_int64, C.POINTER(TrainOpts_c), dp]
    L.isrs_surrogate_predict.argtypes = [vp, vp, vp, C.c_int64, vp, vp]
    L.isrs_surrogate_eval_points.argtypes = [vp, vp, vp, C.c_int64, C.c_double, vp, C.POINTER(C.c_int64)]
    L.isrs_closed_form_points.argtypes = [vp, vp, C.c_int64, vp]
    L.isrs_surrogate_calibrate.argtypes = [vp, vp, vp, C.c_int64, C.c_double, dp, dp, dp]
    L.isrs_surrogate_num_params.argtypes = [C.POINTER(C.c_int64)]
    L.isrs_surrogate_get_params.argtypes = [vp, C.c_int32, fp]
    L.isrs_surrogate_set_params.argtypes = [vp, vp, C.c_int32, fp]
    L.isrs_surrogate_grad.argtypes = [vp, vp, C.c_int32, vp, vp, C.c_int64, fp, dp]
    L.isrs_surrogate_save.argtypes = [vp, C.c_char_p]
    L.isrs_surrogate_load.argtypes = [vp, vp, C.c_char_p]
    L.isrs_surrogate_get_target_scale.argtypes = [vp, dp, dp]
    L.isrs_surrogate_datagen_batch.argtypes = [vp, vp, C.c_int32, C.c_int64, C.c_uint64, vp, vp, vp,
                                               C.POINTER(C.c_int64)]
    L.isrs_eval_eta_dz.argtypes = [vp, C.POINTER(Numerics_c), ip, C.c_int32, dp, dp, dp, dp]
    L.isrs_choose_dz.argtypes = [vp, C.POINTER(Numerics_c), ip, C.c_int32, dp, C.c_int32, C.c_double, dp, dp]
    L.isrs_eval_eta_surrogate.argtypes = [vp, vp, C.POINTER(Numerics_c), ip, C.c_int32, C.c_double, dp, dp]
    for name in EXPORTED:
        f = getattr(L, name)
        if f.restype is C.c_int:  # default
            f.restype = C.c_int32
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class _SpectrumArgs:
    def __init__(self, spectrum):
        self.p = _f64(spectrum.power_w)
        self.phi = _f64(spectrum.phi)
        self.psi = _f64(spectrum.psi)
        self.c = Spectrum_c(int(spectrum.n_ch), float(getattr(spectrum, "f_center_thz", 193.4)),
                            float(spectrum.spacing_thz), float(spectrum.symbol_rate_thz),
                            float(spectrum.rolloff), _dp(self.p), _dp(self.phi), _dp(self.psi))


def span_structs(spans):
    """Structured span records (or an [n, 6] array) -> ctypes array of Span_c."""
    if getattr(spans, "dtype", None) is not None and spans.dtype.names:
        cols = ["length_km", "alpha_db_km", "beta2_ps2_km", "beta3_ps3_km", "gamma_w_km", "cr_w_km_thz"]
        arr = np.stack([np.asarray(spans[c], np.float64) for c in cols], axis=1)
    else:
        arr = _f64(spans).reshape(-1, 6)
    out = (Span_c * arr.shape[0])()
    for i, row in enumerate(arr):
        out[i] = Span_c(*[float(x) for x in row])
    return out


def numerics_struct(numerics, **override):
    d = dict(n=int(numerics.n_grid), n_f=int(numerics.n_f), dz=float(numerics.dz_km),
             egn=int(numerics.egn), precision=int(numerics.precision),
             mu_method=int(getattr(numerics, "mu_method", 0)))
    d.update(override)
    return Numerics_c(d["dz"], d["n"], d["n"], d["n_f"], d["egn"], d["precision"], d["mu_method"])


def validate_spectrum(spectrum):
    a = _SpectrumArgs(spectrum)
    return lib().isrs_validate_spectrum(C.byref(a.c))


def validate_link(spans, gain_mode=0):
    s = span_structs(spans)
    return lib().isrs_validate_link(s, len(s), int(gain_mode))


def validate_numerics(numerics):
    n = numerics if isinstance(numerics, Numerics_c) else numerics_struct(numerics)
    return lib().isrs_validate_numerics(C.byref(n))


class _BatchArgs:
    """CSR packing of a list of workloads.Workload into isrs_link_batch."""

    def __init__(self, workloads):
        n = len(workloads)
        ch, sp, cu = [0], [0], [0]
        spacing, rs, ro, gm = [], [], [], []
        power, phi, psi, cuts, spans = [], [], [], [], []
        for w in workloads:
            s = w.spectrum
            power.append(_f64(s.power_w))
            phi.append(_f64(s.phi))
            psi.append(_f64(s.psi))
            ch.append(ch[-1] + int(s.n_ch))
            spacing.append(s.spacing_thz)
            rs.append(s.symbol_rate_thz)
            ro.append(s.rolloff)
            gm.append(int(w.link.gain_mode))
            sarr = span_structs(w.link.spans)
            spans.extend(sarr)
            sp.append(sp[-1] + len(sarr))
            c = np.asarray(w.cuts, dtype=np.int32)
            cuts.append(c)
            cu.append(cu[-1] + len(c))
        self.ch = np.asarray(ch, np.int32)
        self.sp = np.asarray(sp, np.int32)
        self.cu = np.asarray(cu, np.int32)
        self.cuts = np.ascontiguousarray(np.concatenate(cuts).astype(np.int32))
        self.spacing = _f64(spacing)
        self.rs = _f64(rs)
        self.ro = _f64(ro)
        self.gm = np.asarray(gm, np.int32)
        self.power = _f64(np.concatenate(power))
        self.phi = _f64(np.concatenate(phi))
        self.psi = _f64(np.concatenate(psi))
        self.spans = (Span_c * len(spans))(*spans)
        self.c = LinkBatch_c(n, _ip(self.ch), _ip(self.sp), _ip(self.cu), _ip(self.cuts), _dp(self.spacing),
                             _dp(self.rs), _dp(self.ro), _ip(self.gm), _dp(self.power), _dp(self.phi),
                             _dp(self.psi), C.cast(self.spans, C.c_void_p))
        self.n_cuts = int(self.cu[-1])


class Batch:
    """Many links evaluated through one work queue (isrs_batch_*)."""

    def __init__(self, engine, workloads):
        self._e = engine
        self._args = _BatchArgs(workloads)
        self._h = C.c_void_p()
        engine._check(engine._L.isrs_batch_create(engine._h, C.byref(self._args.c), C.byref(self._h)))
        n = C.c_int64()
        engine._check(engine._L.isrs_batch_num_cuts(self._h, C.byref(n)))
        self.n_cuts = int(n.value)
        self.cut_offset = self._args.cu.copy()

    def close(self):
        if self._h:
            self._e._L.isrs_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eval(self, numerics, **override):
        nu = numerics if isinstance(numerics, Numerics_c) else numerics_struct(numerics, **override)
        out = np.zeros(self.n_cuts)
        self._e._check(self._e._L.isrs_batch_eval(self._e._h, self._h, C.byref(nu), _dp(out)))
        return out

    def eval_dev(self, numerics, eta_dev, **override):
        nu = numerics if isinstance(numerics, Numerics_c) else numerics_struct(numerics, **override)
        if str(eta_dev.dtype) != "torch.float64" or not eta_dev.is_cuda or eta_dev.numel() < self.n_cuts:
            raise ValueError("eta_dev must be a float64 GPU tensor with n_cuts elements")
        self._e._check(self._e._L.isrs_batch_eval_dev(self._e._h, self._h, C.byref(nu), C.c_void_p(eta_dev.data_ptr())))

    def autotune(self, numerics, cache_path=None, **override):
        nu = numerics if isinstance(numerics, Numerics_c) else numerics_struct(numerics, **override)
        p = cache_path.encode() if cache_path else None
        self._e._check(self._e._L.isrs_autotune(self._e._h, self._h, C.byref(nu), p))
        return self.tuning()

    def tuning(self):
        v = [C.c_int32() for _ in range(5)]
        self._e._check(self._e._L.isrs_batch_get_tuning(self._h, *[C.byref(x) for x in v]))
        return {"mode": v[0].value, "blocks_per_cu": v[1].value, "sort": v[2].value, "slices": v[3].value,
                "points_per_run": v[4].value}


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _dev(t, dtype, n):
    """Device pointer of a contiguous torch GPU tensor with at least n elements."""
    if t is None:
        return None
    if str(t.dtype) != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"expected a contiguous {dtype} GPU tensor with at least {n} elements")
    return C.c_void_p(t.data_ptr())


class Surrogate:
    """MLP ensemble of the per-span FWM efficiency (isrs_surrogate_*).

    Query points are float32 device tensors [n, 16] of scaled features."""

    def __init__(self, engine, n_members=4, seed=0):
        self._e = engine
        self._h = C.c_void_p()
        engine._check(engine._L.isrs_surrogate_create(engine._h, int(n_members), int(seed), C.byref(self._h)))
        self.n_members = int(n_members)
        n = C.c_int64()
        engine._check(engine._L.isrs_surrogate_num_params(C.byref(n)))
        self.n_params = int(n.value)

    def close(self):
        if self._h:
            self._e._L.isrs_surrogate_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def train(self, x, r, steps, batch=1024, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, member=-1):
        n = r.numel()
        o = TrainOpts_c(int(steps), int(batch), float(lr), float(beta1), float(beta2), float(eps), int(member))
        loss = np.zeros(self.n_members)
        self._e._check(self._e._L.isrs_surrogate_train(self._e._h, self._h, _dev(x, "torch.float32", 16 * n),
                                                       _dev(r, "torch.float32", n), n, C.byref(o), _dp(loss)))
        return loss

    def predict(self, x, mean=None, spread=None):
        n = x.numel() // SUR_FEATURES
        self._e._check(self._e._L.isrs_surrogate_predict(self._e._h, self._h, _dev(x, "torch.float32", 16 * n), n,
                                                         _dev(mean, "torch.float32", n),
                                                         _dev(spread, "torch.float32", n)))

    def eval_points(self, x, y, spread_db_threshold):
        n = x.numel() // SUR_FEATURES
        nf = C.c_int64()
        self._e._check(self._e._L.isrs_surrogate_eval_points(
            self._e._h, self._h, _dev(x, "torch.float32", 16 * n), n, float(spread_db_threshold),
            _dev(y, "torch.float32", n), C.byref(nf)))
        return int(nf.value)

    def calibrate(self, x, target_db):
        """Fallback threshold from labelled points x: returns (threshold_db,
        max accepted error dB, accepted fraction)."""
        n = x.numel() // SUR_FEATURES
        t, e, f = C.c_double(), C.c_double(), C.c_double()
        self._e._check(self._e._L.isrs_surrogate_calibrate(self._e._h, self._h, _dev(x, "torch.float32", 16 * n), n,
                                                           float(target_db), C.byref(t), C.byref(e), C.byref(f)))
        return t.value, e.value, f.value

    def get_params(self, member):
        p = np.zeros(self.n_params, dtype=np.float32)
        self._e._check(self._e._L.isrs_surrogate_get_params(self._h, int(member), _fp(p)))
        return p

    def set_params(self, member, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if p.size != self.n_params:
            raise ValueError("wrong parameter count")
        self._e._check(self._e._L.isrs_surrogate_set_params(self._e._h, self._h, int(member), _fp(p)))

    def grad(self, member, x, r):
        n = r.numel()
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = C.c_double()
        self._e._check(self._e._L.isrs_surrogate_grad(self._e._h, self._h, int(member),
                                                      _dev(x, "torch.float32", 16 * n),
                                                      _dev(r, "torch.float32", n), n, _fp(g), C.byref(loss)))
        return g, loss.value

    def eval_eta(self, numerics, cuts, spread_db_threshold, **override):
        """eta of the engine's loaded link with the surrogate in the loop;
        returns (eta, fallback_fraction)."""
        nu = numerics if isinstance(numerics, Numerics_c) else numerics_struct(numerics, **override)
        cuts = np.ascontiguousarray(np.asarray(cuts, dtype=np.int32))
        eta = np.zeros(len(cuts))
        fb = C.c_double()
        self._e._check(self._e._L.isrs_eval_eta_surrogate(self._e._h, self._h, C.byref(nu), _ip(cuts), len(cuts),
                                                          float(spread_db_threshold), _dp(eta), C.byref(fb)))
        return eta, fb.value

    def target_scale(self):
        """(shift, scale): the network's raw output predicts (r - shift) / scale."""
        a, b = C.c_double(), C.c_double()
        self._e._check(self._e._L.isrs_surrogate_get_target_scale(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def save(self, path):
        self._e._check(self._e._L.isrs_surrogate_save(self._h, str(path).encode()))

    def load(self, path):
        self._e._check(self._e._L.isrs_surrogate_load(self._e._h, self._h, str(path).encode()))


@dataclass
class Stats:
    region_ms: float
    egn_ms: float
    assemble_ms: float
    host_prep_ms: float
    region_launches: int
    n_squares: int
    n_delta_squares: int
    n_points_live: int
    horner_steps: int
    alg_flop: float


class Engine:
    """One library context on one GPU.  Mirrors the C-ABI calls."""

    def __init__(self, device: int = 0, stream=None):
        """stream: None (the library's own stream), a hipStream_t handle or a
        torch.cuda.Stream.  The null stream cannot be shared: a NULL handle
        means "own stream" in the C-ABI, whose work would then not be ordered
        with the caller's."""
        L = lib()
        self._h = C.c_void_p()
        s = None
        if stream is not None:
            h = int(getattr(stream, "cuda_stream", stream))
            if h == 0:
                raise ValueError("pass a created stream (e.g. torch.cuda.Stream()) or None, not the null stream")
            s = C.c_void_p(h)
        rc = L.isrs_create(C.byref(self._h), int(device), s)
        if rc != ISRS_OK:
            raise IsrsError(rc, L.isrs_last_error(None).decode())
        self._L = L

    def close(self):
        if self._h:
            self._L.isrs_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc):
        if rc != ISRS_OK:
            raise IsrsError(rc, self._L.isrs_last_error(self._h).decode())

    def set_spectrum(self, spectrum):
        a = _SpectrumArgs(spectrum)
        self._check(self._L.isrs_set_spectrum(self._h, C.byref(a.c)))

    def set_link(self, spans, gain_mode=0):
        s = span_structs(spans)
        self._check(self._L.isrs_set_link(self._h, s, len(s), int(gain_mode)))

    def set_ptot_override(self, w):
        self._check(self._L.isrs_set_ptot_override(self._h, float(w)))

    def set_profiling(self, on=True):
        self._check(self._L.isrs_set_profiling(self._h, 1 if on else 0))

    def load(self, workload):
        """set_spectrum + set_link (+ ptot override) from a workloads.Workload."""
        self.set_spectrum(workload.spectrum)
        self.set_link(workload.link.spans, workload.link.gain_mode)
        self.set_ptot_override(workload.link.ptot_override_w)

    def eval_eta(self, numerics, cuts, **override):
        nu = numerics if isinstance(numerics, Numerics_c) else numerics_struct(numerics, **override)
        cuts = np.ascontiguousarray(np.asarray(cuts, dtype=np.int32))
        n = len(cuts)
        eta = np.zeros(n)
        s2 = np.zeros(n)
        terms = np.zeros((n, 5))
        self._check(self._L.isrs_eval_eta(self._h, C.byref(nu), _ip(cuts), n, _dp(eta), _dp(s2), _dp(terms)))
        return {"eta": eta, "sigma2": s2, "terms": terms}

    def eval_eta_dz(self, numerics, cuts, dz_km, **override):
        """eta with a sampling step per CUT (dz_km[q] for cuts[q])."""
        nu = numerics if isinstance(numerics, Numerics_c) else numerics_struct(numerics, **override)
        cuts = np.ascontiguousarray(np.asarray(cuts, dtype=np.int32))
        dz = np.ascontiguousarray(np.asarray(dz_km, dtype=np.float64))
        if dz.shape != cuts.shape:
            raise ValueError("one step per CUT")
        n = len(cuts)
        eta, s2, terms = np.zeros(n), np.zeros(n), np.zeros((n, 5))
        self._check(self._L.isrs_eval_eta_dz(self._h, C.byref(nu), _ip(cuts), n, _dp(dz), _dp(eta), _dp(s2),
                                             _dp(terms)))
        return {"eta": eta, "sigma2": s2, "terms": terms}

    def choose_dz(self, numerics, cuts, candidates, target_db, **override):
        """Per-CUT step from the error model; returns (dz [n_cut], err_db [n_cand, n_cut])."""
        nu = numerics if isinstance(numerics, Numerics_c) else numerics_struct(numerics, **override)
        cuts = np.ascontiguousarray(np.asarray(cuts, dtype=np.int32))
        cand = np.ascontiguousarray(np.asarray(candidates, dtype=np.float64))
        dz = np.zeros(len(cuts))
        err = np.zeros((len(cand), len(cuts)))
        self._check(self._L.isrs_choose_dz(self._h, C.byref(nu), _ip(cuts), len(cuts), _dp(cand), len(cand),
                                           float(target_db), _dp(dz), _dp(err)))
        return dz, err

    def eval_eta_dev(self, numerics, cuts, eta_dev, sigma2_dev=None, terms_dev=None, noalloc=False, **override):
        """Device outputs (torch tensors of float64 on the context's GPU); stream-ordered.
        noalloc=True calls isrs_eval_eta_dev_noalloc (device scratch from the library's fixed array)."""
        nu = numerics if isinstance(numerics, Numerics_c) else numerics_struct(numerics, **override)
        cuts = np.ascontiguousarray(np.asarray(cuts, dtype=np.int32))
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
        for t in (eta_dev, sigma2_dev, terms_dev):
            if t is not None and (str(t.dtype) != "torch.float64" or not t.is_cuda or not t.is_contiguous()):
                raise ValueError("device outputs must be contiguous float64 GPU tensors")
        if eta_dev.numel() < len(cuts):
            raise ValueError("eta_dev too small")
        if sigma2_dev is not None and sigma2_dev.numel() < len(cuts):
            raise ValueError("sigma2_dev too small")
        if terms_dev is not None and terms_dev.numel() < 5 * len(cuts):
            raise ValueError("terms_dev too small")
        fn = self._L.isrs_eval_eta_dev_noalloc if noalloc else self._L.isrs_eval_eta_dev
        self._check(fn(self._h, C.byref(nu), _ip(cuts), len(cuts), ptr(eta_dev), ptr(sigma2_dev), ptr(terms_dev)))

    def eval_psd(self, numerics, cuts, **override):
        nu = numerics if isinstance(numerics, Numerics_c) else numerics_struct(numerics, **override)
        cuts = np.ascontiguousarray(np.asarray(cuts, dtype=np.int32))
        n = len(cuts)
        f = np.zeros((n, nu.n_f))
        psd = np.zeros((n, nu.n_f))
        self._check(self._L.isrs_eval_psd(self._h, C.byref(nu), _ip(cuts), n, _dp(f), _dp(psd)))
        return f, psd

    def eval_islands(self, numerics, cut, squares, **override):
        """Bare D, E, F, G, H per island: array [m, 3 (l = -1, 0, 1), 5]."""
        nu = numerics if isinstance(numerics, Numerics_c) else numerics_struct(numerics, **override)
        sq = np.ascontiguousarray(np.asarray(squares, dtype=np.int32).reshape(-1, 2))
        m = sq.shape[0]
        out = np.zeros(m * 15)
        self._check(self._L.isrs_eval_islands(self._h, C.byref(nu), int(cut), _ip(sq), m, _dp(out)))
        return out.reshape(m, 3, 5)

    def batch(self, workloads):
        return Batch(self, workloads)

    def surrogate(self, n_members=4, seed=0):
        return Surrogate(self, n_members, seed)

    def surrogate_datagen(self, x, r, seed, y6=None):
        """Fills x [n, 16], r [n] (and y6 [n]) with labelled query points."""
        n = r.numel()
        self._check(self._L.isrs_surrogate_datagen(self._h, n, int(seed), _dev(x, "torch.float32", 16 * n),
                                                   _dev(r, "torch.float32", n), _dev(y6, "torch.float32", n)))

    def surrogate_datagen_batch(self, batch, n_grid, x, r, seed, y6=None):
        """Fills x [n, 16], r [n] (and y6) with query points drawn from the links
        of a Batch; returns the number of draws rejected as outside the box."""
        n = r.numel()
        rej = C.c_int64()
        self._check(self._L.isrs_surrogate_datagen_batch(self._h, batch._h, int(n_grid), n, int(seed),
                                                         _dev(x, "torch.float32", 16 * n), _dev(r, "torch.float32", n),
                                                         _dev(y6, "torch.float32", n), C.byref(rej)))
        return int(rej.value)

    def closed_form_points(self, x, y):
        n = x.numel() // SUR_FEATURES
        self._check(self._L.isrs_closed_form_points(self._h, _dev(x, "torch.float32", 16 * n), n,
                                                    _dev(y, "torch.float32", n)))

    def stats(self) -> Stats:
        s = Stats_c()
        self._check(self._L.isrs_get_stats(self._h, C.byref(s)))
        return Stats(*[getattr(s, f[0]) for f in Stats_c._fields_])
