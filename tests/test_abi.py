"""Host-side checks of the C-ABI library: it loads, exports every function the
header declares, and its pure-host validation rejects bad inputs.  No compute
call is made here (no GPU in this environment)."""
import ctypes as C
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from paper_2412_11614_amd import _lib, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "isrs_egn.h")


def _read(path):
    with open(path) as f:
        return f.read()


def _declared():
    src = _read(HEADER)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(isrs_[a-z_]+)\s*\(", src)))


def test_header_functions_are_exported():
    names = _declared()
    assert len(names) >= 16
    L = _lib.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", out), f"{n} not exported with C linkage"
    assert set(names) == set(_lib.EXPORTED)


def test_header_compiles_as_c():
    src = f'#include "{HEADER}"\nint main(void) {{ isrs_numerics n; (void)n; return 0; }}\n'
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-x", "c", "-", "-fsyntax-only"],
                       input=src, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_struct_layouts_match_header():
    # offsets the ctypes mirror relies on, checked against the C compiler
    prog = f'''#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
 printf("%zu %zu %zu %zu\\n", sizeof(isrs_spectrum), offsetof(isrs_spectrum, power_w), sizeof(isrs_span), sizeof(isrs_numerics));
 printf("%zu %zu %zu\\n", offsetof(isrs_numerics, n1), offsetof(isrs_numerics, mu_method), sizeof(isrs_stats));
 return 0; }}'''
    exe = "/tmp/isrs_layout_check"
    r = subprocess.run(["gcc", "-x", "c", "-", "-o", exe], input=prog, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    vals = subprocess.run([exe], capture_output=True, text=True).stdout.split()
    vals = [int(v) for v in vals]
    assert vals[0] == C.sizeof(_lib.Spectrum_c)
    assert vals[1] == _lib.Spectrum_c.power_w.offset
    assert vals[2] == C.sizeof(_lib.Span_c)
    assert vals[3] == C.sizeof(_lib.Numerics_c)
    assert vals[4] == _lib.Numerics_c.n1.offset
    assert vals[5] == _lib.Numerics_c.mu_method.offset
    assert vals[6] == C.sizeof(_lib.Stats_c)


def test_version_string():
    assert b"gfx950" in _lib.lib().isrs_version()


def test_validate_spectrum():
    wl = W.cl_100ch_10span()
    assert _lib.validate_spectrum(wl.spectrum) == _lib.ISRS_OK
    bad = W.cl_100ch_10span().spectrum
    bad.rolloff = 0.1          # 96 GBd * 1.1 > 100 GHz: overlapping channels
    assert _lib.validate_spectrum(bad) == _lib.ISRS_E_SPECTRUM
    bad = W.cl_100ch_10span().spectrum
    bad.power_w[3] = np.nan
    assert _lib.validate_spectrum(bad) == _lib.ISRS_E_SPECTRUM
    bad = W.cl_100ch_10span().spectrum
    bad.power_w[3] = -1e-3
    assert _lib.validate_spectrum(bad) == _lib.ISRS_E_SPECTRUM
    bad = W.cl_100ch_10span().spectrum
    bad.power_w[:] = 0.0
    assert _lib.validate_spectrum(bad) == _lib.ISRS_E_SPECTRUM
    bad = W.cl_100ch_10span().spectrum
    bad.symbol_rate_thz = 0.0
    assert _lib.validate_spectrum(bad) == _lib.ISRS_E_SPECTRUM
    bad = W.cl_100ch_10span().spectrum
    bad.phi[0] = np.inf
    assert _lib.validate_spectrum(bad) == _lib.ISRS_E_SPECTRUM
    assert _lib.lib().isrs_validate_spectrum(None) == _lib.ISRS_E_ARG


def test_validate_link():
    spans = W.make_spans([80.0, 90.0])
    assert _lib.validate_link(spans) == _lib.ISRS_OK
    assert _lib.validate_link(spans, gain_mode=1) == _lib.ISRS_OK
    assert _lib.validate_link(spans, gain_mode=7) == _lib.ISRS_E_LINK
    for field, val in [("length_km", 0.0), ("length_km", -5.0), ("alpha_db_km", 0.0),
                       ("beta2_ps2_km", np.nan), ("cr_w_km_thz", -0.1), ("gamma_w_km", np.inf)]:
        s = W.make_spans([80.0, 90.0])
        s[field][1] = val
        assert _lib.validate_link(s) == _lib.ISRS_E_LINK, field
    assert _lib.lib().isrs_validate_link(None, 1, 0) == _lib.ISRS_E_ARG


def test_validate_numerics():
    ok = _lib.numerics_struct(W.Numerics(n_grid=64))
    assert _lib.validate_numerics(ok) == _lib.ISRS_OK
    for kw in [dict(n=0), dict(n=9000), dict(n_f=0), dict(dz=0.0), dict(dz=float("nan")),
               dict(egn=2), dict(precision=5), dict(mu_method=3)]:
        nu = _lib.numerics_struct(W.Numerics(n_grid=64), **kw)
        assert _lib.validate_numerics(nu) == _lib.ISRS_E_ARG, kw
    nu = _lib.numerics_struct(W.Numerics(n_grid=64))
    nu.n2 = 32
    assert _lib.validate_numerics(nu) == _lib.ISRS_E_ARG


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(_lib.IsrsError) as ei:
        _lib.Engine(0)
    assert ei.value.code == _lib.ISRS_E_DEVICE
    assert _lib.lib().isrs_last_error(None)


def test_null_context_is_rejected():
    L = _lib.lib()
    assert L.isrs_destroy(None) == _lib.ISRS_E_ARG
    assert L.isrs_set_spectrum(None, None) == _lib.ISRS_E_ARG
    assert L.isrs_set_profiling(None, 1) == _lib.ISRS_E_ARG
    assert L.isrs_get_stats(None, None) == _lib.ISRS_E_ARG
    assert L.isrs_eval_eta(None, None, None, 0, None, None, None) == _lib.ISRS_E_ARG
    assert L.isrs_eval_islands(None, None, 0, None, 0, None) == _lib.ISRS_E_ARG
    assert L.isrs_last_error(None) is not None


def test_package_import_does_not_load_library():
    code = ("import sys; sys.path.insert(0, %r); import paper_2412_11614_amd as p; "
            "from paper_2412_11614_amd import _lib; print(_lib._lib is None)") % ROOT
    r = subprocess.run(["python", "-c", code], capture_output=True, text=True)
    assert r.stdout.strip() == "True", r.stderr


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.lib()


def test_product_code_never_touches_the_oracle():
    """The package (HIP path, binding, workloads) neither imports nor loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2412_11614_amd")
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle)|liboracle|isrs_oracle", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = _read(os.path.join(dirpath, f))
                assert not pat.search(txt), f


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message before
    touching a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
