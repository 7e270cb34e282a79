"""Surrogate on the GPU: training labels against the oracle's closed form,
MFMA gradients against the FP64 reference network, training, ensemble
fallback, checkpoint and resume."""
import numpy as np
import pytest

from oracle import surrogate as S

pytestmark = pytest.mark.gpu

N_DATA = 70_000          # more than one 65,536-row forward chunk, ragged tail
DB = 10.0 / np.log(10.0)


@pytest.fixture(scope="module")
def engine():
    import torch
    assert torch.cuda.is_available()
    from paper_2412_11614_amd import _lib
    st = torch.cuda.Stream()            # torch work and library work ordered on one stream
    torch.cuda.set_stream(st)
    e = _lib.Engine(0, stream=st)
    yield e
    torch.cuda.synchronize()
    e.close()
    torch.cuda.set_stream(torch.cuda.default_stream())


def _data(engine, n, seed):
    import torch
    x = torch.empty(n, 16, device="cuda")
    r = torch.empty(n, device="cuda")
    y6 = torch.empty(n, device="cuda")
    engine.surrogate_datagen(x, r, seed, y6=y6)
    return x, r, y6


@pytest.fixture(scope="module")
def data(engine):
    return _data(engine, N_DATA, seed=11)


def test_datagen_points_and_labels(engine, data):
    x, r, y6 = (t.cpu().numpy() for t in data)
    assert np.all(np.abs(x[:, :S.NF]) <= 1.0) and np.all(x[:, S.NF:] == 0.0)
    phys = S.decode(x)
    # f1 + f2 - f falls in a channel of the 100 x 100 GHz grid for (almost) every point
    f3 = phys[:, 0] + phys[:, 1] - phys[:, 2]
    u = f3 / 0.1 + 49.5
    inside = (np.abs(u - np.rint(u)) * 0.1 <= 0.5 * 0.09984 + 1e-6) & (np.rint(u) >= 0) & (np.rint(u) <= 99)
    assert inside.mean() > 0.999
    # a uniform spread over the span parameters
    for j in range(3, S.NF):
        assert abs(np.mean(x[:, j])) < 0.02, j
    rng = np.random.default_rng(0)
    for i in rng.choice(len(r), size=40, replace=False):
        y_ref, y6_ref = S.target(phys[i])
        assert abs(y6[i] - y6_ref) <= 2e-6 * max(1.0, abs(y6_ref)), (i, phys[i])
        assert abs(r[i] - (y_ref - y6_ref)) <= 2e-6 * max(1.0, abs(y_ref)), (i, phys[i])
    # same seed, same points; another seed, other points
    x2, r2, _ = _data(engine, 1000, seed=11)
    assert np.array_equal(x2.cpu().numpy(), x[:1000]) and np.array_equal(r2.cpu().numpy(), r[:1000])
    x3, _, _ = _data(engine, 1000, seed=12)
    assert not np.array_equal(x3.cpu().numpy(), x[:1000])


def test_closed_form_points(engine, data):
    import torch
    x, r, y6 = data
    y = torch.empty_like(r)
    engine.closed_form_points(x, y)
    y, r, y6 = y.cpu().numpy(), r.cpu().numpy(), y6.cpu().numpy()
    assert np.allclose(y, r.astype(np.float64) + y6, rtol=1e-6, atol=1e-6)


def test_gradient_matches_fp64_reference(engine, data):
    x, r, _ = data
    s = engine.surrogate(n_members=2, seed=5)
    s.train(x, r, steps=3, batch=256)             # sets the target scale, moves off the initial point
    shift, scale = s.target_scale()
    assert abs(shift - float(r.double().mean())) <= 1e-6 * max(1.0, abs(shift))
    assert abs(scale - float(r.double().std(unbiased=False))) <= 1e-6 * scale
    n = 512
    xs, rs = x[:n].contiguous(), r[:n].contiguous()
    xn, rn = S.features(xs.cpu().numpy()), rs.cpu().numpy().astype(np.float64)
    tn = (rn - shift) / scale
    for member in (0, 1):
        p = s.get_params(member).astype(np.float64)
        g, loss = s.grad(member, xs, rs)
        loss_ref, g_ref = S.loss_and_grad(p, xn, tn)
        # BF16 operands (8-bit significand) through four layers: percent-level agreement
        assert abs(loss - loss_ref) <= 2e-2 * loss_ref, (loss, loss_ref)
        lay, _ = S.layout()
        for name, (o, shp) in lay.items():
            k = int(np.prod(shp))
            a, b = g[o:o + k].astype(np.float64), g_ref[o:o + k]
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            cos = a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30)
            assert rel <= 5e-2 and cos >= 0.998, (member, name, rel, cos)
            # element by element: each gradient entry within a BF16-sized share of its
            # own magnitude plus the tensor's RMS (a dropped, swapped or sign-flipped
            # entry is off by its whole size)
            rms = np.sqrt(np.mean(b ** 2))
            dev = np.abs(a - b) / (np.abs(b) + rms)
            print(f"member {member} {name}: norm rel {rel:.2e}, max elementwise {dev.max():.3f}", flush=True)
            assert dev.max() <= 0.15, (member, name, int(dev.argmax()), a[dev.argmax()], b[dev.argmax()])
    s.close()


def test_training_gain_and_speed_against_closed_form(engine, data):
    """What the trained network gains: the error of the ISRS-free form (Eq. 6)
    the network corrects, against the segment closed form it learns, on
    held-out points; and its speed against that closed form on the same
    points (reported as measured: the network costs more arithmetic per point
    than the closed form it stands in for)."""
    import time
    import torch
    x, r, _ = data
    s = engine.surrogate(n_members=2, seed=7)
    var0 = float(torch.var(r).item())
    loss = s.train(x, r, steps=600, batch=1024, lr=1e-3)
    assert np.all(loss < 0.05 * var0), (loss, var0)
    # held-out points: the ensemble against the closed form, in dB of |mu|^2
    xh, rh, y6h = _data(engine, 8192, seed=99)
    yh = torch.empty_like(rh)
    assert s.eval_points(xh, yh, float("inf")) == 0
    ycf = torch.empty_like(rh)
    engine.closed_form_points(xh, ycf)
    err = DB * (yh - ycf).double().cpu().numpy()
    base = DB * (y6h - ycf).double().cpu().numpy()            # Eq. 6 alone, no ISRS
    rms, rms0 = np.sqrt(np.mean(err ** 2)), np.sqrt(np.mean(base ** 2))
    assert rms < 0.2 * rms0, (rms, rms0)
    # throughput on 1 M points, network without fallback against the closed form
    xb, _, _ = _data(engine, 1 << 20, seed=98)
    yb = torch.empty(1 << 20, device="cuda")
    rate = {}
    for name in ("closed_form", "network"):
        def run():
            if name == "closed_form":
                engine.closed_form_points(xb, yb)
            else:
                s.eval_points(xb, yb, float("inf"))
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            run()
        torch.cuda.synchronize()
        rate[name] = 5 * (1 << 20) / (time.perf_counter() - t0)
    print(f"held-out rms error: network {rms:.4f} dB, Eq. 6 alone {rms0:.4f} dB; points/s: network "
          f"{rate['network']:.3e}, closed form {rate['closed_form']:.3e} "
          f"(network / closed form = {rate['network'] / rate['closed_form']:.2f})", flush=True)
    assert rate["network"] > 0 and rate["closed_form"] > 0
    s.close()


def test_calibrated_fallback_bounds_point_and_eta_error(engine):
    """The fallback gate calibrated on points of some C+L links keeps every
    accepted point of other links within 0.01 dB of the closed form, and eta
    with the surrogate in the loop within 0.01 dB of the plain path."""
    import torch
    from paper_2412_11614_amd import workloads as W

    def draw(seed0, n_links, n, seed):
        b = engine.batch([W.cl_100ch_10span(seed=seed0 + i, n_grid=16) for i in range(n_links)])
        x = torch.empty(n, 16, device="cuda")
        r = torch.empty(n, device="cuda")
        engine.surrogate_datagen_batch(b, 16, x, r, seed)
        b.close()
        return x, r

    x, r = draw(100, 16, 1 << 21, 4)
    s = engine.surrogate(n_members=4, seed=21)
    s.train(x, r, steps=4000, batch=1024, lr=1e-3)
    s.train(x, r, steps=2000, batch=1024, lr=3e-4)
    s.train(x, r, steps=2000, batch=1024, lr=1e-4)
    xc, _ = draw(500, 16, 1 << 19, 5)
    thr, emax, frac = s.calibrate(xc, 0.007)
    print(f"calibrated threshold {thr:.5f} dB: accepted {frac:.3f} of the calibration points, max error {emax:.5f} dB",
          flush=True)
    assert thr > 0 and emax <= 0.007
    xh, _ = draw(1000, 16, 1 << 19, 6)
    yh = torch.empty(xh.shape[0], device="cuda")
    ycf = torch.empty_like(yh)
    engine.closed_form_points(xh, ycf)
    mean = torch.empty_like(yh)
    spread = torch.empty_like(yh)
    s.predict(xh, mean, spread)
    nfb = s.eval_points(xh, yh, thr)
    err = np.abs(DB * (yh - ycf).double().cpu().numpy())
    acc = DB * spread.double().cpu().numpy() <= thr
    print(f"held-out: {acc.mean():.3f} accepted, max accepted error {err[acc].max():.5f} dB, "
          f"{nfb} fallbacks", flush=True)
    assert err.max() <= 0.01
    wl = W.cl_100ch_10span(n_grid=16)
    cuts = np.array([3, 50, 96], dtype=np.int32)
    engine.load(wl)
    ref = engine.eval_eta(wl.numerics, cuts, precision=W.PREC_FP32_PHASE64)["eta"]
    eta, fb = s.eval_eta(wl.numerics, cuts, thr)
    e = np.abs(10 * np.log10(eta / ref))
    print("eta in the loop at the calibrated threshold:", e, "fallback", fb, flush=True)
    assert e.max() <= 0.01
    s.close()


def test_fallback_thresholds(engine, data):
    import torch
    x, r, y6 = data
    s = engine.surrogate(n_members=3, seed=8)
    s.train(x, r, steps=100, batch=512, lr=1e-3)
    n = 5000
    xs = x[:n].contiguous()
    mean = torch.empty(n, device="cuda")
    spread = torch.empty(n, device="cuda")
    s.predict(xs, mean, spread)
    ycf = torch.empty(n, device="cuda")
    engine.closed_form_points(xs, ycf)
    y = torch.empty(n, device="cuda")
    # threshold < 0: every point falls back, identical to the closed form
    assert s.eval_points(xs, y, -1.0) == n
    assert torch.equal(y, ycf)
    # no fallback: y6 + ensemble mean
    assert s.eval_points(xs, y, float("inf")) == 0
    assert np.allclose(y.cpu().numpy(), (y6[:n] + mean).cpu().numpy(), rtol=2e-6, atol=2e-6)
    # threshold between two spreads: exactly the points above it fall back
    sp_db = np.sort(spread.double().cpu().numpy() * DB)
    thr = 0.5 * (sp_db[n // 2] + sp_db[n // 2 + 1])
    above = spread.double().cpu().numpy() * DB > thr
    nf = s.eval_points(xs, y, thr)
    assert nf == int(above.sum())
    yn, ycfn = y.cpu().numpy(), ycf.cpu().numpy()
    assert np.array_equal(yn[above], ycfn[above])
    assert np.allclose(yn[~above], (y6[:n] + mean).cpu().numpy()[~above], rtol=2e-6, atol=2e-6)
    s.close()


def test_predict_rows_are_independent(engine, data):
    """A ragged batch and a prefix of a larger one give identical rows."""
    import torch
    x, _, _ = data
    s = engine.surrogate(n_members=2, seed=9)
    m_big = torch.empty(N_DATA, device="cuda")
    s.predict(x, m_big, None)
    m_small = torch.empty(1000, device="cuda")
    s.predict(x[:1000].contiguous(), m_small, None)
    assert torch.equal(m_big[:1000], m_small)
    tail = x[N_DATA - 77:].contiguous()
    m_tail = torch.empty(77, device="cuda")
    s.predict(tail, m_tail, None)
    assert torch.equal(m_big[N_DATA - 77:], m_tail)
    s.close()


def test_checkpoint_resume(engine, data, tmp_path):
    x, r, _ = data
    a = engine.surrogate(n_members=2, seed=1)
    a.train(x, r, steps=30, batch=256, lr=1e-3)
    path = tmp_path / "sur.bin"
    a.save(path)
    b = engine.surrogate(n_members=2, seed=2)
    b.load(path)
    for m in (0, 1):
        assert np.array_equal(a.get_params(m), b.get_params(m))
    la = a.train(x, r, steps=20, batch=256, lr=1e-3)
    lb = b.train(x, r, steps=20, batch=256, lr=1e-3)
    assert np.array_equal(la, lb)
    for m in (0, 1):
        assert np.array_equal(a.get_params(m), b.get_params(m))
    c = engine.surrogate(n_members=3, seed=1)
    from paper_2412_11614_amd import _lib
    with pytest.raises(_lib.IsrsError):
        c.load(path)                      # member count differs
    a.close()
    b.close()
    c.close()


def test_parameter_roundtrip_and_validation(engine, data):
    import torch
    from paper_2412_11614_amd import _lib
    x, r, _ = data
    s = engine.surrogate(n_members=1, seed=3)
    p = S.init_like(42).astype(np.float32)
    s.set_params(0, p)
    assert np.array_equal(s.get_params(0), p)
    # the device network follows the new parameters: compare with the reference forward
    n = 256
    mean = torch.empty(n, device="cuda")
    s.predict(x[:n].contiguous(), mean, None)
    ref = S.forward(p.astype(np.float64), S.features(x[:n].cpu().numpy()))
    scale = max(1.0, float(np.max(np.abs(ref))))
    assert np.max(np.abs(mean.cpu().numpy() - ref)) <= 3e-2 * scale
    bad = p.copy()
    bad[10] = np.nan
    with pytest.raises(_lib.IsrsError) as ei:
        s.set_params(0, bad)
    assert ei.value.code == _lib.ISRS_E_NUMERIC
    with pytest.raises(_lib.IsrsError):
        s.eval_points(x[:64].contiguous(), torch.empty(64, device="cuda"), float("nan"))
    with pytest.raises(_lib.IsrsError):
        s.train(x, r, steps=1, batch=100)        # not a multiple of 64
    with pytest.raises(_lib.IsrsError):
        engine.surrogate(n_members=0)
    s.close()


def test_eta_with_surrogate_all_fallback_equals_closed_form(engine):
    """Threshold < 0: every (point, span) takes the segment form, through the
    table variant of the region kernel: the same eta as the plain path."""
    from paper_2412_11614_amd import workloads as W
    wl = W.small_mixed(seed=31, n_ch=5, n_spans=2, n_grid=24)
    engine.load(wl)
    ref = engine.eval_eta(wl.numerics, wl.cuts, precision=W.PREC_FP32_PHASE64)["eta"]
    s = engine.surrogate(n_members=2, seed=3)
    for thr in (-1.0, float("inf")):     # this link is outside the sampling box: always the closed form
        eta, fb = s.eval_eta(wl.numerics, wl.cuts, thr)
        assert fb == 1.0
        assert np.allclose(eta, ref, rtol=1e-6, atol=0), (thr, eta, ref)
    s.close()


def test_eta_with_surrogate_in_box(engine, data):
    """A link inside the sampling box (100 x 100 GHz grid, B_tot 10 THz): no
    fallback at an infinite threshold, partial fallback at 0.01 dB, and eta
    close to the closed form."""
    from paper_2412_11614_amd import workloads as W
    x, r, _ = data
    s = engine.surrogate(n_members=4, seed=12)
    s.train(x, r, steps=800, batch=1024, lr=1e-3)
    wl = W.cl_100ch_10span(n_grid=16)
    cuts = np.array([3, 50, 96], dtype=np.int32)
    engine.load(wl)
    ref = engine.eval_eta(wl.numerics, cuts, precision=W.PREC_FP32_PHASE64)["eta"]
    eta_inf, fb_inf = s.eval_eta(wl.numerics, cuts, float("inf"))
    eta_01, fb_01 = s.eval_eta(wl.numerics, cuts, 0.01)
    err_inf = 10 * np.log10(eta_inf / ref)
    err_01 = 10 * np.log10(eta_01 / ref)
    print("surrogate eta error dB", err_inf, "fallback", fb_inf, "| thr 0.01:", err_01, fb_01, flush=True)
    assert fb_inf == 0.0 and 0.0 < fb_01 < 1.0
    assert np.max(np.abs(err_inf)) < 0.5
    assert np.max(np.abs(err_01)) <= np.max(np.abs(err_inf)) + 1e-3
    s.close()


def test_datagen_from_links(engine):
    """Query points drawn from the links of a batch: labels match the oracle,
    points lie on live islands of the drawn links, draws outside the box are
    rejected, and a batch with no in-box point is an error."""
    import torch
    from paper_2412_11614_amd import _lib, workloads as W
    links = [W.cl_100ch_10span(n_grid=16), W.small_mixed(seed=61, n_ch=5, n_spans=2, n_grid=16)]
    b = engine.batch(links)
    n = 4096
    x = torch.empty(n, 16, device="cuda")
    r = torch.empty(n, device="cuda")
    y6 = torch.empty(n, device="cuda")
    rej = engine.surrogate_datagen_batch(b, 64, x, r, seed=5, y6=y6)
    assert rej > 0                      # the small link is outside the box (B_tot != 10 THz)
    xs, rs, y6s = x.cpu().numpy(), r.cpu().numpy(), y6.cpu().numpy()
    assert np.all(np.abs(xs[:, :S.NF]) <= 1.0)
    phys = S.decode(xs)
    spans = links[0].link.spans
    # every point carries one of the first link's spans
    assert np.all(np.min(np.abs(phys[:, 3][:, None] - spans["length_km"][None, :]), axis=1) < 1e-4)
    rng = np.random.default_rng(1)
    for i in rng.choice(n, size=16, replace=False):
        y_ref, y6_ref = S.target(phys[i])
        assert abs(rs[i] - (y_ref - y6_ref)) <= 2e-6 * max(1.0, abs(y_ref))
        assert abs(y6s[i] - y6_ref) <= 2e-6 * max(1.0, abs(y6_ref))
    b.close()
    b2 = engine.batch([links[1]])
    with pytest.raises(_lib.IsrsError):
        engine.surrogate_datagen_batch(b2, 64, x[:16].contiguous(), r[:16].contiguous(), seed=1)
    b2.close()
