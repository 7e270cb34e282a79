// isrs_api.cpp -- host side of the C-ABI declared in include/isrs_egn.h.
//
// Validates inputs, builds the per-span segment tables (Eqs. 8-10, 25), the
// per-anti-diagonal island tables (Eq. 16 on the grid), the f1 <-> f2 folded
// work list of channel-pair squares, and launches the gfx950 kernels on the
// context's stream.  No model arithmetic runs on the CPU beyond these tables:
// every grid point is evaluated on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/isrs_egn.h"
#include "isrs_internal.h"

using namespace isrs;

namespace {

constexpr int MAX_SPANS = 4096;
constexpr int MAX_GRID = 8192;
constexpr int MAX_NF = 4096;
constexpr int MAX_CH = 100000;
constexpr double TIE_TOL = 1e-9;          // island-boundary tie tolerance in grid steps
constexpr size_t DEFAULT_YCAP = size_t(8) << 30;  // bytes of coherent-sum buffer per launch chunk

thread_local std::string g_create_error;

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        size_t want = std::max(bytes, size_t(256));
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <typename T>
    T* as() const { return reinterpret_cast<T*>(p); }
};

struct HostBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        size_t want = std::max(bytes * 3 / 2, size_t(4096));
        hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release()
    {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
};

bool is_fin(double x) { return std::isfinite(x); }

}  // namespace

struct isrs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    bool has_spec = false;
    int n_ch = 0;
    double spacing = 0, rs = 0, rolloff = 0, f_center = 0;
    std::vector<double> power, phi, psi;

    bool has_link = false;
    std::vector<isrs_span> spans;
    int gain_mode = ISRS_GAIN_EQUALIZED;
    double ptot_override = 0.0;

    bool profiling = false;
    isrs_stats stats{};
    size_t ycap = DEFAULT_YCAP;

    DevBuf d_spans, d_seg, d_Sg, d_wt, d_s3, d_livep, d_insts, d_items, d_partD, d_partE, d_Y, d_dlist,
        d_out, d_power, d_phi, d_psi;
    HostBuf h_stage;
    hipEvent_t ev_upload = nullptr;
    std::vector<hipEvent_t> ev_pool;
};

namespace {

int32_t fail(isrs_ctx* c, int32_t code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

int32_t hip_fail(isrs_ctx* c, hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, e == hipErrorOutOfMemory ? ISRS_E_NOMEM : ISRS_E_DEVICE, m);
}

#define HIP_TRY(ctx, expr)                                        \
    do {                                                          \
        hipError_t _e = (expr);                                   \
        if (_e != hipSuccess) return hip_fail((ctx), _e, #expr); \
    } while (0)

std::string validate_spectrum_msg(const isrs_spectrum* s)
{
    if (!s) return "spectrum is null";
    if (s->n_ch < 1 || s->n_ch > MAX_CH) return "n_ch out of range";
    if (!s->power_w || !s->phi || !s->psi) return "spectrum arrays must not be null";
    if (!(is_fin(s->spacing_thz) && s->spacing_thz > 0)) return "spacing must be finite and > 0";
    if (!(is_fin(s->symbol_rate_thz) && s->symbol_rate_thz > 0)) return "symbol rate must be finite and > 0";
    if (!(is_fin(s->rolloff) && s->rolloff >= 0 && s->rolloff <= 1)) return "roll-off must be in [0, 1]";
    if (!is_fin(s->f_center_thz)) return "f_center must be finite";
    if ((1.0 + s->rolloff) * s->symbol_rate_thz > s->spacing_thz * (1.0 + 1e-12))
        return "(1 + rolloff) * symbol rate exceeds the channel spacing (channels would overlap)";
    int active = 0;
    for (int k = 0; k < s->n_ch; ++k) {
        if (!(is_fin(s->power_w[k]) && s->power_w[k] >= 0)) return "power must be finite and >= 0";
        if (!is_fin(s->phi[k]) || !is_fin(s->psi[k])) return "phi / psi must be finite";
        active += s->power_w[k] > 0;
    }
    if (!active) return "no active channel";
    return "";
}

std::string validate_link_msg(const isrs_span* sp, int32_t n, int32_t gain_mode)
{
    if (!sp) return "span array is null";
    if (n < 1 || n > MAX_SPANS) return "n_spans out of range";
    if (gain_mode != ISRS_GAIN_EQUALIZED && gain_mode != ISRS_GAIN_LOSS_ONLY) return "unknown gain mode";
    for (int s = 0; s < n; ++s) {
        const isrs_span& x = sp[s];
        if (!(is_fin(x.length_km) && x.length_km > 0)) return "span length must be finite and > 0";
        if (!(is_fin(x.alpha_db_km) && x.alpha_db_km > 0)) return "attenuation must be finite and > 0";
        if (!is_fin(x.beta2_ps2_km) || !is_fin(x.beta3_ps3_km)) return "dispersion must be finite";
        if (!(is_fin(x.gamma_w_km) && x.gamma_w_km >= 0)) return "gamma must be finite and >= 0";
        if (!(is_fin(x.cr_w_km_thz) && x.cr_w_km_thz >= 0)) return "Raman slope must be finite and >= 0";
    }
    return "";
}

std::string validate_numerics_msg(const isrs_numerics* nu)
{
    if (!nu) return "numerics is null";
    if (nu->n1 < 1 || nu->n1 > MAX_GRID) return "grid size out of range";
    if (nu->n2 != nu->n1) return "n1 and n2 must be equal";
    if (nu->n_f < 1 || nu->n_f > MAX_NF) return "n_f out of range";
    if (!(is_fin(nu->dz_km) && nu->dz_km > 0)) return "dz must be finite and > 0";
    if (nu->egn != 0 && nu->egn != 1) return "egn must be 0 or 1";
    if (nu->precision != ISRS_PREC_FP64 && nu->precision != ISRS_PREC_FP32_PHASE64) return "unknown precision";
    if (nu->mu_method != ISRS_MU_SEGMENT && nu->mu_method != ISRS_MU_MACLAURIN) return "unknown mu method";
    return "";
}

// Raised-cosine shape, 1 in the flat part, 0 outside (1+ro) Rs / 2.
double rc(double x, double rs, double ro)
{
    const double ax = std::fabs(x), lo = 0.5 * (1.0 - ro) * rs, hi = 0.5 * (1.0 + ro) * rs;
    if (ax <= lo) return 1.0;
    if (ax > hi) return 0.0;
    return 0.5 * (1.0 + std::cos(M_PI * (ax - lo) / (ro * rs)));
}

double field_S(double x, double rs, double ro) { return std::sqrt(rc(x, rs, ro)) / rs; }

struct Plan {
    int N, n_f, AD, nt, n_groups, spb;
    double W, h, B, ptot;
    bool fp32;
    std::vector<SpanConst> spans;
    std::vector<SegRow64> seg64;
    std::vector<SegRow32> seg32;
    std::vector<double> Sg, wt, s3, fs;
    std::vector<int> livep;
    std::vector<long long> livepts;  // [n_f][8 masks][2N] prefix of points on live anti-diagonals
    std::vector<InstDesc> insts;
    std::vector<SquareItem> items;
    std::vector<int> chunk_begin;    // item index where each launch chunk starts (+ end)
    std::vector<int> dlist;          // coherent-sum squares in item order
    std::vector<int> dchunk_begin;
    long long horner_steps = 0, live_points = 0;
    double alg_flop = 0;
    int sumK = 0;
};

// Tables of Eqs. 8-10 / 25 per span, island tables per outer sample.
void build_tables(const isrs_ctx* c, const isrs_numerics* nu, Plan& p)
{
    p.N = nu->n1;
    p.n_f = nu->n_f;
    p.AD = 2 * p.N - 1;
    p.W = (1.0 + c->rolloff) * c->rs;
    p.h = p.W / p.N;
    p.B = c->n_ch * c->spacing;
    double pt = 0.0;
    for (double x : c->power) pt += x;
    p.ptot = c->ptot_override > 0 ? c->ptot_override : pt;
    p.fp32 = nu->precision == ISRS_PREC_FP32_PHASE64;

    const int ns = (int)c->spans.size();
    p.spans.resize(ns);
    // LOSS_ONLY gain: per span A(L) and zeta(L) of rho(L, x) = A e^{-zeta x} e^{-alpha L}
    std::vector<double> lnA(ns), zL(ns);
    double b2L = 0.0, b3L = 0.0;
    int off = 0;
    p.seg64.clear();
    for (int s = 0; s < ns; ++s) {
        const isrs_span& sp = c->spans[s];
        const double alpha = sp.alpha_db_km * std::log(10.0) / 10.0;
        const double L = sp.length_km;
        int K = (int)std::ceil(L / nu->dz_km);
        if (K < 1) K = 1;
        const double dl = L / K;
        SpanConst& q = p.spans[s];
        q.c2r = 2.0 * M_PI * sp.beta2_ps2_km * dl;
        q.c3r = 2.0 * M_PI * M_PI * sp.beta3_ps3_km * dl;
        q.c2x = 4.0 * M_PI * M_PI * sp.beta2_ps2_km;
        q.c3x = 4.0 * M_PI * M_PI * M_PI * sp.beta3_ps3_km;
        q.p2r = 2.0 * M_PI * b2L;
        q.p3r = 2.0 * M_PI * M_PI * b3L;
        q.c2L = 2.0 * M_PI * sp.beta2_ps2_km * L;
        q.c3L = 2.0 * M_PI * M_PI * sp.beta3_ps3_km * L;
        q.em = std::exp(-alpha * dl);
        q.emL = std::exp(-alpha * L);
        q.em2L = std::exp(-2.0 * alpha * L);
        q.alpha = alpha;
        q.gamma = sp.gamma_w_km;
        q.pcr = p.ptot * sp.cr_w_km_thz;
        q.K = K;
        q.off = off;
        b2L += sp.beta2_ps2_km * L;
        b3L += sp.beta3_ps3_km * L;
        for (int k = 0; k < K; ++k) {
            const double z = (k + 0.5) / K * L;
            const double leff = -std::expm1(-alpha * z) / alpha;
            const double X = p.B * p.ptot * sp.cr_w_km_thz * leff;
            const double A = X == 0.0 ? 1.0 : X / (2.0 * std::sinh(0.5 * X));
            const double zeta = X / p.B;
            p.seg64.push_back({A, zeta, std::exp(-zeta * p.h), 0.0});
        }
        const double leffL = -std::expm1(-alpha * L) / alpha;
        const double XL = p.B * p.ptot * sp.cr_w_km_thz * leffL;
        lnA[s] = XL == 0.0 ? 0.0 : std::log(XL / (2.0 * std::sinh(0.5 * XL)));
        zL[s] = XL / p.B;
        off += K;
    }
    p.sumK = off;
    double TA = 0.0, TZ = 0.0;
    for (int s = 0; s < ns; ++s) {
        TA += lnA[s];
        TZ += zL[s];
    }
    double PA = 0.0, PZ = 0.0;
    for (int s = 0; s < ns; ++s) {
        // ln Pi_s = sum_{s'<s} [1.5 lnA - 0.5 zeta (a + b + x3)] + sum_{s'>=s} [0.5 lnA - 0.5 zeta c],
        // with a + b + x3 = 2 (a + b) - c
        p.spans[s].pi_a = PA + 0.5 * TA;
        p.spans[s].pi_s = PZ;
        p.spans[s].pi_c = PZ - 0.5 * TZ;
        PA += lnA[s];
        PZ += zL[s];
    }
    p.seg32.resize(p.seg64.size());
    for (size_t i = 0; i < p.seg64.size(); ++i)
        p.seg32[i] = {(float)p.seg64[i].A, (float)p.seg64[i].zeta, (float)p.seg64[i].ratio, 0.0f};

    // S at the grid points of a channel
    p.Sg.resize(p.N);
    for (int i = 0; i < p.N; ++i) p.Sg[i] = field_S((i + 0.5 - 0.5 * p.N) * p.h, c->rs, c->rolloff);

    // outer samples and island tables
    p.fs.resize(p.n_f);
    for (int n = 0; n < p.n_f; ++n) p.fs[n] = p.n_f == 1 ? 0.0 : -0.5 * c->rs + (n + 0.5) * c->rs / p.n_f;
    const int AD = p.AD;
    p.wt.assign((size_t)p.n_f * 3 * AD, 0.0);
    p.s3.assign((size_t)p.n_f * 3 * AD, 0.0);
    p.livep.assign((size_t)p.n_f * 3 * (AD + 1), 0);
    p.livepts.assign((size_t)p.n_f * 8 * (AD + 1), 0);
    const double ratio = c->spacing / p.h, half = 0.5 * p.N;
    for (int n = 0; n < p.n_f; ++n) {
        const double f = p.fs[n];
        std::vector<unsigned char> liv(3 * AD, 0);
        for (int l = 0; l < 3; ++l) {
            for (int m = 0; m < AD; ++m) {
                const double u = (double)(m + 1 - p.N) - f / p.h - (l - 1) * ratio;  // f3 / h
                const double au = std::fabs(u);
                double w = 0.0, sv = 0.0;
                if (au < half - TIE_TOL) {
                    w = 1.0;
                    sv = field_S(u * p.h, c->rs, c->rolloff);
                } else if (au <= half + TIE_TOL) {
                    w = 0.5;  // boundary: the cell is split between two islands
                    sv = c->rolloff == 0.0 ? 1.0 / c->rs : field_S(u * p.h, c->rs, c->rolloff);
                }
                const size_t o = ((size_t)n * 3 + l) * AD + m;
                p.wt[o] = w;
                p.s3[o] = sv;
                liv[l * AD + m] = (w > 0.0 && sv != 0.0);
                p.livep[((size_t)n * 3 + l) * (AD + 1) + m + 1] = p.livep[((size_t)n * 3 + l) * (AD + 1) + m] + liv[l * AD + m];
            }
        }
        for (int mask = 0; mask < 8; ++mask) {
            long long* pp = &p.livepts[((size_t)n * 8 + mask) * (AD + 1)];
            for (int m = 0; m < AD; ++m) {
                bool any = false;
                for (int l = 0; l < 3; ++l) any |= ((mask >> l) & 1) && liv[l * AD + m];
                const int len = std::min(m + 1, 2 * p.N - 1 - m);
                pp[m + 1] = pp[m] + (any ? len : 0);
            }
        }
    }
    p.nt = (p.N + TILE - 1) / TILE;
}

// Work list over (CUT, f sample) instances and their folded squares.
void build_work(const isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int n_cut,
                const int32_t* kappa12, int m_explicit, size_t ycap, Plan& p)
{
    const int nc = c->n_ch, AD = p.AD;
    p.insts.clear();
    p.items.clear();
    p.dlist.clear();
    const size_t ybytes = (size_t)p.N * p.N * (p.fp32 ? 8 : 16);
    const bool explicit_sq = kappa12 != nullptr;
    double ksum = 0.0;
    for (const SpanConst& s : p.spans) ksum += 8.0 * s.K + 30.0;
    long long steps_per_point = 0;
    for (const SpanConst& s : p.spans) steps_per_point += s.K;
    for (int q = 0; q < n_cut; ++q) {
        const int cut = cuts[q];
        for (int n = 0; n < p.n_f; ++n) {
            InstDesc in;
            in.f = p.fs[n];
            in.cut = cut;
            in.nf_idx = n;
            in.sq_begin = (int)p.items.size();
            const int* lp = &p.livep[(size_t)n * 3 * (AD + 1)];
            int any_live[3];
            for (int l = 0; l < 3; ++l) any_live[l] = lp[l * (AD + 1) + AD] > 0;
            const int n_sq = explicit_sq ? m_explicit : nc * nc;
            for (int t = 0; t < n_sq; ++t) {
                int k1, k2;
                if (explicit_sq) {
                    k1 = kappa12[2 * t];
                    k2 = kappa12[2 * t + 1];
                } else {
                    k1 = t / nc;
                    k2 = t % nc;
                    if (k2 < k1) continue;  // f1 <-> f2 symmetry: the mirror is folded in
                }
                if (!(c->power[k1] > 0 && c->power[k2] > 0)) {
                    if (!explicit_sq) continue;
                }
                SquareItem it{};
                it.inst = (int)p.insts.size();
                it.k1 = k1;
                it.k2 = k2;
                it.lmask = 0;
                it.egn_mask = 0;
                it.y_slot = -1;
                it.d_index = -1;
                it.mult = explicit_sq ? 1.0f : (k1 < k2 ? 2.0f : 1.0f);
                const bool pair_active = c->power[k1] > 0 && c->power[k2] > 0;
                for (int l = -1; l <= 1; ++l) {
                    const int k3 = k1 + k2 - cut + l;
                    if (!pair_active || k3 < 0 || k3 >= nc || !(c->power[k3] > 0) || !any_live[l + 1]) continue;
                    it.lmask |= 1 << (l + 1);
                    if (explicit_sq) {
                        it.egn_mask |= 0xF << (4 * (l + 1));
                    } else if (nu->egn) {
                        if (k3 == k1) it.egn_mask |= 1 << (4 * (l + 1) + 0);
                        if (k3 == k2) it.egn_mask |= 1 << (4 * (l + 1) + 1);
                        if (k1 == k2) it.egn_mask |= 1 << (4 * (l + 1) + 2);
                        if (k1 == k2 && k3 == k2) it.egn_mask |= 1 << (4 * (l + 1) + 3);
                    }
                }
                if (it.lmask == 0 && !explicit_sq) continue;
                const long long pts = p.livepts[((size_t)n * 8 + it.lmask) * (AD + 1) + AD];
                p.live_points += pts;
                p.horner_steps += pts * steps_per_point;
                p.alg_flop += (double)pts * ksum;
                p.items.push_back(it);
            }
            in.sq_end = (int)p.items.size();
            p.insts.push_back(in);
        }
    }
    // launch chunks: bound the coherent-sum buffer of each chunk by ycap
    const size_t per_chunk = std::max<size_t>(1, ycap / std::max<size_t>(ybytes, 1));
    p.chunk_begin.assign(1, 0);
    p.dchunk_begin.assign(1, 0);
    size_t slots = 0;
    for (size_t i = 0; i < p.items.size(); ++i) {
        SquareItem& it = p.items[i];
        if (it.egn_mask == 0) continue;
        if (slots == per_chunk) {
            p.chunk_begin.push_back((int)i);
            p.dchunk_begin.push_back((int)p.dlist.size());
            slots = 0;
        }
        it.y_slot = (int)slots++;
        it.d_index = (int)p.dlist.size();
        p.dlist.push_back((int)i);
    }
    p.chunk_begin.push_back((int)p.items.size());
    p.dchunk_begin.push_back((int)p.dlist.size());
    // strip groups: enough blocks to fill the chip, few partials
    const long long n_items = (long long)p.items.size();
    const long long target = 32768;
    int spb = (int)std::min<long long>(p.nt, std::max<long long>(1, n_items * p.nt / target));
    p.spb = spb;
    p.n_groups = (p.nt + spb - 1) / spb;
}

template <typename T>
int32_t upload(isrs_ctx* c, DevBuf& d, const std::vector<T>& v, char*& stage)
{
    const size_t bytes = v.size() * sizeof(T);
    HIP_TRY(c, d.ensure(bytes));
    if (bytes) {
        std::memcpy(stage, v.data(), bytes);
        HIP_TRY(c, hipMemcpyAsync(d.p, stage, bytes, hipMemcpyHostToDevice, c->stream));
        stage += (bytes + 255) & ~size_t(255);
    }
    return ISRS_OK;
}

template <typename T>
size_t staged(const std::vector<T>& v)
{
    return (v.size() * sizeof(T) + 255) & ~size_t(255);
}

hipEvent_t pool_event(isrs_ctx* c, size_t i)
{
    while (c->ev_pool.size() <= i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[i];
}

// Shared evaluation path.  Outputs are device pointers (eta, sigma2, terms,
// psd nullable except eta); partials_host receives island partials for the
// explicit-square mode.
int32_t evaluate(isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int n_cut, const int32_t* kappa12,
                 int m_explicit, double* eta_d, double* s2_d, double* terms_d, double* psd_d,
                 double* partials_host)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!c) return ISRS_E_ARG;
    if (!c->has_spec || !c->has_link) return fail(c, ISRS_E_STATE, "set the spectrum and the link first");
    std::string m = validate_numerics_msg(nu);
    if (!m.empty()) return fail(c, ISRS_E_ARG, m);
    if (!cuts || n_cut < 1) return fail(c, ISRS_E_ARG, "need at least one CUT");
    for (int q = 0; q < n_cut; ++q) {
        if (cuts[q] < 0 || cuts[q] >= c->n_ch) return fail(c, ISRS_E_ARG, "CUT index out of range");
        if (!(c->power[cuts[q]] > 0)) return fail(c, ISRS_E_ARG, "CUT is an inactive channel");
    }
    if (kappa12) {
        for (int t = 0; t < 2 * m_explicit; ++t)
            if (kappa12[t] < 0 || kappa12[t] >= c->n_ch) return fail(c, ISRS_E_ARG, "square index out of range");
    }
    for (const isrs_span& s : c->spans)
        if (std::ceil(s.length_km / nu->dz_km) > 1e6) return fail(c, ISRS_E_ARG, "dz too small: more than 1e6 segments");

    HIP_TRY(c, hipSetDevice(c->device));
    Plan p;
    try {
        build_tables(c, nu, p);
        build_work(c, nu, cuts, n_cut, kappa12, m_explicit, c->ycap, p);
    } catch (const std::bad_alloc&) {
        return fail(c, ISRS_E_NOMEM, "host allocation failed");
    }

    // upload through pinned staging; wait for the previous call's copies first
    if (c->ev_upload) HIP_TRY(c, hipEventSynchronize(c->ev_upload));
    const size_t need = staged(p.spans) + (p.fp32 ? staged(p.seg32) : staged(p.seg64)) + staged(p.Sg) +
                        staged(p.wt) + staged(p.s3) + staged(p.livep) + staged(p.insts) + staged(p.items) +
                        staged(p.dlist) + 3 * ((c->n_ch * sizeof(double) + 255) & ~size_t(255));
    HIP_TRY(c, c->h_stage.ensure(need));
    char* stage = reinterpret_cast<char*>(c->h_stage.p);
    int32_t rc;
    if ((rc = upload(c, c->d_spans, p.spans, stage))) return rc;
    if (p.fp32) {
        if ((rc = upload(c, c->d_seg, p.seg32, stage))) return rc;
    } else {
        if ((rc = upload(c, c->d_seg, p.seg64, stage))) return rc;
    }
    if ((rc = upload(c, c->d_Sg, p.Sg, stage))) return rc;
    if ((rc = upload(c, c->d_wt, p.wt, stage))) return rc;
    if ((rc = upload(c, c->d_s3, p.s3, stage))) return rc;
    if ((rc = upload(c, c->d_livep, p.livep, stage))) return rc;
    if ((rc = upload(c, c->d_insts, p.insts, stage))) return rc;
    if ((rc = upload(c, c->d_items, p.items, stage))) return rc;
    if ((rc = upload(c, c->d_dlist, p.dlist, stage))) return rc;
    if ((rc = upload(c, c->d_power, c->power, stage))) return rc;
    if ((rc = upload(c, c->d_phi, c->phi, stage))) return rc;
    if ((rc = upload(c, c->d_psi, c->psi, stage))) return rc;
    if (!c->ev_upload) HIP_TRY(c, hipEventCreateWithFlags(&c->ev_upload, hipEventDisableTiming));
    HIP_TRY(c, hipEventRecord(c->ev_upload, c->stream));

    const size_t n_items = p.items.size();
    HIP_TRY(c, c->d_partD.ensure(std::max<size_t>(1, n_items) * p.n_groups * 3 * sizeof(double)));
    HIP_TRY(c, c->d_partE.ensure(std::max<size_t>(1, p.dlist.size()) * 12 * sizeof(double)));
    size_t max_slots = 0;
    for (size_t ch = 0; ch + 1 < p.dchunk_begin.size(); ++ch)
        max_slots = std::max<size_t>(max_slots, p.dchunk_begin[ch + 1] - p.dchunk_begin[ch]);
    const size_t ybytes = (size_t)p.N * p.N * (p.fp32 ? 8 : 16);
    HIP_TRY(c, c->d_Y.ensure(std::max<size_t>(1, max_slots) * ybytes));

    auto t1 = std::chrono::steady_clock::now();

    RegionArgs ra{};
    ra.spans = c->d_spans.as<SpanConst>();
    ra.seg = c->d_seg.p;
    ra.Sg = c->d_Sg.as<double>();
    ra.wt = c->d_wt.as<double>();
    ra.s3 = c->d_s3.as<double>();
    ra.livep = c->d_livep.as<int>();
    ra.insts = c->d_insts.as<InstDesc>();
    ra.items = c->d_items.as<SquareItem>();
    ra.partD = c->d_partD.as<double>();
    ra.ybuf = c->d_Y.p;
    ra.n_groups = p.n_groups;
    ra.spb = p.spb;
    ra.nt = p.nt;
    ra.N = p.N;
    ra.n_ch = c->n_ch;
    ra.n_sp = (int)p.spans.size();
    ra.gain_mode = c->gain_mode;
    ra.mu_method = nu->mu_method;
    ra.h = p.h;
    ra.spacing = c->spacing;

    EgnArgs ea{};
    ea.Sg = ra.Sg;
    ea.wt = ra.wt;
    ea.s3 = ra.s3;
    ea.insts = ra.insts;
    ea.items = ra.items;
    ea.ybuf = c->d_Y.p;
    ea.partE = c->d_partE.as<double>();
    ea.N = p.N;
    ea.h = p.h;

    const size_t n_chunks = p.chunk_begin.size() - 1;
    size_t ev_i = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> reg_ev, egn_ev;
    for (size_t ch = 0; ch < n_chunks; ++ch) {
        const int b = p.chunk_begin[ch], e = p.chunk_begin[ch + 1];
        ra.item0 = b;
        hipEvent_t a0 = nullptr, a1 = nullptr;
        if (c->profiling) {
            a0 = pool_event(c, ev_i++);
            a1 = pool_event(c, ev_i++);
            if (!a0 || !a1) return fail(c, ISRS_E_DEVICE, "event creation failed");
            HIP_TRY(c, hipEventRecord(a0, c->stream));
        }
        HIP_TRY(c, launch_region(ra, e - b, p.fp32, c->stream));
        if (c->profiling) {
            HIP_TRY(c, hipEventRecord(a1, c->stream));
            reg_ev.push_back({a0, a1});
        }
        const int db = p.dchunk_begin[ch], de = p.dchunk_begin[ch + 1];
        if (de > db) {
            ea.dlist = c->d_dlist.as<int>() + db;
            hipEvent_t b0 = nullptr, b1 = nullptr;
            if (c->profiling) {
                b0 = pool_event(c, ev_i++);
                b1 = pool_event(c, ev_i++);
                if (!b0 || !b1) return fail(c, ISRS_E_DEVICE, "event creation failed");
                HIP_TRY(c, hipEventRecord(b0, c->stream));
            }
            HIP_TRY(c, launch_egn(ea, de - db, p.fp32, c->stream));
            if (c->profiling) {
                HIP_TRY(c, hipEventRecord(b1, c->stream));
                egn_ev.push_back({b0, b1});
            }
        }
    }

    if (!partials_host) {
        AssembleArgs aa{};
        aa.insts = ra.insts;
        aa.items = ra.items;
        aa.partD = ra.partD;
        aa.partE = ea.partE;
        aa.power = c->d_power.as<double>();
        aa.phi = c->d_phi.as<double>();
        aa.psi = c->d_psi.as<double>();
        aa.eta = eta_d;
        aa.sigma2 = s2_d;
        aa.terms = terms_d;
        aa.psd = psd_d;
        aa.n_groups = p.n_groups;
        aa.n_f = p.n_f;
        aa.rs = c->rs;
        aa.h = p.h;
        aa.n_cut = n_cut;
        hipEvent_t c0 = nullptr, c1 = nullptr;
        if (c->profiling) {
            c0 = pool_event(c, ev_i++);
            c1 = pool_event(c, ev_i++);
            if (!c0 || !c1) return fail(c, ISRS_E_DEVICE, "event creation failed");
            HIP_TRY(c, hipEventRecord(c0, c->stream));
        }
        HIP_TRY(c, launch_assemble(aa, c->stream));
        if (c->profiling) {
            HIP_TRY(c, hipEventRecord(c1, c->stream));
            HIP_TRY(c, hipEventSynchronize(c1));
            float ms = 0;
            HIP_TRY(c, hipEventElapsedTime(&ms, c0, c1));
            c->stats.assemble_ms = ms;
        }
    } else {
        // island partials: D per group summed on the host, coherent sums as computed
        std::vector<double> pd(n_items * p.n_groups * 3), pe(std::max<size_t>(1, p.dlist.size()) * 12);
        HIP_TRY(c, hipMemcpyAsync(pd.data(), ra.partD, pd.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(pe.data(), ea.partE, pe.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        const double h2 = p.h * p.h;
        for (int t = 0; t < m_explicit; ++t) {
            const SquareItem& it = p.items[t];
            for (int l = 0; l < 3; ++l) {
                double D = 0.0;
                for (int g = 0; g < p.n_groups; ++g) D += pd[((size_t)t * p.n_groups + g) * 3 + l];
                double* o = partials_host + (size_t)t * 15 + l * 5;
                const bool valid = (it.lmask >> l) & 1;
                o[0] = valid ? h2 * D : 0.0;
                for (int u = 0; u < 4; ++u) o[1 + u] = (valid && it.d_index >= 0) ? pe[(size_t)it.d_index * 12 + l * 4 + u] : 0.0;
            }
        }
    }

    auto t2 = std::chrono::steady_clock::now();
    c->stats.host_prep_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    c->stats.region_launches = (int64_t)n_chunks;
    c->stats.n_squares = (int64_t)n_items;
    c->stats.n_delta_squares = (int64_t)p.dlist.size();
    c->stats.n_points_live = p.live_points;
    c->stats.horner_steps = nu->mu_method == ISRS_MU_SEGMENT ? p.horner_steps : 0;
    c->stats.alg_flop = p.alg_flop;
    if (c->profiling) {
        double rms = 0, ems = 0;
        for (auto& e : reg_ev) {
            HIP_TRY(c, hipEventSynchronize(e.second));
            float ms = 0;
            HIP_TRY(c, hipEventElapsedTime(&ms, e.first, e.second));
            rms += ms;
        }
        for (auto& e : egn_ev) {
            HIP_TRY(c, hipEventSynchronize(e.second));
            float ms = 0;
            HIP_TRY(c, hipEventElapsedTime(&ms, e.first, e.second));
            ems += ms;
        }
        c->stats.region_ms = rms;
        c->stats.egn_ms = ems;
    } else {
        c->stats.region_ms = c->stats.egn_ms = c->stats.assemble_ms = 0;
    }
    (void)t2;
    return ISRS_OK;
}

}  // namespace

extern "C" {

const char* isrs_version(void) { return "isrs-egn 0.1 (gfx950)"; }

int32_t isrs_validate_spectrum(const isrs_spectrum* s)
{
    if (!s) return ISRS_E_ARG;
    return validate_spectrum_msg(s).empty() ? ISRS_OK : ISRS_E_SPECTRUM;
}

int32_t isrs_validate_link(const isrs_span* sp, int32_t n, int32_t gain_mode)
{
    if (!sp) return ISRS_E_ARG;
    if (n < 1 || n > MAX_SPANS) return ISRS_E_ARG;
    return validate_link_msg(sp, n, gain_mode).empty() ? ISRS_OK : ISRS_E_LINK;
}

int32_t isrs_validate_numerics(const isrs_numerics* nu)
{
    return validate_numerics_msg(nu).empty() ? ISRS_OK : ISRS_E_ARG;
}

int32_t isrs_create(isrs_ctx** out, int32_t device, void* hip_stream)
{
    g_create_error.clear();
    if (!out) {
        g_create_error = "out is null";
        return ISRS_E_ARG;
    }
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        g_create_error = "no HIP device";
        return ISRS_E_DEVICE;
    }
    if (device < 0 || device >= n) {
        g_create_error = "device ordinal out of range";
        return ISRS_E_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        g_create_error = "hipGetDeviceProperties failed";
        return ISRS_E_DEVICE;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_create_error = std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950";
        return ISRS_E_DEVICE;
    }
    isrs_ctx* c = new (std::nothrow) isrs_ctx();
    if (!c) {
        g_create_error = "host allocation failed";
        return ISRS_E_NOMEM;
    }
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        g_create_error = "hipSetDevice failed";
        return ISRS_E_DEVICE;
    }
    if (hip_stream) {
        c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            g_create_error = "stream creation failed";
            return ISRS_E_DEVICE;
        }
        c->own_stream = true;
    }
    *out = c;
    return ISRS_OK;
}

int32_t isrs_destroy(isrs_ctx* c)
{
    if (!c) return ISRS_E_ARG;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    DevBuf* bufs[] = {&c->d_spans, &c->d_seg, &c->d_Sg, &c->d_wt, &c->d_s3, &c->d_livep, &c->d_insts, &c->d_items,
                      &c->d_partD, &c->d_partE, &c->d_Y, &c->d_dlist, &c->d_out, &c->d_power, &c->d_phi, &c->d_psi};
    for (DevBuf* b : bufs) b->release();
    c->h_stage.release();
    if (c->ev_upload) (void)hipEventDestroy(c->ev_upload);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return ISRS_OK;
}

const char* isrs_last_error(const isrs_ctx* c)
{
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

int32_t isrs_set_spectrum(isrs_ctx* c, const isrs_spectrum* s)
{
    if (!c) return ISRS_E_ARG;
    if (!s) return fail(c, ISRS_E_ARG, "spectrum is null");
    std::string m = validate_spectrum_msg(s);
    if (!m.empty()) return fail(c, ISRS_E_SPECTRUM, m);
    c->n_ch = s->n_ch;
    c->spacing = s->spacing_thz;
    c->rs = s->symbol_rate_thz;
    c->rolloff = s->rolloff;
    c->f_center = s->f_center_thz;
    c->power.assign(s->power_w, s->power_w + s->n_ch);
    c->phi.assign(s->phi, s->phi + s->n_ch);
    c->psi.assign(s->psi, s->psi + s->n_ch);
    c->has_spec = true;
    c->err.clear();
    return ISRS_OK;
}

int32_t isrs_set_link(isrs_ctx* c, const isrs_span* spans, int32_t n, int32_t gain_mode)
{
    if (!c) return ISRS_E_ARG;
    if (!spans || n < 1 || n > MAX_SPANS) return fail(c, ISRS_E_ARG, "bad span array or count");
    std::string m = validate_link_msg(spans, n, gain_mode);
    if (!m.empty()) return fail(c, ISRS_E_LINK, m);
    c->spans.assign(spans, spans + n);
    c->gain_mode = gain_mode;
    c->has_link = true;
    c->err.clear();
    return ISRS_OK;
}

int32_t isrs_set_ptot_override(isrs_ctx* c, double ptot_w)
{
    if (!c) return ISRS_E_ARG;
    if (!(is_fin(ptot_w) && ptot_w >= 0)) return fail(c, ISRS_E_ARG, "ptot override must be finite and >= 0");
    c->ptot_override = ptot_w;
    return ISRS_OK;
}

int32_t isrs_set_profiling(isrs_ctx* c, int32_t profile)
{
    if (!c) return ISRS_E_ARG;
    c->profiling = profile != 0;
    return ISRS_OK;
}

int32_t isrs_get_stats(const isrs_ctx* c, isrs_stats* out)
{
    if (!c || !out) return ISRS_E_ARG;
    *out = c->stats;
    return ISRS_OK;
}

int32_t isrs_eval_eta_dev(isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int32_t n_cut, double* eta_dev,
                          double* sigma2_dev, double* terms_dev)
{
    if (!c) return ISRS_E_ARG;
    if (!eta_dev) return fail(c, ISRS_E_ARG, "eta output is null");
    return evaluate(c, nu, cuts, n_cut, nullptr, 0, eta_dev, sigma2_dev, terms_dev, nullptr, nullptr);
}

int32_t isrs_eval_eta(isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int32_t n_cut, double* eta,
                      double* sigma2, double* terms)
{
    if (!c) return ISRS_E_ARG;
    if (!eta) return fail(c, ISRS_E_ARG, "eta output is null");
    if (n_cut < 1) return fail(c, ISRS_E_ARG, "need at least one CUT");
    HIP_TRY(c, hipSetDevice(c->device));
    const size_t n = (size_t)n_cut;
    HIP_TRY(c, c->d_out.ensure(n * 7 * sizeof(double)));
    double* d = c->d_out.as<double>();
    int32_t rc = evaluate(c, nu, cuts, n_cut, nullptr, 0, d, d + n, d + 2 * n, nullptr, nullptr);
    if (rc) return rc;
    std::vector<double> h(n * 7);
    HIP_TRY(c, hipMemcpyAsync(h.data(), d, n * 7 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t q = 0; q < n; ++q) {
        if (!is_fin(h[q]) || !is_fin(h[n + q])) return fail(c, ISRS_E_NUMERIC, "non-finite NLI result");
        eta[q] = h[q];
        if (sigma2) sigma2[q] = h[n + q];
        if (terms)
            for (int u = 0; u < 5; ++u) terms[q * 5 + u] = h[2 * n + q * 5 + u];
    }
    return ISRS_OK;
}

int32_t isrs_eval_psd(isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int32_t n_cut, double* f_thz,
                      double* psd)
{
    if (!c) return ISRS_E_ARG;
    if (!f_thz || !psd) return fail(c, ISRS_E_ARG, "output is null");
    std::string m = validate_numerics_msg(nu);
    if (!m.empty()) return fail(c, ISRS_E_ARG, m);
    if (n_cut < 1) return fail(c, ISRS_E_ARG, "need at least one CUT");
    HIP_TRY(c, hipSetDevice(c->device));
    const size_t n = (size_t)n_cut, nf = (size_t)nu->n_f;
    HIP_TRY(c, c->d_out.ensure(n * (1 + nf) * sizeof(double)));
    double* d = c->d_out.as<double>();
    int32_t rc = evaluate(c, nu, cuts, n_cut, nullptr, 0, d, nullptr, nullptr, d + n, nullptr);
    if (rc) return rc;
    std::vector<double> h(n * nf);
    HIP_TRY(c, hipMemcpyAsync(h.data(), d + n, n * nf * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t q = 0; q < n; ++q)
        for (size_t k = 0; k < nf; ++k) {
            if (!is_fin(h[q * nf + k])) return fail(c, ISRS_E_NUMERIC, "non-finite PSD");
            psd[q * nf + k] = h[q * nf + k];
            f_thz[q * nf + k] = nf == 1 ? 0.0 : -0.5 * c->rs + (k + 0.5) * c->rs / nf;
        }
    return ISRS_OK;
}

int32_t isrs_eval_islands(isrs_ctx* c, const isrs_numerics* nu, int32_t cut, const int32_t* kappa12, int32_t m,
                          double* partials)
{
    if (!c) return ISRS_E_ARG;
    if (!kappa12 || m < 1 || !partials) return fail(c, ISRS_E_ARG, "bad square list or output");
    if (nu && nu->n_f != 1) return fail(c, ISRS_E_ARG, "island partials are defined at f = 0 (n_f = 1)");
    int32_t cuts[1] = {cut};
    int32_t rc = evaluate(c, nu, cuts, 1, kappa12, m, nullptr, nullptr, nullptr, nullptr, partials);
    if (rc) return rc;
    for (size_t t = 0; t < (size_t)m * 15; ++t)
        if (!is_fin(partials[t])) return fail(c, ISRS_E_NUMERIC, "non-finite island partial");
    return ISRS_OK;
}

}  // extern "C"
