// isrs_api.cpp -- host side of the C-ABI declared in include/isrs_egn.h.
//
// Validates inputs, builds the per-span segment tables (Eqs. 8-10, 25), the
// per-anti-diagonal island tables (Eq. 16 on the grid), the f1 <-> f2 folded
// work list of channel-pair squares of one or many links, and launches the
// gfx950 kernels on the context's stream.  No model arithmetic runs on the
// CPU beyond these tables: every grid point is evaluated on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <numeric>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "../../include/isrs_egn.h"
#include "isrs_internal.h"

using namespace isrs;

namespace {

constexpr int MAX_SPANS = 4096;
constexpr int MAX_GRID = 8192;
constexpr int MAX_NF = 4096;
constexpr int MAX_CH = 100000;
constexpr double TIE_TOL = 1e-9;                   // island-boundary tie tolerance in grid steps

thread_local std::string g_create_error;

bool is_fin(double x) { return std::isfinite(x); }

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap && p) return hipSuccess;
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
        if (bytes <= cap && p) return hipSuccess;
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

// One link as the planner sees it (pointers into context or batch storage).
struct LinkInput {
    int n_ch = 0;
    double spacing = 0, rs = 0, rolloff = 0;
    const double* power = nullptr;
    const double* phi = nullptr;
    const double* psi = nullptr;
    const isrs_span* spans = nullptr;
    int n_sp = 0;
    int gain_mode = ISRS_GAIN_EQUALIZED;
    double ptot_override = 0.0;
    const int32_t* cuts = nullptr;
    int n_cut = 0;
};

// Launch shape of the region kernel.
struct Tuning {
    int mode = 1;           // 0: one block per work unit, 1: persistent blocks on a queue
    int blocks_per_cu = 0;  // queue mode; 0 = as many as fit
    int sort = 1;           // queue mode: cost-sorted order
    int spb = 0;            // slices per unit; 0 = automatic
    int ppt = 0;            // points per run (region_ppt_supported); 0 = the precision's default
};

// Everything one evaluation uploads and launches.
struct Plan {
    int N = 0, n_f = 0, AD = 0, n_slices = 0, n_groups = 1, spb = 1, ppt = 0;
    bool fp32 = false;
    int mu_method = 0;
    std::vector<LinkDesc> links;
    std::vector<SpanConst> spans;
    std::vector<SegRow64> seg64;
    std::vector<SegRow32> seg32;
    std::vector<double> Sg, wt, s3;
    std::vector<int> livep;
    std::vector<int> runs;           // runs of PPT points by anti-diagonal (region kernel layout)
    std::vector<int> adrun;          // [2N] first run of each anti-diagonal, then the run count
    std::vector<double> power, phi, psi;
    std::vector<InstDesc> insts;
    std::vector<SquareItem> items;
    std::vector<double> item_cost;   // per square: live points x (sum K + span count)
    std::vector<int> chunk_begin;    // square index where each launch chunk starts (+ end)
    std::vector<int> dlist;          // coherent-sum squares in square order
    std::vector<int> order;          // per chunk: cost-sorted permutation of its units
    Tuning tu;                       // launch shape (queue mode whenever there are coherent sums)
    std::vector<std::vector<long long>> livepts;  // per link: [n_f][8 masks][2N] prefix of live points
    long long horner_steps = 0, live_points = 0;
    double alg_flop = 0;
    int n_cut_total = 0;
    int queue_blocks = 0;            // persistent blocks of a queue launch
};

// Squares and instances of some links, before they join a plan.
struct WorkPart {
    std::vector<InstDesc> insts;
    std::vector<SquareItem> items;
    std::vector<double> item_cost;
    long long live_points = 0, horner_steps = 0;
    double alg_flop = 0;
    int n_cut = 0;
};

// Device side of a plan.
struct Workspace {
    DevBuf links, spans, seg, Sg, wt, s3, livep, runs, adrun, insts, items, order, partD, partE, eacc, dlist,
        counter, out, power, phi, psi, sur;
    HostBuf stage;
    hipEvent_t ev_upload = nullptr;
    std::vector<hipEvent_t> ev_pool;
    void release()
    {
        DevBuf* bufs[] = {&links, &spans, &seg, &Sg, &wt, &s3, &livep, &runs, &adrun, &insts, &items, &order,
                          &partD, &partE, &eacc, &dlist, &counter, &out, &power, &phi, &psi, &sur};
        for (DevBuf* b : bufs) b->release();
        stage.release();
        if (ev_upload) (void)hipEventDestroy(ev_upload);
        ev_upload = nullptr;
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        ev_pool.clear();
    }
};

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
    int n_cu = 0;

    Workspace* ws = nullptr;

    // allocation-free evaluation: this device's scratch array, the host plan
    // of the last such call (its tables may still be on their way to the
    // device) and an event after its uploads
    void* scratch = nullptr;
    Plan* scratch_plan = nullptr;
    hipEvent_t ev_scratch = nullptr;
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

std::string validate_spectrum_fields(int n_ch, double spacing, double rs, double ro, const double* power,
                                     const double* phi, const double* psi)
{
    if (n_ch < 1 || n_ch > MAX_CH) return "n_ch out of range";
    if (!power || !phi || !psi) return "spectrum arrays must not be null";
    if (!(is_fin(spacing) && spacing > 0)) return "spacing must be finite and > 0";
    if (!(is_fin(rs) && rs > 0)) return "symbol rate must be finite and > 0";
    if (!(is_fin(ro) && ro >= 0 && ro <= 1)) return "roll-off must be in [0, 1]";
    if ((1.0 + ro) * rs > spacing * (1.0 + 1e-12))
        return "(1 + rolloff) * symbol rate exceeds the channel spacing (channels would overlap)";
    int active = 0;
    for (int k = 0; k < n_ch; ++k) {
        if (!(is_fin(power[k]) && power[k] >= 0)) return "power must be finite and >= 0";
        if (!is_fin(phi[k]) || !is_fin(psi[k])) return "phi / psi must be finite";
        active += power[k] > 0;
    }
    if (!active) return "no active channel";
    return "";
}

std::string validate_spectrum_msg(const isrs_spectrum* s)
{
    if (!s) return "spectrum is null";
    if (!is_fin(s->f_center_thz)) return "f_center must be finite";
    return validate_spectrum_fields(s->n_ch, s->spacing_thz, s->symbol_rate_thz, s->rolloff, s->power_w, s->phi,
                                    s->psi);
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
    if (nu->mu_method != ISRS_MU_SEGMENT && nu->mu_method != ISRS_MU_MACLAURIN && nu->mu_method != ISRS_MU_INTEGRAL)
        return "unknown mu method";
    return "";
}

std::string validate_link_numerics(const LinkInput& L, const isrs_numerics* nu)
{
    for (int s = 0; s < L.n_sp; ++s)
        if (std::ceil(L.spans[s].length_km / nu->dz_km) > 1e6) return "dz too small: more than 1e6 segments";
    for (int q = 0; q < L.n_cut; ++q) {
        if (L.cuts[q] < 0 || L.cuts[q] >= L.n_ch) return "CUT index out of range";
        if (!(L.power[L.cuts[q]] > 0)) return "CUT is an inactive channel";
    }
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

// Run table of the region kernel: runs of ppt consecutive points along each
// anti-diagonal m = i + j, and the first run of every anti-diagonal.
void plan_runs(Plan& p, int ppt)
{
    p.ppt = ppt > 0 ? ppt : ppt_of(p.fp32);
    p.runs.clear();
    p.adrun.assign(1, 0);
    for (int m = 0; m < p.AD; ++m) {
        for (int i = std::max(0, m - p.N + 1); i <= std::min(m, p.N - 1); i += p.ppt)
            p.runs.push_back(m << RUN_SHIFT | i);
        p.adrun.push_back((int)p.runs.size());
    }
    p.n_slices = (int)((p.runs.size() + THREADS - 1) / THREADS);
}

// Most anti-diagonals one slice of the run table spans (the kernel stages
// that many gain rows; NAD at most).
int plan_max_slice_rows(const Plan& p)
{
    int w = 0;
    for (size_t c0 = 0; c0 < p.runs.size(); c0 += THREADS) {
        const size_t c1 = std::min(c0 + THREADS, p.runs.size()) - 1;
        w = std::max(w, (p.runs[c1] >> RUN_SHIFT) - (p.runs[c0] >> RUN_SHIFT) + 1);
    }
    return w;
}

void plan_begin(const isrs_numerics* nu, Plan& p, int ppt = 0)
{
    p.N = nu->n1;
    p.n_f = nu->n_f;
    p.AD = 2 * p.N - 1;
    p.fp32 = nu->precision == ISRS_PREC_FP32_PHASE64 || nu->mu_method == MU_SUR;
    p.mu_method = nu->mu_method;
    plan_runs(p, ppt);
}

// Tables of one link (Eqs. 8-10 / 25 per span, islands per outer sample).
void plan_link_tables(const LinkInput& L, const isrs_numerics* nu, Plan& p)
{
    LinkDesc d{};
    const double W = (1.0 + L.rolloff) * L.rs, h = W / p.N, B = L.n_ch * L.spacing;
    double pt = 0.0;
    for (int k = 0; k < L.n_ch; ++k) pt += L.power[k];
    const double ptot = L.ptot_override > 0 ? L.ptot_override : pt;
    d.span0 = (int)p.spans.size();
    d.n_sp = L.n_sp;
    d.n_ch = L.n_ch;
    d.gain_mode = L.gain_mode;
    d.ch0 = (int)p.power.size();
    d.spacing = L.spacing;
    d.h = h;
    d.rs = L.rs;
    p.power.insert(p.power.end(), L.power, L.power + L.n_ch);
    p.phi.insert(p.phi.end(), L.phi, L.phi + L.n_ch);
    p.psi.insert(p.psi.end(), L.psi, L.psi + L.n_ch);

    // LOSS_ONLY gain: per span A(L) and zeta(L) of rho(L, x) = A e^{-zeta x} e^{-alpha L}
    std::vector<double> lnA(L.n_sp), zL(L.n_sp);
    double b2L = 0.0, b3L = 0.0;
    for (int s = 0; s < L.n_sp; ++s) {
        const isrs_span& sp = L.spans[s];
        const double alpha = sp.alpha_db_km * std::log(10.0) / 10.0;
        const double len = sp.length_km;
        int K = (int)std::ceil(len / nu->dz_km);
        if (K < 1) K = 1;
        const double dl = len / K;
        SpanConst q{};
        q.c2r = 2.0 * M_PI * sp.beta2_ps2_km * dl;
        q.c3r = 2.0 * M_PI * M_PI * sp.beta3_ps3_km * dl;
        q.c2x = 4.0 * M_PI * M_PI * sp.beta2_ps2_km;
        q.c3x = 4.0 * M_PI * M_PI * M_PI * sp.beta3_ps3_km;
        q.wd = 2.0 * M_PI / dl;
        q.L = len;
        q.cr = sp.cr_w_km_thz;
        q.ptot = ptot;
        q.btot = B;
        q.p2r = 2.0 * M_PI * b2L;
        q.p3r = 2.0 * M_PI * M_PI * b3L;
        q.c2L = 2.0 * M_PI * sp.beta2_ps2_km * len;
        q.c3L = 2.0 * M_PI * M_PI * sp.beta3_ps3_km * len;
        q.em = std::exp(-alpha * dl);
        q.emL = std::exp(-alpha * len);
        q.em2L = std::exp(-2.0 * alpha * len);
        q.alpha = alpha;
        q.gamma = sp.gamma_w_km;
        q.f_alpha = (float)q.alpha;
        q.f_em = (float)q.em;
        q.f_ms = (float)(-(q.em * q.em));
        q.f_wd = (float)q.wd;
        q.f_gamma = (float)q.gamma;
        q.f_emL = (float)q.emL;
        q.f_em2L = (float)q.em2L;
        q.f_pad = 0.0f;
        q.pcr = ptot * sp.cr_w_km_thz;
        q.K = K;
        q.off = (int)p.seg64.size();
        b2L += sp.beta2_ps2_km * len;
        b3L += sp.beta3_ps3_km * len;
        const int nodes = p.mu_method == MU_INT ? INT_NODES : 1;
        for (int n = 0; n < nodes; ++n)
            for (int k = 0; k < K; ++k) {
                const double z = (k + 0.5 + (nodes > 1 ? 0.5 * INT_U[n] : 0.0)) / K * len;
                const double leff = -std::expm1(-alpha * z) / alpha;
                const double X = B * ptot * sp.cr_w_km_thz * leff;
                const double A = X == 0.0 ? 1.0 : X / (2.0 * std::sinh(0.5 * X));
                const double zeta = X / B;
                p.seg64.push_back({A, zeta, std::exp(-zeta * h), 0.0});
            }
        const double leffL = -std::expm1(-alpha * len) / alpha;
        const double XL = B * ptot * sp.cr_w_km_thz * leffL;
        lnA[s] = XL == 0.0 ? 0.0 : std::log(XL / (2.0 * std::sinh(0.5 * XL)));
        zL[s] = XL / B;
        p.spans.push_back(q);
    }
    double TA = 0.0, TZ = 0.0, PA = 0.0, PZ = 0.0;
    for (int s = 0; s < L.n_sp; ++s) {
        TA += lnA[s];
        TZ += zL[s];
    }
    for (int s = 0; s < L.n_sp; ++s) {
        // ln Pi_s = sum_{s'<s} [1.5 lnA - 0.5 zeta (a + b + x3)] + sum_{s'>=s} [0.5 lnA - 0.5 zeta c],
        // with a + b + x3 = 2 (a + b) - c
        SpanConst& q = p.spans[d.span0 + s];
        q.pi_a = PA + 0.5 * TA;
        q.pi_s = PZ;
        q.pi_c = PZ - 0.5 * TZ;
        PA += lnA[s];
        PZ += zL[s];
    }

    d.sg0 = (int)p.Sg.size();
    for (int i = 0; i < p.N; ++i) p.Sg.push_back(field_S((i + 0.5 - 0.5 * p.N) * h, L.rs, L.rolloff));

    const int AD = p.AD;
    d.tab0 = (int)p.wt.size();
    d.livep0 = (int)p.livep.size();
    p.wt.resize(p.wt.size() + (size_t)p.n_f * 3 * AD, 0.0);
    p.s3.resize(p.s3.size() + (size_t)p.n_f * 3 * AD, 0.0);
    p.livep.resize(p.livep.size() + (size_t)p.n_f * 3 * (AD + 1), 0);
    std::vector<long long> lpts((size_t)p.n_f * 8 * (AD + 1), 0);
    const double ratio = L.spacing / h, half = 0.5 * p.N;
    for (int n = 0; n < p.n_f; ++n) {
        const double f = p.n_f == 1 ? 0.0 : -0.5 * L.rs + (n + 0.5) * L.rs / p.n_f;
        std::vector<unsigned char> liv(3 * AD, 0);
        for (int l = 0; l < 3; ++l) {
            int* lp = &p.livep[d.livep0 + ((size_t)n * 3 + l) * (AD + 1)];
            for (int m = 0; m < AD; ++m) {
                const double u = (double)(m + 1 - p.N) - f / h - (l - 1) * ratio;  // f3 / h
                const double au = std::fabs(u);
                double w = 0.0, sv = 0.0;
                if (au < half - TIE_TOL) {
                    w = 1.0;
                    sv = field_S(u * h, L.rs, L.rolloff);
                } else if (au <= half + TIE_TOL) {
                    w = 0.5;  // boundary: the cell is split between two islands
                    sv = L.rolloff == 0.0 ? 1.0 / L.rs : field_S(u * h, L.rs, L.rolloff);
                }
                const size_t o = d.tab0 + ((size_t)n * 3 + l) * AD + m;
                p.wt[o] = w;
                p.s3[o] = sv;
                liv[l * AD + m] = (w > 0.0 && sv != 0.0);
                lp[m + 1] = lp[m] + liv[l * AD + m];
            }
        }
        for (int mask = 0; mask < 8; ++mask) {
            long long* pp = &lpts[((size_t)n * 8 + mask) * (AD + 1)];
            for (int m = 0; m < AD; ++m) {
                bool any = false;
                for (int l = 0; l < 3; ++l) any |= ((mask >> l) & 1) && liv[l * AD + m];
                const int len = std::min(m + 1, 2 * p.N - 1 - m);
                pp[m + 1] = pp[m] + (any ? len : 0);
            }
        }
    }
    p.livepts.push_back(std::move(lpts));
    p.links.push_back(d);
}

// Instances and folded squares of one link's CUTs.
// Squares of one link's instances, appended to w; instance and square
// indices are offset by inst_base and item_base (their positions in the plan).
void plan_link_work_into(const LinkInput& L, int link, const isrs_numerics* nu, const int32_t* kappa12,
                         int m_explicit, const Plan& p, WorkPart& w, int inst_base, int item_base)
{
    const int nc = L.n_ch, AD = p.AD;
    const LinkDesc& d = p.links[link];
    const bool explicit_sq = kappa12 != nullptr;
    double ksum = 0.0;
    long long steps_per_point = 0;
    for (int s = 0; s < d.n_sp; ++s) {
        ksum += 8.0 * p.spans[d.span0 + s].K + 30.0;
        steps_per_point += p.spans[d.span0 + s].K;
    }
    const double unit_cost = (double)steps_per_point + 15.0 * d.n_sp;
    // square list of one instance: explicit pairs, or every pair of active
    // channels with k1 <= k2 (f1 <-> f2 symmetry: the mirror is folded in)
    std::vector<std::pair<int, int>> pairs;
    if (explicit_sq) {
        for (int t = 0; t < m_explicit; ++t) pairs.emplace_back(kappa12[2 * t], kappa12[2 * t + 1]);
    } else {
        std::vector<int> act;
        for (int k = 0; k < nc; ++k)
            if (L.power[k] > 0) act.push_back(k);
        for (size_t i = 0; i < act.size(); ++i)
            for (size_t j = i; j < act.size(); ++j) pairs.emplace_back(act[i], act[j]);
    }
    for (int q = 0; q < L.n_cut; ++q) {
        const int cut = L.cuts[q];
        for (int n = 0; n < p.n_f; ++n) {
            InstDesc in{};
            in.f = p.n_f == 1 ? 0.0 : -0.5 * L.rs + (n + 0.5) * L.rs / p.n_f;
            in.link = link;
            in.cut = cut;
            in.nf_idx = n;
            in.sq_begin = item_base + (int)w.items.size();
            const int* lp = &p.livep[d.livep0 + (size_t)n * 3 * (AD + 1)];
            int any_live[3];
            for (int l = 0; l < 3; ++l) any_live[l] = lp[l * (AD + 1) + AD] > 0;
            for (const auto& pr : pairs) {
                const int k1 = pr.first, k2 = pr.second;
                const bool pair_active = L.power[k1] > 0 && L.power[k2] > 0;
                SquareItem it{};
                it.inst = inst_base + (int)w.insts.size();
                it.k1 = k1;
                it.k2 = k2;
                it.d_index = -1;
                it.mult = explicit_sq ? 1.0f : (k1 < k2 ? 2.0f : 1.0f);
                for (int l = -1; l <= 1; ++l) {
                    const int k3 = k1 + k2 - cut + l;
                    if (!pair_active || k3 < 0 || k3 >= nc || !(L.power[k3] > 0) || !any_live[l + 1]) continue;
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
                const long long pts = p.livepts[link][((size_t)n * 8 + it.lmask) * (AD + 1) + AD];
                w.live_points += pts;
                w.horner_steps += pts * steps_per_point;
                w.alg_flop += (double)pts * ksum;
                w.items.push_back(it);
                w.item_cost.push_back((double)pts * unit_cost + 1.0);
            }
            in.sq_end = item_base + (int)w.items.size();
            w.insts.push_back(in);
        }
        w.n_cut++;
    }
}

void plan_append(Plan& p, WorkPart& w)
{
    p.insts.insert(p.insts.end(), w.insts.begin(), w.insts.end());
    p.items.insert(p.items.end(), w.items.begin(), w.items.end());
    p.item_cost.insert(p.item_cost.end(), w.item_cost.begin(), w.item_cost.end());
    p.live_points += w.live_points;
    p.horner_steps += w.horner_steps;
    p.alg_flop += w.alg_flop;
    p.n_cut_total += w.n_cut;
    w = WorkPart();
}

void plan_link_work(const LinkInput& L, int link, const isrs_numerics* nu, const int32_t* kappa12, int m_explicit,
                    Plan& p)
{
    WorkPart w;
    plan_link_work_into(L, link, nu, kappa12, m_explicit, p, w, (int)p.insts.size(), (int)p.items.size());
    plan_append(p, w);
}

// The squares of many links, built on host threads (one contiguous range of
// links each) and joined in link order, so the plan does not depend on the
// thread count.
void plan_links_work_parallel(const std::vector<LinkInput>& Ls, const isrs_numerics* nu, Plan& p)
{
    const int n = (int)Ls.size();
    const int nt = std::max(1, std::min<int>(n, std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
    std::vector<WorkPart> parts(n);
    std::vector<std::thread> th;
    std::vector<char> failed(nt, 0);
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            try {
                for (int l = (int)((long long)n * t / nt); l < (int)((long long)n * (t + 1) / nt); ++l)
                    plan_link_work_into(Ls[l], l, nu, nullptr, 0, p, parts[l], 0, 0);
            } catch (...) {
                failed[t] = 1;
            }
        });
    for (auto& x : th) x.join();
    for (char f : failed)
        if (f) throw std::bad_alloc();
    size_t n_items = p.items.size(), n_insts = p.insts.size();
    for (const WorkPart& w : parts) {
        n_items += w.items.size();
        n_insts += w.insts.size();
    }
    p.items.reserve(n_items);
    p.item_cost.reserve(n_items);
    p.insts.reserve(n_insts);
    for (WorkPart& w : parts) {
        const int ib = (int)p.insts.size(), sb = (int)p.items.size();
        for (SquareItem& it : w.items) it.inst += ib;
        for (InstDesc& in : w.insts) {
            in.sq_begin += sb;
            in.sq_end += sb;
        }
        plan_append(p, w);
    }
}



// Coherent-sum rows, launch chunks (surrogate tables only), slice groups and
// queue order.  A plan with coherent sums always runs on the queue: each of
// its persistent blocks owns one accumulator slot.
void plan_finish(Plan& p, const Tuning& tu, int max_items = 0)
{
    p.seg32.resize(p.seg64.size());
    for (size_t i = 0; i < p.seg64.size(); ++i)
        p.seg32[i] = {(float)p.seg64[i].A, (float)p.seg64[i].zeta, (float)p.seg64[i].ratio, 0.0f};
    p.chunk_begin.assign(1, 0);
    p.dlist.clear();
    for (size_t i = 0; i < p.items.size(); ++i) {
        SquareItem& it = p.items[i];
        it.d_index = -1;
        if (max_items > 0 && (int)i - p.chunk_begin.back() == max_items) p.chunk_begin.push_back((int)i);
        if (it.egn_mask == 0) continue;
        it.d_index = (int)p.dlist.size();
        p.dlist.push_back((int)i);
    }
    p.chunk_begin.push_back((int)p.items.size());
    p.tu = tu;
    if (!p.dlist.empty()) p.tu.mode = 1;
    // slice groups: by default enough units to fill the chip with few partials
    const long long n_items = (long long)p.items.size();
    int spb = tu.spb > 0 ? std::min(tu.spb, p.n_slices)
                         : (int)std::min<long long>(p.n_slices, std::max<long long>(1, n_items * p.n_slices / 32768));
    p.spb = spb;
    p.n_groups = (p.n_slices + spb - 1) / spb;
    // queue order per chunk: longest units first.  A square's cost splits
    // evenly over its groups, except that a square with coherent sums runs
    // whole in group 0 (its other groups are empty and go last).
    const size_t n_units = p.items.size() * p.n_groups;
    p.order.resize(n_units);
    std::iota(p.order.begin(), p.order.end(), 0);
    if (p.tu.mode == 1 && p.tu.sort) {
        // stable bucket sort on a cost class (1/64 octave): the queue only needs
        // the longest units first, and the order stays deterministic
        constexpr int NB = 4096;
        auto cls = [&](size_t u) -> int {
            const size_t i = u / p.n_groups;
            double cost = p.item_cost[i] / p.n_groups;
            if (p.items[i].egn_mask != 0) cost = (u % p.n_groups == 0) ? p.item_cost[i] : 0.0;
            const double lc = 64.0 * std::log2(std::max(1.0, cost));
            return (int)(NB - 1 - std::min<double>(NB - 1, std::floor(lc)));
        };
        std::vector<uint16_t> ucls(n_units);
        for (size_t u = 0; u < n_units; ++u) ucls[u] = (uint16_t)cls(u);
        std::vector<int> tmp;
        for (size_t ch = 0; ch + 1 < p.chunk_begin.size(); ++ch) {
            const size_t b = (size_t)p.chunk_begin[ch] * p.n_groups, e = (size_t)p.chunk_begin[ch + 1] * p.n_groups;
            std::vector<size_t> start(NB + 1, 0);
            for (size_t u = b; u < e; ++u) start[ucls[u] + 1]++;
            for (int k = 0; k < NB; ++k) start[k + 1] += start[k];
            tmp.resize(e - b);
            for (size_t u = b; u < e; ++u) tmp[start[ucls[u]]++] = (int)u;
            std::copy(tmp.begin(), tmp.end(), p.order.begin() + b);
        }
    }
}

template <typename T>
size_t staged(const std::vector<T>& v)
{
    return (v.size() * sizeof(T) + 255) & ~size_t(255);
}

template <typename T>
int32_t upload(isrs_ctx* c, hipStream_t st, DevBuf& d, const std::vector<T>& v, char*& stage)
{
    const size_t bytes = v.size() * sizeof(T);
    HIP_TRY(c, d.ensure(bytes));
    if (bytes) {
        std::memcpy(stage, v.data(), bytes);
        HIP_TRY(c, hipMemcpyAsync(d.p, stage, bytes, hipMemcpyHostToDevice, st));
        stage += (bytes + 255) & ~size_t(255);
    }
    return ISRS_OK;
}

// Host-side consistency of the tables the kernels index (every row a kernel
// can address must exist in the uploaded arrays).
std::string plan_check(const Plan& p)
{
    size_t rows = 0;
    const size_t nodes = p.mu_method == MU_INT ? INT_NODES : 1;
    for (const SpanConst& q : p.spans) rows = std::max<size_t>(rows, (size_t)q.off + nodes * q.K);
    if ((p.fp32 ? p.seg32.size() : p.seg64.size()) < rows) return "segment table shorter than the spans need";
    const size_t AD = p.AD;
    for (const LinkDesc& d : p.links) {
        if ((size_t)d.span0 + d.n_sp > p.spans.size()) return "span range out of bounds";
        if ((size_t)d.tab0 + (size_t)p.n_f * 3 * AD > p.wt.size() || p.wt.size() != p.s3.size())
            return "island table out of bounds";
        if ((size_t)d.livep0 + (size_t)p.n_f * 3 * (AD + 1) > p.livep.size()) return "live table out of bounds";
        if ((size_t)d.sg0 + p.N > p.Sg.size()) return "grid table out of bounds";
        if ((size_t)d.ch0 + d.n_ch > p.power.size()) return "channel table out of bounds";
    }
    for (const InstDesc& in : p.insts)
        if (in.link < 0 || in.link >= (int)p.links.size() || in.sq_begin < 0 || in.sq_end > (int)p.items.size() ||
            in.nf_idx < 0 || in.nf_idx >= p.n_f)
            return "instance out of bounds";
    for (const SquareItem& it : p.items) {
        if (it.inst < 0 || it.inst >= (int)p.insts.size()) return "square instance out of bounds";
        const LinkDesc& d = p.links[p.insts[it.inst].link];
        if (it.k1 < 0 || it.k2 < 0 || it.k1 >= d.n_ch || it.k2 >= d.n_ch) return "square channel out of bounds";
    }
    if (p.order.size() != p.items.size() * (size_t)p.n_groups) return "queue order has the wrong length";
    if (p.N > RUN_MASK + 1 || p.runs.empty() || p.n_slices != (int)((p.runs.size() + THREADS - 1) / THREADS))
        return "run table does not match the grid";
    for (size_t c0 = 0; c0 < p.runs.size(); c0 += THREADS) {
        const size_t c1 = std::min(c0 + THREADS, p.runs.size()) - 1;
        if ((p.runs[c1] >> RUN_SHIFT) - (p.runs[c0] >> RUN_SHIFT) + 1 > NAD) return "slice spans too many anti-diagonals";
    }
    for (int r : p.runs)
        if ((r >> RUN_SHIFT) >= p.AD || (r & RUN_MASK) >= p.N) return "run out of the grid";
    if (!region_ppt_supported(p.fp32, p.mu_method, p.ppt)) return "no kernel for this run length";
    if (p.adrun.size() != (size_t)p.AD + 1 || p.adrun.back() != (int)p.runs.size()) return "anti-diagonal run table";
    for (int m = 0; m < p.AD; ++m)
        if (p.adrun[m] >= p.adrun[m + 1] || (p.runs[p.adrun[m]] >> RUN_SHIFT) != m ||
            (p.runs[p.adrun[m]] & RUN_MASK) != std::max(0, m - p.N + 1))
            return "anti-diagonal run table";
    if (!p.dlist.empty() && (p.tu.mode != 1 || p.queue_blocks < 1)) return "coherent sums need the queue";
    for (size_t d = 0; d < p.dlist.size(); ++d)
        if (p.dlist[d] < 0 || p.dlist[d] >= (int)p.items.size() || p.items[p.dlist[d]].d_index != (int)d)
            return "coherent-sum list";
    return "";
}

// Persistent grid of a queue launch (occupancy query: never inside a capture).
void plan_queue_shape(const isrs_ctx* c, Plan& p)
{
    p.queue_blocks = 0;
    if (p.tu.mode != 1) return;
    const int per_cu = region_blocks_per_cu(p.fp32, p.mu_method, p.ppt);
    p.queue_blocks = std::max(1, c->n_cu) * (p.tu.blocks_per_cu > 0 ? std::min(p.tu.blocks_per_cu, per_cu) : per_cu);
}

int32_t plan_upload(isrs_ctx* c, Workspace& w, const Plan& p, hipStream_t st)
{
    const std::string bad = plan_check(p);
    if (!bad.empty()) return fail(c, ISRS_E_ARG, "internal plan check: " + bad);
    if (w.ev_upload) HIP_TRY(c, hipEventSynchronize(w.ev_upload));  // previous copies out of staging
    const size_t need = staged(p.links) + staged(p.spans) + (p.fp32 ? staged(p.seg32) : staged(p.seg64)) +
                        staged(p.Sg) + staged(p.wt) + staged(p.s3) + staged(p.livep) + staged(p.runs) + staged(p.adrun) + staged(p.insts) +
                        staged(p.items) + staged(p.dlist) + staged(p.order) + staged(p.power) + staged(p.phi) +
                        staged(p.psi);
    HIP_TRY(c, w.stage.ensure(need));
    char* stage = reinterpret_cast<char*>(w.stage.p);
    int32_t rc;
    if ((rc = upload(c, st, w.links, p.links, stage))) return rc;
    if ((rc = upload(c, st, w.spans, p.spans, stage))) return rc;
    if (p.fp32) {
        if ((rc = upload(c, st, w.seg, p.seg32, stage))) return rc;
    } else {
        if ((rc = upload(c, st, w.seg, p.seg64, stage))) return rc;
    }
    if ((rc = upload(c, st, w.Sg, p.Sg, stage))) return rc;
    if ((rc = upload(c, st, w.wt, p.wt, stage))) return rc;
    if ((rc = upload(c, st, w.s3, p.s3, stage))) return rc;
    if ((rc = upload(c, st, w.livep, p.livep, stage))) return rc;
    if ((rc = upload(c, st, w.runs, p.runs, stage))) return rc;
    if ((rc = upload(c, st, w.adrun, p.adrun, stage))) return rc;
    if ((rc = upload(c, st, w.insts, p.insts, stage))) return rc;
    if ((rc = upload(c, st, w.items, p.items, stage))) return rc;
    if ((rc = upload(c, st, w.dlist, p.dlist, stage))) return rc;
    if ((rc = upload(c, st, w.order, p.order, stage))) return rc;
    if ((rc = upload(c, st, w.power, p.power, stage))) return rc;
    if ((rc = upload(c, st, w.phi, p.phi, stage))) return rc;
    if ((rc = upload(c, st, w.psi, p.psi, stage))) return rc;
    if (!w.ev_upload) HIP_TRY(c, hipEventCreateWithFlags(&w.ev_upload, hipEventDisableTiming));
    HIP_TRY(c, hipEventRecord(w.ev_upload, st));

    HIP_TRY(c, w.partD.ensure(std::max<size_t>(1, p.items.size()) * p.n_groups * 3 * sizeof(double)));
    HIP_TRY(c, w.partE.ensure(std::max<size_t>(1, p.dlist.size()) * 12 * sizeof(double)));
    if (!p.dlist.empty()) HIP_TRY(c, w.eacc.ensure((size_t)p.queue_blocks * eslot(p.N) * sizeof(double2)));
    HIP_TRY(c, w.counter.ensure(sizeof(int) * std::max<size_t>(1, p.chunk_begin.size())));
    return ISRS_OK;
}

// Device side of a plan carved out of the allocation-free scratch: the
// buffers of plan_upload at fixed offsets, filled by copies from the plan's
// own host vectors, with nothing allocated.  A plan with coherent sums gets as
// many persistent blocks (one accumulator slot each) as fit after its tables.
int32_t plan_upload_scratch(isrs_ctx* c, Workspace& w, Plan& p, char* base, size_t bytes, hipStream_t st)
{
    size_t off = 0;
    auto carve = [&](DevBuf& d, size_t n) {
        d.p = base + off;
        d.cap = n;
        off += (n + 255) & ~size_t(255);
    };
    auto nb = [](const auto& v) { return v.size() * sizeof(v[0]); };
    carve(w.links, nb(p.links));
    carve(w.spans, nb(p.spans));
    carve(w.seg, p.fp32 ? nb(p.seg32) : nb(p.seg64));
    carve(w.Sg, nb(p.Sg));
    carve(w.wt, nb(p.wt));
    carve(w.s3, nb(p.s3));
    carve(w.livep, nb(p.livep));
    carve(w.runs, nb(p.runs));
    carve(w.adrun, nb(p.adrun));
    carve(w.insts, nb(p.insts));
    carve(w.items, nb(p.items));
    carve(w.order, nb(p.order));
    carve(w.power, nb(p.power));
    carve(w.phi, nb(p.phi));
    carve(w.psi, nb(p.psi));
    carve(w.partD, std::max<size_t>(1, p.items.size()) * p.n_groups * 3 * sizeof(double));
    carve(w.partE, std::max<size_t>(1, p.dlist.size()) * 12 * sizeof(double));
    carve(w.counter, sizeof(int) * std::max<size_t>(1, p.chunk_begin.size()));
    const size_t slot = eslot(p.N) * sizeof(double2);
    if (!p.dlist.empty()) {
        const size_t fit = off < bytes ? (bytes - off) / slot : 0;
        if (fit >= 1) {
            p.queue_blocks = (int)std::min<size_t>((size_t)p.queue_blocks, fit);
            carve(w.eacc, (size_t)p.queue_blocks * slot);
        } else {
            off += slot;
        }
    }
    if (off > bytes)
        return fail(c, ISRS_E_ARG, "the evaluation needs " + std::to_string(off) +
                                       " bytes of device scratch; the allocation-free entry point has " +
                                       std::to_string(bytes));
    const std::string bad = plan_check(p);
    if (!bad.empty()) return fail(c, ISRS_E_ARG, "internal plan check: " + bad);
    auto put = [&](DevBuf& d, const void* src, size_t n) -> int32_t {
        if (n) HIP_TRY(c, hipMemcpyAsync(d.p, src, n, hipMemcpyHostToDevice, st));
        return ISRS_OK;
    };
    int32_t rc;
    if ((rc = put(w.links, p.links.data(), nb(p.links)))) return rc;
    if ((rc = put(w.spans, p.spans.data(), nb(p.spans)))) return rc;
    if (p.fp32) {
        if ((rc = put(w.seg, p.seg32.data(), nb(p.seg32)))) return rc;
    } else {
        if ((rc = put(w.seg, p.seg64.data(), nb(p.seg64)))) return rc;
    }
    if ((rc = put(w.Sg, p.Sg.data(), nb(p.Sg)))) return rc;
    if ((rc = put(w.wt, p.wt.data(), nb(p.wt)))) return rc;
    if ((rc = put(w.s3, p.s3.data(), nb(p.s3)))) return rc;
    if ((rc = put(w.livep, p.livep.data(), nb(p.livep)))) return rc;
    if ((rc = put(w.runs, p.runs.data(), nb(p.runs)))) return rc;
    if ((rc = put(w.adrun, p.adrun.data(), nb(p.adrun)))) return rc;
    if ((rc = put(w.insts, p.insts.data(), nb(p.insts)))) return rc;
    if ((rc = put(w.items, p.items.data(), nb(p.items)))) return rc;
    if ((rc = put(w.order, p.order.data(), nb(p.order)))) return rc;
    if ((rc = put(w.power, p.power.data(), nb(p.power)))) return rc;
    if ((rc = put(w.phi, p.phi.data(), nb(p.phi)))) return rc;
    if ((rc = put(w.psi, p.psi.data(), nb(p.psi)))) return rc;
    return ISRS_OK;
}

hipEvent_t pool_event(Workspace& w, size_t i)
{
    while (w.ev_pool.size() <= i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        w.ev_pool.push_back(e);
    }
    return w.ev_pool[i];
}

struct Timings {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> reg, asm_;
};

// Stream-ordered launches of a plan (graph-capturable when timing is off).
int32_t plan_enqueue(isrs_ctx* c, Workspace& w, const Plan& p, hipStream_t st, double* eta_d,
                     double* s2_d, double* terms_d, double* psd_d, bool assemble, Timings* tm,
                     SurrogateFill* sf = nullptr, float* sur_tab = nullptr)
{
    RegionArgs ra{};
    ra.links = w.links.as<LinkDesc>();
    ra.spans = w.spans.as<SpanConst>();
    ra.seg = w.seg.p;
    ra.Sg = w.Sg.as<double>();
    ra.wt = w.wt.as<double>();
    ra.s3 = w.s3.as<double>();
    ra.livep = w.livep.as<int>();
    ra.insts = w.insts.as<InstDesc>();
    ra.items = w.items.as<SquareItem>();
    ra.partD = w.partD.as<double>();
    ra.partE = w.partE.as<double>();
    ra.eacc = p.dlist.empty() ? nullptr : w.eacc.as<double2>();
    ra.adrun = w.adrun.as<int>();
    ra.n_groups = p.n_groups;
    ra.spb = p.spb;
    ra.n_slices = p.n_slices;
    ra.runs = w.runs.as<int>();
    ra.n_runs = (int)p.runs.size();
    ra.N = p.N;
    ra.mu_method = p.mu_method;
    int blocks = 0;
    if (p.tu.mode == 1) {
        blocks = p.queue_blocks;  // fixed at plan time, outside any stream capture
        ra.order = w.order.as<int>();
    }

    size_t ev_i = 0;
    using EvList = std::vector<std::pair<hipEvent_t, hipEvent_t>>;
    auto mark = [&](EvList* v, bool begin) -> int32_t {
        if (!v) return ISRS_OK;
        hipEvent_t e = pool_event(w, ev_i++);
        if (!e) return fail(c, ISRS_E_DEVICE, "event creation failed");
        HIP_TRY(c, hipEventRecord(e, st));
        if (begin)
            v->push_back({e, nullptr});
        else
            v->back().second = e;
        return ISRS_OK;
    };
    EvList* ev_reg = tm ? &tm->reg : nullptr;
    EvList* ev_asm = tm ? &tm->asm_ : nullptr;
    int32_t rc;
    const size_t n_chunks = p.chunk_begin.size() - 1;
    for (size_t ch = 0; ch < n_chunks; ++ch) {
        const int b = p.chunk_begin[ch], e = p.chunk_begin[ch + 1];
        ra.unit0 = b * p.n_groups;
        ra.n_units = (e - b) * p.n_groups;
        if (p.tu.mode == 1) {
            ra.counter = w.counter.as<int>() + ch;
            HIP_TRY(c, launch_zero_counter(ra.counter, st));
        }
        if (sf) {
            ra.sur_tab = sur_tab;
            ra.sur_item0 = b;
            if ((rc = sf->fill(c, ra, b, e, p.links[0].n_sp, sur_tab, st))) return rc;
        }
        if ((rc = mark(ev_reg, true))) return rc;
        HIP_TRY(c, launch_region(ra, blocks, p.fp32, p.ppt, st));
        if ((rc = mark(ev_reg, false))) return rc;
    }
    if (assemble) {
        AssembleArgs aa{};
        aa.links = ra.links;
        aa.insts = ra.insts;
        aa.items = ra.items;
        aa.partD = ra.partD;
        aa.partE = ra.partE;
        aa.power = w.power.as<double>();
        aa.phi = w.phi.as<double>();
        aa.psi = w.psi.as<double>();
        aa.eta = eta_d;
        aa.sigma2 = s2_d;
        aa.terms = terms_d;
        aa.psd = psd_d;
        aa.n_groups = p.n_groups;
        aa.n_f = p.n_f;
        aa.n_cut = p.n_cut_total;
        if ((rc = mark(ev_asm, true))) return rc;
        HIP_TRY(c, launch_assemble(aa, st));
        if ((rc = mark(ev_asm, false))) return rc;
    }
    return ISRS_OK;
}

int32_t collect_timings(isrs_ctx* c, Timings& tm)
{
    auto sum = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, double& out) -> int32_t {
        out = 0;
        for (auto& e : v) {
            HIP_TRY(c, hipEventSynchronize(e.second));
            float ms = 0;
            HIP_TRY(c, hipEventElapsedTime(&ms, e.first, e.second));
            out += ms;
        }
        return ISRS_OK;
    };
    int32_t rc;
    if ((rc = sum(tm.reg, c->stats.region_ms))) return rc;
    c->stats.egn_ms = 0.0;  // the coherent sums run inside the region kernel
    if ((rc = sum(tm.asm_, c->stats.assemble_ms))) return rc;
    return ISRS_OK;
}

void record_stats(isrs_ctx* c, const Plan& p, double host_ms, bool timed)
{
    c->stats.host_prep_ms = host_ms;
    c->stats.region_launches = (int64_t)(p.chunk_begin.size() - 1);
    c->stats.n_squares = (int64_t)p.items.size();
    c->stats.n_delta_squares = (int64_t)p.dlist.size();
    c->stats.n_points_live = p.live_points;
    c->stats.horner_steps = p.mu_method == ISRS_MU_SEGMENT ? p.horner_steps : 0;
    c->stats.alg_flop = p.alg_flop;
    if (!timed) c->stats.region_ms = c->stats.egn_ms = c->stats.assemble_ms = 0;
}

LinkInput ctx_link(const isrs_ctx* c, const int32_t* cuts, int n_cut)
{
    LinkInput L;
    L.n_ch = c->n_ch;
    L.spacing = c->spacing;
    L.rs = c->rs;
    L.rolloff = c->rolloff;
    L.power = c->power.data();
    L.phi = c->phi.data();
    L.psi = c->psi.data();
    L.spans = c->spans.data();
    L.n_sp = (int)c->spans.size();
    L.gain_mode = c->gain_mode;
    L.ptot_override = c->ptot_override;
    L.cuts = cuts;
    L.n_cut = n_cut;
    return L;
}

// Single-link evaluation on the context's workspace.  Outputs are device
// pointers; partials_host receives island partials in explicit-square mode.
// dz_per_cut (nullable): a sampling step per CUT; CUTs sharing a step form one
// link entry of the plan, so the outputs come in plan order, returned in
// plan_order (plan position -> input index).
int32_t evaluate(isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int n_cut, const int32_t* kappa12,
                 int m_explicit, double* eta_d, double* s2_d, double* terms_d, double* psd_d,
                 double* partials_host, SurrogateFill* sf = nullptr, const double* dz_per_cut = nullptr,
                 std::vector<int>* plan_order = nullptr, bool noalloc = false)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!c) return ISRS_E_ARG;
    if (!c->has_spec || !c->has_link) return fail(c, ISRS_E_STATE, "set the spectrum and the link first");
    std::string m = validate_numerics_msg(nu);
    if (!m.empty()) return fail(c, ISRS_E_ARG, m);
    if (!cuts || n_cut < 1) return fail(c, ISRS_E_ARG, "need at least one CUT");
    LinkInput L = ctx_link(c, cuts, n_cut);
    m = validate_link_numerics(L, nu);
    if (!m.empty()) return fail(c, ISRS_E_ARG, m);
    // groups of CUTs by sampling step
    std::vector<double> gdz;
    std::vector<std::vector<int32_t>> gcuts;
    std::vector<int> order;
    if (dz_per_cut) {
        std::vector<int> idx(n_cut);
        std::iota(idx.begin(), idx.end(), 0);
        for (int q = 0; q < n_cut; ++q) {
            isrs_numerics t = *nu;
            t.dz_km = dz_per_cut[q];
            m = validate_numerics_msg(&t);
            if (m.empty()) m = validate_link_numerics(ctx_link(c, cuts + q, 1), &t);
            if (!m.empty()) return fail(c, ISRS_E_ARG, "CUT " + std::to_string(q) + ": " + m);
        }
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return dz_per_cut[a] < dz_per_cut[b]; });
        for (int q : idx) {
            if (gdz.empty() || dz_per_cut[q] != gdz.back()) {
                gdz.push_back(dz_per_cut[q]);
                gcuts.emplace_back();
            }
            gcuts.back().push_back(cuts[q]);
            order.push_back(q);
        }
    } else {
        gdz.push_back(nu->dz_km);
        gcuts.emplace_back(cuts, cuts + n_cut);
        for (int q = 0; q < n_cut; ++q) order.push_back(q);
    }
    if (plan_order) *plan_order = order;
    if (kappa12) {
        for (int t = 0; t < 2 * m_explicit; ++t)
            if (kappa12[t] < 0 || kappa12[t] >= c->n_ch) return fail(c, ISRS_E_ARG, "square index out of range");
    }
    HIP_TRY(c, hipSetDevice(c->device));
    // the surrogate path: FP32 integrand, residual table with segment fallback
    isrs_numerics nn = *nu;
    int max_items = 0;
    if (sf) {
        nn.precision = ISRS_PREC_FP32_PHASE64;
        nn.mu_method = MU_SUR;
        const int64_t rows_per_item = (int64_t)nu->n1 * nu->n1 * (int64_t)c->spans.size();
        max_items = (int)std::max<int64_t>(1, SUR_TAB_ROWS / std::max<int64_t>(1, rows_per_item));
    }
    Plan p;
    Tuning tu;
    try {
        plan_begin(&nn, p);
        for (size_t g = 0; g < gdz.size(); ++g) {
            isrs_numerics ng = nn;
            ng.dz_km = gdz[g];
            LinkInput Lg = L;
            Lg.cuts = gcuts[g].data();
            Lg.n_cut = (int)gcuts[g].size();
            plan_link_tables(Lg, &ng, p);
            plan_link_work(Lg, (int)g, &ng, kappa12, m_explicit, p);
        }
        plan_finish(p, tu, max_items);
        plan_queue_shape(c, p);
    } catch (const std::bad_alloc&) {
        return fail(c, ISRS_E_NOMEM, "host allocation failed");
    }
    int32_t rc;
    if (noalloc) {
        // the device buffers are views into the scratch array; the plan's host
        // vectors stay with the context until the uploads are done
        if (!c->scratch || !c->ev_scratch || sf || partials_host || psd_d)
            return fail(c, ISRS_E_STATE, "allocation-free evaluation unavailable");
        HIP_TRY(c, hipEventSynchronize(c->ev_scratch));
        Workspace view;
        if ((rc = plan_upload_scratch(c, view, p, static_cast<char*>(c->scratch), NOALLOC_BYTES, c->stream)))
            return rc;
        HIP_TRY(c, hipEventRecord(c->ev_scratch, c->stream));
        auto t1 = std::chrono::steady_clock::now();
        if ((rc = plan_enqueue(c, view, p, c->stream, eta_d, s2_d, terms_d, nullptr, true, nullptr))) return rc;
        record_stats(c, p, std::chrono::duration<double, std::milli>(t1 - t0).count(), false);
        std::swap(*c->scratch_plan, p);
        return ISRS_OK;
    }
    Workspace& w = *c->ws;
    if ((rc = plan_upload(c, w, p, c->stream))) return rc;
    if (sf) HIP_TRY(c, w.sur.ensure((size_t)max_items * p.N * p.N * p.links[0].n_sp * sizeof(float)));
    auto t1 = std::chrono::steady_clock::now();
    Timings tm;
    if ((rc = plan_enqueue(c, w, p, c->stream, eta_d, s2_d, terms_d, psd_d, partials_host == nullptr,
                           c->profiling ? &tm : nullptr, sf, sf ? w.sur.as<float>() : nullptr)))
        return rc;
    if (partials_host) {
        std::vector<double> pd(p.items.size() * p.n_groups * 3), pe(std::max<size_t>(1, p.dlist.size()) * 12);
        HIP_TRY(c, hipMemcpyAsync(pd.data(), w.partD.p, pd.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(pe.data(), w.partE.p, pe.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        const double h2 = p.links[0].h * p.links[0].h;
        for (int t = 0; t < m_explicit; ++t) {
            const SquareItem& it = p.items[t];
            for (int l = 0; l < 3; ++l) {
                double D = 0.0;
                for (int g = 0; g < p.n_groups; ++g) D += pd[((size_t)t * p.n_groups + g) * 3 + l];
                double* o = partials_host + (size_t)t * 15 + l * 5;
                const bool valid = (it.lmask >> l) & 1;
                o[0] = valid ? h2 * D : 0.0;
                for (int u = 0; u < 4; ++u)
                    o[1 + u] = (valid && it.d_index >= 0) ? pe[(size_t)it.d_index * 12 + l * 4 + u] : 0.0;
            }
        }
    }
    record_stats(c, p, std::chrono::duration<double, std::milli>(t1 - t0).count(), c->profiling);
    if (c->profiling) return collect_timings(c, tm);
    return ISRS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
struct isrs_batch {
    isrs_ctx* ctx = nullptr;
    int n_links = 0;
    std::vector<int> ch_off, span_off, cut_off;
    std::vector<int32_t> cuts;
    std::vector<double> spacing, rs, rolloff;
    std::vector<int> gain;
    std::vector<double> power, phi, psi;
    std::vector<isrs_span> spans;
    int64_t n_cuts = 0;

    Workspace ws;
    Plan plan;
    bool planned = false;
    isrs_numerics key{};
    Tuning tuning;
    bool warm = false;      // the current plan has run once outside a capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    DevBuf out;

    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    LinkInput link(int l) const
    {
        LinkInput L;
        L.n_ch = ch_off[l + 1] - ch_off[l];
        L.spacing = spacing[l];
        L.rs = rs[l];
        L.rolloff = rolloff[l];
        L.power = power.data() + ch_off[l];
        L.phi = phi.data() + ch_off[l];
        L.psi = psi.data() + ch_off[l];
        L.spans = spans.data() + span_off[l];
        L.n_sp = span_off[l + 1] - span_off[l];
        L.gain_mode = gain[l];
        L.cuts = cuts.data() + cut_off[l];
        L.n_cut = cut_off[l + 1] - cut_off[l];
        return L;
    }
};

namespace {

bool same_numerics(const isrs_numerics& a, const isrs_numerics& b)
{
    return a.dz_km == b.dz_km && a.n1 == b.n1 && a.n2 == b.n2 && a.n_f == b.n_f && a.egn == b.egn &&
           a.precision == b.precision && a.mu_method == b.mu_method;
}

// Plans a batch for the numerics nu and the batch's tuning.  With reuse, a plan
// built for the same numerics keeps its tables and squares and only takes the
// new launch shape (run length, slice groups, queue order, grid).
int32_t batch_plan(isrs_ctx* c, isrs_batch* b, const isrs_numerics* nu, bool reuse = false)
{
    std::string m = validate_numerics_msg(nu);
    if (!m.empty()) return fail(c, ISRS_E_ARG, m);
    for (int l = 0; l < b->n_links; ++l) {
        m = validate_link_numerics(b->link(l), nu);
        if (!m.empty()) return fail(c, ISRS_E_ARG, "link " + std::to_string(l) + ": " + m);
    }
    const bool keep = reuse && b->planned && same_numerics(b->key, *nu);
    b->drop_graph();
    b->planned = false;
    Plan p;
    try {
        if (keep) {
            p = std::move(b->plan);
            plan_runs(p, b->tuning.ppt);
        } else {
            plan_begin(nu, p, b->tuning.ppt);
            std::vector<LinkInput> Ls;
            for (int l = 0; l < b->n_links; ++l) Ls.push_back(b->link(l));
            for (int l = 0; l < b->n_links; ++l) plan_link_tables(Ls[l], nu, p);
            plan_links_work_parallel(Ls, nu, p);
        }
        if (plan_max_slice_rows(p) > NAD) return fail(c, ISRS_E_ARG, "run length too long for this grid");
        plan_finish(p, b->tuning);
        plan_queue_shape(c, p);
    } catch (const std::bad_alloc&) {
        return fail(c, ISRS_E_NOMEM, "host allocation failed");
    }
    HIP_TRY(c, hipSetDevice(c->device));
    int32_t rc = plan_upload(c, b->ws, p, c->stream);
    if (rc) return rc;
    HIP_TRY(c, b->out.ensure(std::max<int64_t>(1, b->n_cuts) * sizeof(double)));
    b->plan = std::move(p);
    b->key = *nu;
    b->planned = true;
    b->warm = false;
    return ISRS_OK;
}

// Runs a planned batch into eta_d.  A new plan runs eagerly once (every
// kernel is loaded and launched outside a capture); later calls capture the
// launches into a graph once and replay it.
int32_t batch_run(isrs_ctx* c, isrs_batch* b, double* eta_d, bool use_graph)
{
    if (c->profiling || !use_graph || !b->warm) {
        b->warm = true;
        Timings tm;
        int32_t rc = plan_enqueue(c, b->ws, b->plan, c->stream, eta_d, nullptr, nullptr, nullptr, true,
                                  c->profiling ? &tm : nullptr);
        if (rc) return rc;
        record_stats(c, b->plan, 0.0, c->profiling);
        if (c->profiling) return collect_timings(c, tm);
        return ISRS_OK;
    }
    if (!b->exec) {
        HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        int32_t rc = plan_enqueue(c, b->ws, b->plan, c->stream, b->out.as<double>(), nullptr, nullptr,
                                  nullptr, true, nullptr);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
        b->graph = g;
        HIP_TRY(c, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    HIP_TRY(c, hipGraphLaunch(b->exec, c->stream));
    if (eta_d != b->out.as<double>())
        HIP_TRY(c, hipMemcpyAsync(eta_d, b->out.p, b->n_cuts * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    record_stats(c, b->plan, 0.0, false);
    return ISRS_OK;
}

std::string tune_key(const isrs_batch* b, const isrs_numerics* nu, const char* arch)
{
    int kmax = 0, smax = 0;
    for (int l = 0; l < b->n_links; ++l) {
        const LinkInput L = b->link(l);
        smax = std::max(smax, L.n_sp);
        for (int s = 0; s < L.n_sp; ++s) kmax = std::max(kmax, (int)std::ceil(L.spans[s].length_km / nu->dz_km));
    }
    std::ostringstream os;
    os << arch << "|runs|N" << nu->n1 << "|K" << ((kmax + 31) / 32) * 32 << "|S" << ((smax + 7) / 8) * 8 << "|P"
       << nu->precision << "|M" << nu->mu_method << "|F" << nu->n_f;
    return os.str();
}

// Minimal line-oriented cache: one `key mode bpc sort spb ms` record per line.
std::map<std::string, std::vector<double>> read_cache(const char* path)
{
    std::map<std::string, std::vector<double>> out;
    if (!path) return out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        // {"key": "...", "mode": m, "blocks_per_cu": b, "sort": s, "slices": p, "ppt": r, "ms": t}
        auto kpos = line.find("\"key\": \"");
        if (kpos == std::string::npos) continue;
        auto kend = line.find('"', kpos + 8);
        std::string key = line.substr(kpos + 8, kend - kpos - 8);
        std::vector<double> v;
        for (const char* name :
             {"\"mode\": ", "\"blocks_per_cu\": ", "\"sort\": ", "\"slices\": ", "\"ppt\": ", "\"ms\": "}) {
            auto p = line.find(name);
            if (p == std::string::npos) break;
            v.push_back(std::atof(line.c_str() + p + std::strlen(name)));
        }
        if (v.size() == 6) out[key] = v;
    }
    return out;
}

bool write_cache(const char* path, const std::map<std::string, std::vector<double>>& m)
{
    if (!path) return true;
    std::ofstream f(path, std::ios::trunc);
    if (!f) return false;
    f << "[\n";
    size_t i = 0;
    for (auto& kv : m) {
        f << "{\"key\": \"" << kv.first << "\", \"mode\": " << (int)kv.second[0]
          << ", \"blocks_per_cu\": " << (int)kv.second[1] << ", \"sort\": " << (int)kv.second[2]
          << ", \"slices\": " << (int)kv.second[3] << ", \"ppt\": " << (int)kv.second[4]
          << ", \"ms\": " << kv.second[5] << "}"
          << (++i < m.size() ? ",\n" : "\n");
    }
    f << "]\n";
    return (bool)f;
}

}  // namespace

namespace isrs {
hipStream_t ctx_stream(isrs_ctx* c) { return c->stream; }
int ctx_device(const isrs_ctx* c) { return c->device; }
int ctx_num_cu(const isrs_ctx* c) { return c->n_cu; }
int32_t ctx_fail(isrs_ctx* c, int32_t code, const char* msg) { return fail(c, code, msg); }

int batch_num_links(const isrs_batch* b) { return b ? b->n_links : 0; }

LinkView batch_link_view(const isrs_batch* b, int link)
{
    const LinkInput L = b->link(link);
    return {L.n_ch, L.spacing, L.rs, L.rolloff, L.power, L.spans, L.n_sp, L.cuts, L.n_cut};
}

int32_t eval_eta_table(isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int n_cut, SurrogateFill& sf,
                       double* eta_host)
{
    if (!c) return ISRS_E_ARG;
    if (!eta_host) return fail(c, ISRS_E_ARG, "eta output is null");
    if (n_cut < 1) return fail(c, ISRS_E_ARG, "need at least one CUT");
    HIP_TRY(c, hipSetDevice(c->device));
    const size_t n = (size_t)n_cut;
    HIP_TRY(c, c->ws->out.ensure(n * 7 * sizeof(double)));
    double* d = c->ws->out.as<double>();
    int32_t rc = evaluate(c, nu, cuts, n_cut, nullptr, 0, d, d + n, d + 2 * n, nullptr, nullptr, &sf);
    if (rc) return rc;
    std::vector<double> h(n);
    HIP_TRY(c, hipMemcpyAsync(h.data(), d, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t q = 0; q < n; ++q) {
        if (!is_fin(h[q])) return fail(c, ISRS_E_NUMERIC, "non-finite NLI result");
        eta_host[q] = h[q];
    }
    return ISRS_OK;
}
}  // namespace isrs

namespace isrs {
// Status of an exception caught at the C-ABI boundary (none may cross it).
int32_t abi_exception(isrs_ctx* c)
{
    try {
        throw;
    } catch (const std::bad_alloc&) {
        return c ? fail(c, ISRS_E_NOMEM, "host allocation failed") : ISRS_E_NOMEM;
    } catch (...) {
        return c ? fail(c, ISRS_E_DEVICE, "unexpected host exception") : ISRS_E_DEVICE;
    }
}
}  // namespace isrs

extern "C" {

const char* isrs_version(void) { return "isrs-egn 0.2 (gfx950)"; }

int32_t isrs_validate_spectrum(const isrs_spectrum* s)
{
    try {
        if (!s) return ISRS_E_ARG;
        return validate_spectrum_msg(s).empty() ? ISRS_OK : ISRS_E_SPECTRUM;
    } catch (...) {
        return abi_exception(nullptr);
    }
}

int32_t isrs_validate_link(const isrs_span* sp, int32_t n, int32_t gain_mode)
{
    try {
        if (!sp) return ISRS_E_ARG;
        if (n < 1 || n > MAX_SPANS) return ISRS_E_ARG;
        return validate_link_msg(sp, n, gain_mode).empty() ? ISRS_OK : ISRS_E_LINK;
    } catch (...) {
        return abi_exception(nullptr);
    }
}

int32_t isrs_validate_numerics(const isrs_numerics* nu)
{
    try {
        return validate_numerics_msg(nu).empty() ? ISRS_OK : ISRS_E_ARG;
    } catch (...) {
        return abi_exception(nullptr);
    }
}

int32_t isrs_create(isrs_ctx** out, int32_t device, void* hip_stream)
{
    try {
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
        Workspace* w = new (std::nothrow) Workspace();
        if (!c || !w) {
            delete c;
            delete w;
            g_create_error = "host allocation failed";
            return ISRS_E_NOMEM;
        }
        c->ws = w;
        c->device = device;
        c->n_cu = prop.multiProcessorCount;
        if (hipSetDevice(device) != hipSuccess) {
            delete w;
            delete c;
            g_create_error = "hipSetDevice failed";
            return ISRS_E_DEVICE;
        }
        // this device's copy of the allocation-free scratch, looked up once per device
        c->scratch_plan = new (std::nothrow) Plan();
        if (!c->scratch_plan || noalloc_scratch(device, &c->scratch) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_scratch, hipEventDisableTiming) != hipSuccess) {
            if (c->ev_scratch) (void)hipEventDestroy(c->ev_scratch);
            delete c->scratch_plan;
            delete w;
            delete c;
            g_create_error = "device scratch lookup failed";
            return ISRS_E_DEVICE;
        }
        if (hip_stream) {
            c->stream = reinterpret_cast<hipStream_t>(hip_stream);
        } else {
            if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
                (void)hipEventDestroy(c->ev_scratch);
                delete c->scratch_plan;
                delete w;
                delete c;
                g_create_error = "stream creation failed";
                return ISRS_E_DEVICE;
            }
            c->own_stream = true;
        }
        *out = c;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(nullptr);
    }
}

int32_t isrs_destroy(isrs_ctx* c)
{
    try {
        if (!c) return ISRS_E_ARG;
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        c->ws->release();
        delete c->ws;
        delete c->scratch_plan;
        if (c->ev_scratch) (void)hipEventDestroy(c->ev_scratch);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

const char* isrs_last_error(const isrs_ctx* c)
{
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

int32_t isrs_set_spectrum(isrs_ctx* c, const isrs_spectrum* s)
{
    try {
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
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_set_link(isrs_ctx* c, const isrs_span* spans, int32_t n, int32_t gain_mode)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!spans || n < 1 || n > MAX_SPANS) return fail(c, ISRS_E_ARG, "bad span array or count");
        std::string m = validate_link_msg(spans, n, gain_mode);
        if (!m.empty()) return fail(c, ISRS_E_LINK, m);
        c->spans.assign(spans, spans + n);
        c->gain_mode = gain_mode;
        c->has_link = true;
        c->err.clear();
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_set_ptot_override(isrs_ctx* c, double ptot_w)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!(is_fin(ptot_w) && ptot_w >= 0)) return fail(c, ISRS_E_ARG, "ptot override must be finite and >= 0");
        c->ptot_override = ptot_w;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_set_profiling(isrs_ctx* c, int32_t profile)
{
    try {
        if (!c) return ISRS_E_ARG;
        c->profiling = profile != 0;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_get_stats(const isrs_ctx* c, isrs_stats* out)
{
    try {
        if (!c || !out) return ISRS_E_ARG;
        *out = c->stats;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(nullptr);
    }
}

int32_t isrs_eval_eta_dev(isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int32_t n_cut, double* eta_dev,
                          double* sigma2_dev, double* terms_dev)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!eta_dev) return fail(c, ISRS_E_ARG, "eta output is null");
        return evaluate(c, nu, cuts, n_cut, nullptr, 0, eta_dev, sigma2_dev, terms_dev, nullptr, nullptr);
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_eval_eta_dev_noalloc(isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int32_t n_cut,
                                  double* eta_dev, double* sigma2_dev, double* terms_dev)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!eta_dev) return fail(c, ISRS_E_ARG, "eta output is null");
        return evaluate(c, nu, cuts, n_cut, nullptr, 0, eta_dev, sigma2_dev, terms_dev, nullptr, nullptr, nullptr,
                        nullptr, nullptr, true);
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_eval_eta(isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int32_t n_cut, double* eta,
                      double* sigma2, double* terms)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!eta) return fail(c, ISRS_E_ARG, "eta output is null");
        if (n_cut < 1) return fail(c, ISRS_E_ARG, "need at least one CUT");
        HIP_TRY(c, hipSetDevice(c->device));
        const size_t n = (size_t)n_cut;
        HIP_TRY(c, c->ws->out.ensure(n * 7 * sizeof(double)));
        double* d = c->ws->out.as<double>();
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
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_eval_eta_dz(isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int32_t n_cut,
                         const double* dz_km, double* eta, double* sigma2, double* terms)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!eta || !dz_km) return fail(c, ISRS_E_ARG, "eta output or step array is null");
        if (n_cut < 1) return fail(c, ISRS_E_ARG, "need at least one CUT");
        HIP_TRY(c, hipSetDevice(c->device));
        const size_t n = (size_t)n_cut;
        HIP_TRY(c, c->ws->out.ensure(n * 7 * sizeof(double)));
        double* d = c->ws->out.as<double>();
        std::vector<int> order;
        int32_t rc = evaluate(c, nu, cuts, n_cut, nullptr, 0, d, d + n, d + 2 * n, nullptr, nullptr, nullptr, dz_km, &order);
        if (rc) return rc;
        std::vector<double> h(n * 7);
        HIP_TRY(c, hipMemcpyAsync(h.data(), d, n * 7 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (size_t pos = 0; pos < n; ++pos) {
            const size_t q = (size_t)order[pos];
            if (!is_fin(h[pos]) || !is_fin(h[n + pos])) return fail(c, ISRS_E_NUMERIC, "non-finite NLI result");
            eta[q] = h[pos];
            if (sigma2) sigma2[q] = h[n + pos];
            if (terms)
                for (int u = 0; u < 5; ++u) terms[q * 5 + u] = h[2 * n + pos * 5 + u];
        }
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_choose_dz(isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int32_t n_cut,
                       const double* candidates, int32_t n_cand, double target_db, double* dz_out,
                       double* err_db_out)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!nu || !cuts || !candidates || !dz_out || n_cut < 1 || n_cand < 1)
            return fail(c, ISRS_E_ARG, "null argument or empty candidate / CUT list");
        if (!(is_fin(target_db) && target_db >= 0)) return fail(c, ISRS_E_ARG, "target must be finite and >= 0");
        std::vector<double> cand(candidates, candidates + n_cand);
        for (double v : cand)
            if (!(is_fin(v) && v > 0)) return fail(c, ISRS_E_ARG, "candidate steps must be finite and > 0");
        std::sort(cand.begin(), cand.end());
        const size_t n = (size_t)n_cut;
        std::vector<double> ref(n), cur(n);
        isrs_numerics t = *nu;
        t.dz_km = cand[0];
        int32_t rc = isrs_eval_eta(c, &t, cuts, n_cut, ref.data(), nullptr, nullptr);
        if (rc) return rc;
        for (size_t q = 0; q < n; ++q) dz_out[q] = cand[0];
        for (int i = 0; i < n_cand; ++i) {
            if (i > 0) {
                t.dz_km = cand[i];
                if ((rc = isrs_eval_eta(c, &t, cuts, n_cut, cur.data(), nullptr, nullptr))) return rc;
            } else {
                cur = ref;
            }
            for (size_t q = 0; q < n; ++q) {
                const double e = 10.0 * std::log10(cur[q] / ref[q]);
                if (err_db_out) err_db_out[(size_t)i * n + q] = e;
                if (std::fabs(e) <= target_db) dz_out[q] = std::max(dz_out[q], cand[i]);
            }
        }
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_eval_psd(isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int32_t n_cut, double* f_thz,
                      double* psd)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!f_thz || !psd) return fail(c, ISRS_E_ARG, "output is null");
        std::string m = validate_numerics_msg(nu);
        if (!m.empty()) return fail(c, ISRS_E_ARG, m);
        if (n_cut < 1) return fail(c, ISRS_E_ARG, "need at least one CUT");
        HIP_TRY(c, hipSetDevice(c->device));
        const size_t n = (size_t)n_cut, nf = (size_t)nu->n_f;
        HIP_TRY(c, c->ws->out.ensure(n * (1 + nf) * sizeof(double)));
        double* d = c->ws->out.as<double>();
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
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_eval_islands(isrs_ctx* c, const isrs_numerics* nu, int32_t cut, const int32_t* kappa12, int32_t m,
                          double* partials)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!kappa12 || m < 1 || !partials) return fail(c, ISRS_E_ARG, "bad square list or output");
        if (nu && nu->n_f != 1) return fail(c, ISRS_E_ARG, "island partials are defined at f = 0 (n_f = 1)");
        int32_t cuts[1] = {cut};
        int32_t rc = evaluate(c, nu, cuts, 1, kappa12, m, nullptr, nullptr, nullptr, nullptr, partials);
        if (rc) return rc;
        for (size_t t = 0; t < (size_t)m * 15; ++t)
            if (!is_fin(partials[t])) return fail(c, ISRS_E_NUMERIC, "non-finite island partial");
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_batch_create(isrs_ctx* c, const isrs_link_batch* in, isrs_batch** out)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!in || !out) return fail(c, ISRS_E_ARG, "batch or output is null");
        *out = nullptr;
        if (in->n_links < 1 || !in->ch_offset || !in->span_offset || !in->spacing_thz || !in->symbol_rate_thz ||
            !in->rolloff || !in->power_w || !in->phi || !in->psi || !in->spans)
            return fail(c, ISRS_E_ARG, "batch arrays must not be null and n_links >= 1");
        if ((in->cut_offset == nullptr) != (in->cuts == nullptr))
            return fail(c, ISRS_E_ARG, "cut_offset and cuts must both be set or both be null");
        isrs_batch* b = new (std::nothrow) isrs_batch();
        if (!b) return fail(c, ISRS_E_NOMEM, "host allocation failed");
        b->ctx = c;
        b->n_links = in->n_links;
        const int nl = in->n_links;
        b->cut_off.push_back(0);
        for (int l = 0; l < nl; ++l) {
            const int c0 = in->ch_offset[l], c1 = in->ch_offset[l + 1];
            const int s0 = in->span_offset[l], s1 = in->span_offset[l + 1];
            const std::string where = "link " + std::to_string(l) + ": ";
            if (c0 < 0 || c1 <= c0 || s0 < 0 || s1 <= s0 || (l == 0 && (c0 != 0 || s0 != 0))) {
                delete b;
                return fail(c, ISRS_E_ARG, where + "bad channel or span offsets");
            }
            std::string m = validate_spectrum_fields(c1 - c0, in->spacing_thz[l], in->symbol_rate_thz[l],
                                                     in->rolloff[l], in->power_w + c0, in->phi + c0, in->psi + c0);
            if (!m.empty()) {
                delete b;
                return fail(c, ISRS_E_SPECTRUM, where + m);
            }
            const int gm = in->gain_mode ? in->gain_mode[l] : ISRS_GAIN_EQUALIZED;
            m = validate_link_msg(in->spans + s0, s1 - s0, gm);
            if (!m.empty()) {
                delete b;
                return fail(c, ISRS_E_LINK, where + m);
            }
            if (in->cuts) {
                const int q0 = in->cut_offset[l], q1 = in->cut_offset[l + 1];
                if (q0 < 0 || q1 < q0 || q0 != b->cut_off.back()) {
                    delete b;
                    return fail(c, ISRS_E_ARG, where + "bad cut offsets");
                }
                for (int q = q0; q < q1; ++q) {
                    const int k = in->cuts[q];
                    if (k < 0 || k >= c1 - c0 || !(in->power_w[c0 + k] > 0)) {
                        delete b;
                        return fail(c, ISRS_E_ARG, where + "CUT out of range or inactive");
                    }
                    b->cuts.push_back(k);
                }
            } else {
                for (int k = 0; k < c1 - c0; ++k)
                    if (in->power_w[c0 + k] > 0) b->cuts.push_back(k);
            }
            b->cut_off.push_back((int)b->cuts.size());
            b->spacing.push_back(in->spacing_thz[l]);
            b->rs.push_back(in->symbol_rate_thz[l]);
            b->rolloff.push_back(in->rolloff[l]);
            b->gain.push_back(gm);
        }
        const int nch = in->ch_offset[nl], nsp = in->span_offset[nl];
        b->ch_off.assign(in->ch_offset, in->ch_offset + nl + 1);
        b->span_off.assign(in->span_offset, in->span_offset + nl + 1);
        b->power.assign(in->power_w, in->power_w + nch);
        b->phi.assign(in->phi, in->phi + nch);
        b->psi.assign(in->psi, in->psi + nch);
        b->spans.assign(in->spans, in->spans + nsp);
        b->n_cuts = (int64_t)b->cuts.size();
        b->tuning.mode = 1;  // queue by default for batches
        *out = b;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_batch_destroy(isrs_batch* b)
{
    try {
        if (!b) return ISRS_E_ARG;
        if (b->ctx) {
            (void)hipSetDevice(b->ctx->device);
            (void)hipStreamSynchronize(b->ctx->stream);
        }
        b->drop_graph();
        b->ws.release();
        b->out.release();
        delete b;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(nullptr);
    }
}

int32_t isrs_batch_num_cuts(const isrs_batch* b, int64_t* n)
{
    try {
        if (!b || !n) return ISRS_E_ARG;
        *n = b->n_cuts;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(nullptr);
    }
}

int32_t isrs_batch_eval_dev(isrs_ctx* c, isrs_batch* b, const isrs_numerics* nu, double* eta_dev)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!b || !eta_dev) return fail(c, ISRS_E_ARG, "batch or output is null");
        if (b->ctx != c) return fail(c, ISRS_E_ARG, "batch belongs to another context");
        std::string m = validate_numerics_msg(nu);
        if (!m.empty()) return fail(c, ISRS_E_ARG, m);
        HIP_TRY(c, hipSetDevice(c->device));
        auto t0 = std::chrono::steady_clock::now();
        if (!b->planned || !same_numerics(b->key, *nu)) {
            int32_t rc = batch_plan(c, b, nu);
            if (rc) return rc;
        }
        auto t1 = std::chrono::steady_clock::now();
        int32_t rc = batch_run(c, b, eta_dev, true);
        c->stats.host_prep_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        return rc;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_batch_eval(isrs_ctx* c, isrs_batch* b, const isrs_numerics* nu, double* eta)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!b || !eta) return fail(c, ISRS_E_ARG, "batch or output is null");
        if (b->ctx != c) return fail(c, ISRS_E_ARG, "batch belongs to another context");
        std::string m = validate_numerics_msg(nu);
        if (!m.empty()) return fail(c, ISRS_E_ARG, m);
        HIP_TRY(c, hipSetDevice(c->device));
        if (!b->planned || !same_numerics(b->key, *nu)) {
            int32_t rc = batch_plan(c, b, nu);
            if (rc) return rc;
        }
        int32_t rc = batch_run(c, b, b->out.as<double>(), true);
        if (rc) return rc;
        std::vector<double> h(b->n_cuts);
        HIP_TRY(c, hipMemcpyAsync(h.data(), b->out.p, b->n_cuts * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int64_t q = 0; q < b->n_cuts; ++q) {
            if (!is_fin(h[q])) return fail(c, ISRS_E_NUMERIC, "non-finite NLI result");
            eta[q] = h[q];
        }
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_batch_get_tuning(const isrs_batch* b, int32_t* mode, int32_t* bpc, int32_t* sort, int32_t* slices,
                              int32_t* points_per_run)
{
    try {
        if (!b) return ISRS_E_ARG;
        const Tuning& t = b->planned ? b->plan.tu : b->tuning;
        if (mode) *mode = t.mode;
        if (bpc) *bpc = t.blocks_per_cu;
        if (sort) *sort = t.sort;
        if (slices) *slices = b->planned ? b->plan.spb : b->tuning.spb;
        if (points_per_run) *points_per_run = b->planned ? b->plan.ppt : b->tuning.ppt;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(nullptr);
    }
}

int32_t isrs_autotune(isrs_ctx* c, isrs_batch* b, const isrs_numerics* nu, const char* cache_path)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!b) return fail(c, ISRS_E_ARG, "batch is null");
        if (b->ctx != c) return fail(c, ISRS_E_ARG, "batch belongs to another context");
        std::string m = validate_numerics_msg(nu);
        if (!m.empty()) return fail(c, ISRS_E_ARG, m);
        HIP_TRY(c, hipSetDevice(c->device));
        hipDeviceProp_t prop;
        HIP_TRY(c, hipGetDeviceProperties(&prop, c->device));
        char arch[64];
        std::snprintf(arch, sizeof arch, "%.20s-%dcu", prop.gcnArchName, prop.multiProcessorCount);
        const std::string key = tune_key(b, nu, arch);
        auto cache = read_cache(cache_path);
        auto hit = cache.find(key);
        if (hit != cache.end()) {
            const auto& v = hit->second;
            b->tuning = {(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4]};
            return batch_plan(c, b, nu, true);
        }
        // candidates: queue mode (the only one for coherent sums) with 2 or 4
        // blocks per CU, the automatic slice grouping or one slice per unit,
        // and every run length with a kernel instance whose slices fit the
        // staged rows; without format terms also the grid mode
        Plan shape;
        plan_begin(nu, shape);
        std::vector<int> ppts;
        for (int r : {ppt_of(shape.fp32), 2, 4, 8}) {
            if (std::find(ppts.begin(), ppts.end(), r) != ppts.end()) continue;
            if (!region_ppt_supported(shape.fp32, nu->mu_method, r)) continue;
            plan_runs(shape, r);
            if (plan_max_slice_rows(shape) <= NAD) ppts.push_back(r);
        }
        std::vector<Tuning> cands;
        for (int r : ppts)
            for (int spb : {0, 1}) {
                if (!nu->egn) cands.push_back({0, 0, 0, spb, r});
                for (int bpc : {4, 2}) cands.push_back({1, bpc, 1, spb, r});
            }
        const bool prof = c->profiling;
        c->profiling = true;
        double best = 1e300;
        Tuning best_t = b->tuning;
        bool first = true;
        for (const Tuning& t : cands) {
            b->tuning = t;
            int32_t rc = batch_plan(c, b, nu, true);
            if (!rc && first) rc = batch_run(c, b, b->out.as<double>(), false);  // loads the kernels
            first = false;
            if (!rc) rc = batch_run(c, b, b->out.as<double>(), false);
            if (rc) {
                c->profiling = prof;
                return rc;
            }
            const double ms = c->stats.region_ms;
            if (ms < best) {
                best = ms;
                best_t = t;
            }
        }
        c->profiling = prof;
        b->tuning = best_t;
        int32_t rc = batch_plan(c, b, nu, true);
        if (rc) return rc;
        cache[key] = {(double)best_t.mode, (double)best_t.blocks_per_cu, (double)best_t.sort, (double)best_t.spb,
                      (double)b->plan.ppt, best};
        if (!write_cache(cache_path, cache)) return fail(c, ISRS_E_ARG, "cannot write the autotune cache file");
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

}  // extern "C"
