// isrs_kernels.hip -- gfx950 kernels of the ISRS-aware EGN hot path.
//
//   region   : per channel-pair square, the link function Upsilon (Eq. 22) on
//              the N x N grid, with the per-span FWM efficiency factor from
//              the segment closed form (Eqs. 7-10) or the Maclaurin form
//              (Eqs. 2-6), and the GN island sums D (Eq. 17).
//   egn      : coherent row / column / anti-diagonal / full sums of Upsilon
//              for the modulation-format terms E, F, G, H (Eqs. 18-21).
//   assemble : per CUT, the ordered FP64 sum over islands of Eq. 15 and the
//              NLI coefficient of Eq. 11.
//
// Segment form as evaluated here: with q = exp((i chi - alpha) Delta) every
// term of Eq. 9 is I_k = q^k I_0, I_0 = (q - 1) / (i chi - alpha), so
//   mu_s = I_0 * P(q),   P(q) = sum_k g_k q^k,   g_k = SRS_G(z_k, f3abs)
// (Eq. 8, z_k of Eq. 10).  P has real coefficients, so it is evaluated with
// the Goertzel recurrence (G. Goertzel, 1958): with t = 2 Re q and s = |q|^2,
//   b_k = g_k + t b_{k+1} - s b_{k+2},   P(q) = b_0 - conj(q) b_1,
// two real FMAs per segment (q and conj(q) are the roots of x^2 - t x + s).
// s = exp(-2 alpha Delta) is a per-span constant.  g_k depends on the point
// only through f1 + f2 (its anti-diagonal), so each thread owns PPT
// consecutive points of one anti-diagonal and reads one staged LDS row for
// all of them.  Phases are formed in FP64 in revolutions and reduced modulo
// one revolution, in FP64, before the sine / cosine.
#include "isrs_internal.h"

#include <mutex>

namespace isrs {

// Scratch of the allocation-free evaluation.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol):
// it passes the device address that hipGetSymbolAddress returns for the
// current device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void** ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

namespace {

template <typename R>
struct Prec;
template <>
struct Prec<float> {
    using V2 = float2;
    using Vec = float4;             // one 16-byte LDS read = 4 segments
    using Seg = SegRow32;
    static constexpr int KC = 128;  // segments staged per pass
    static constexpr int KP = 132;  // LDS row stride (elements): 16-byte rows, 4 banks apart
    static constexpr int VW = 4;    // elements per Vec
};
template <>
struct Prec<double> {
    using V2 = double2;
    using Vec = double2;
    using Seg = SegRow64;
    static constexpr int KC = 100;  // one pass for spans up to 100 km at 1 km; 51 KB of rows, 3 blocks per CU
    static constexpr int KP = 102;
    static constexpr int VW = 2;
};

__device__ __forceinline__ void sincos_rev(float t, float* s, float* c)
{
    // hardware sine / cosine take revolutions; 0 <= t < 1 here
    *s = __builtin_amdgcn_sinf(t);
    *c = __builtin_amdgcn_cosf(t);
}

// Sine and cosine of 2 pi t for a phase t in revolutions (|t| < 2^52), in
// FP64, with no quadrant logic: v = t - rint(t) is exact and |v| <= 1/2; the
// half angle pi v (at most pi/2) takes minimax polynomials sin(pi v) = v S(v^2)
// and cos(pi v) = 1 + v^2 C(v^2) (S and C of degree 7, from
// gen_sincos_coeffs.py), then one doubling: cos 2x = 2 cos^2 x - 1,
// sin 2x = 2 cos x sin x.  Absolute error 5.2e-16 after FP64 evaluation.
__device__ __forceinline__ void sincos_turns(double t, double* s, double* c)
{
    const double v = t - rint(t);
    const double w = v * v;
    double ps = -2.1122952923797757e-05;
    ps = fma(ps, w, 0.00046597761697049093);
    ps = fma(ps, w, -0.0073703610716640494);
    ps = fma(ps, w, 0.08214587825654909);
    ps = fma(ps, w, -0.5992645287757093);
    ps = fma(ps, w, 2.5501640398597765);
    ps = fma(ps, w, -5.167712780049753);
    ps = fma(ps, w, 3.1415926535897927);
    const double sh = v * ps;
    double pc = 4.150750240995467e-06;
    pc = fma(pc, w, -0.00010456780740967329);
    pc = fma(pc, w, 0.00192955681790851);
    pc = fma(pc, w, -0.025806888862681114);
    pc = fma(pc, w, 0.23533063014598704);
    pc = fma(pc, w, -1.3352627688446645);
    pc = fma(pc, w, 4.058712126416545);
    pc = fma(pc, w, -4.934802200544677);
    const double ch = fma(w, pc, 1.0);
    const double c2 = ch + ch;
    *s = c2 * sh;
    *c = fma(c2, ch, -1.0);
}

// t - floor(t) of a phase in revolutions, then in the working precision
template <typename R>
__device__ __forceinline__ R frac_rev(double t)
{
    return R(__builtin_amdgcn_fract(t));
}

// sine and cosine of 2 pi t for a phase t in revolutions given in FP64: the
// FP32 integrand reduces t in FP64 and uses the hardware functions
template <typename R>
__device__ __forceinline__ void sincos_phase(double t, R* s, R* c);
template <>
__device__ __forceinline__ void sincos_phase<float>(double t, float* s, float* c)
{
    sincos_rev(frac_rev<float>(t), s, c);
}
template <>
__device__ __forceinline__ void sincos_phase<double>(double t, double* s, double* c)
{
    sincos_turns(t, s, c);
}

__device__ __forceinline__ float exp_r(float x) { return expf(x); }
__device__ __forceinline__ double exp_r(double x) { return exp(x); }

// a span constant in the working precision (FP32 copies are made on the host)
template <typename R>
__device__ __forceinline__ R spc_r(double d, float f)
{
    if constexpr (sizeof(R) == 4) return f;
    else return d;
}

// e^x of a modest argument: FP32 through the hardware base-2 exponential
__device__ __forceinline__ float exp_fast(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
__device__ __forceinline__ double exp_fast(double x) { return exp(x); }

// exp(-zeta x): FP32 through the hardware base-2 exponential, FP64 exact
__device__ __forceinline__ float exp_neg(float zeta, double x)
{
    return __builtin_amdgcn_exp2f(-zeta * 1.44269504088896341f * float(x));
}
__device__ __forceinline__ double exp_neg(double zeta, double x) { return exp(-zeta * x); }

// 1 / x of a positive normal x: FP32 hardware reciprocal (1 ulp); FP64 the
// hardware approximation refined by one Newton step, which squares its
// relative error (the results agree with a second step to 3e-15 dB)
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(fma(-x, r, 1.0), r, r);
}

// segments 4 kq .. 4 kq + 3 of a staged row
__device__ __forceinline__ void load4(const float4* row, int kq, float& g0, float& g1, float& g2, float& g3)
{
    const float4 v = row[kq];
    g0 = v.x;
    g1 = v.y;
    g2 = v.z;
    g3 = v.w;
}
__device__ __forceinline__ void load4(const double2* row, int kq, double& g0, double& g1, double& g2, double& g3)
{
    const double2 a = row[2 * kq], b = row[2 * kq + 1];
    g0 = a.x;
    g1 = a.y;
    g2 = b.x;
    g3 = b.y;
}

__device__ __forceinline__ float4 pack_vec(const float (&g)[4]) { return float4{g[0], g[1], g[2], g[3]}; }
__device__ __forceinline__ double2 pack_vec(const double (&g)[2]) { return double2{g[0], g[1]}; }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Deterministic block sum (fixed shuffle tree, then waves in order).
__device__ double block_sum(double v, double* sh)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    for (int q = 0; q < THREADS / 64; ++q) r += sh[q];
    return r;
}


template <typename R>
using VecOf = typename Prec<R>::Vec;

// m_j = int_{-1}^{1} u^j e^{a u} du, j = 0..3, for a = (ar, ai), e^{a} = (er, ei).
// Power series for |a| < 1; otherwise m_0 = (e^a - e^{-a}) / a and the
// integration-by-parts step m_j = (e^a - (-1)^j e^{-a}) / a - (j / a) m_{j-1}.
template <typename R>
__device__ __forceinline__ void node_moments(R ar, R ai, R er, R ei, R (&mr)[4], R (&mi)[4])
{
    const R a2 = ar * ar + ai * ai;
    if (a2 < R(1)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            mr[j] = R(0);
            mi[j] = R(0);
        }
        R tr = R(1), ti = R(0);   // a^n / n!
        constexpr int TERMS = sizeof(R) == 8 ? 22 : 12;
#pragma unroll
        for (int n = 0; n < TERMS; ++n) {
            if (n > 0) {
                const R inv_n = R(1) / R(n);
                const R nr = (tr * ar - ti * ai) * inv_n;
                ti = (tr * ai + ti * ar) * inv_n;
                tr = nr;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (((j + n) & 1) == 0) {
                    const R w = R(2) / R(j + n + 1);
                    mr[j] += w * tr;
                    mi[j] += w * ti;
                }
        }
        return;
    }
    // 1 / a and e^{-a} = conj(e^a) / |e^a|^2
    const R ir = ar / a2, ii = -ai / a2;
    const R e2 = er * er + ei * ei;
    const R fr = er / e2, fi = -ei / e2;
    R pr = R(0), pim = R(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const R sgn = (j & 1) ? R(-1) : R(1);
        // (e^a - (-1)^j e^{-a} - j m_{j-1}) / a
        const R nr = er - sgn * fr - R(j) * pr, ni = ei - sgn * fi - R(j) * pim;
        mr[j] = nr * ir - ni * ii;
        mi[j] = nr * ii + ni * ir;
        pr = mr[j];
        pim = mi[j];
    }
}

// W_n = sum_j L[n][j] m_j with l_n(u) = sum_j L[n][j] u^j the Lagrange basis of
// the four Gauss-Legendre nodes (monomial coefficients of the inverse Vandermonde).
__constant__ double c_lag[INT_NODES][4] = {
    {-0.092326598440728888, 0.10721484763524003, 0.79876206302836739, -0.92756750850486841},
    {0.59232659844072888, -1.7422341910450931, -0.79876206302836739, 2.3494311759443818},
    {0.59232659844072888, 1.7422341910450931, -0.79876206302836739, -2.3494311759443818},
    {-0.092326598440728888, -0.10721484763524003, 0.79876206302836739, 0.92756750850486841}};

template <typename R>
__device__ __forceinline__ void node_weight(int n, const R (&mr)[4], const R (&mi)[4], R& wr, R& wi)
{
    wr = R(0);
    wi = R(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const R c = R(c_lag[n][j]);
        wr += c * mr[j];
        wi += c * mi[j];
    }
}

// Coherent sums of one slice of a square with format terms (Eqs. 18-21,
// restructured so that each inner integral is a row, column or anti-diagonal
// sum of Upsilon).  The slice's Upsilon goes through LDS (over the staged gain
// rows, which are no longer read); every row, column and anti-diagonal the
// slice touches adds its part, summed in a fixed order, to the block's
// accumulator slot in FP64.  Row and column j belong to thread j mod THREADS,
// anti-diagonal m to thread m mod THREADS, in every slice and square, so no
// two threads ever touch one accumulator and the result is deterministic.
template <typename R, int PPT>
__device__ void egn_slice(const int em, const int N, const int c0, const int c1, const int mlo, const int mhi,
                          const int m, const int i0, const int ihi, const bool has, const R (&ur)[PPT],
                          const R (&ui)[PPT], const double* Sg, const double* wt, const double* s3,
                          const int* __restrict__ adrun, void* lds, double2* acc)
{
    using V2 = typename Prec<R>::V2;
    const int tid = threadIdx.x, AD = 2 * N - 1, nrows = mhi - mlo + 1;
    V2* ys = reinterpret_cast<V2*>(lds);                           // [THREADS * PPT] Upsilon by run position
    double2* rp = reinterpret_cast<double2*>(ys + THREADS * PPT);  // [THREADS] per run: sum of S1 S2 Upsilon
    double* ws = reinterpret_cast<double*>(rp + THREADS);          // [3][NAD] island weight * S(f3)
    int* adr = reinterpret_cast<int*>(ws + 3 * NAD);               // [NAD + 1] first run of each anti-diagonal
    const bool need_ad = (em & 0xCCC) != 0;
    __syncthreads();
    double gr = 0.0, gi = 0.0;
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
        const int ip = i0 + r;
        const bool ok = has && ip <= ihi;
        ys[tid * PPT + r] = ok ? V2{ur[r], ui[r]} : V2{R(0), R(0)};
        if (ok && need_ad) {
            const double w = Sg[ip] * Sg[m - ip];
            gr += w * (double)ur[r];
            gi += w * (double)ui[r];
        }
    }
    rp[tid] = double2{gr, gi};
    if (tid <= nrows) {
        adr[tid] = adrun[mlo + tid];
        if (tid < nrows)
            for (int l = 0; l < 3; ++l) ws[l * NAD + tid] = wt[l * AD + mlo + tid] * s3[l * AD + mlo + tid];
    }
    __syncthreads();
    // rows and columns the slice touches: [lo, hi]; this thread's first one
    const int lo = max(0, mlo - (N - 1)), hi = min(N - 1, mhi);
    const int first = lo + ((tid - lo) % THREADS + THREADS) % THREADS;
    // E (t = 0): row j, the sum over i of w S1 S3 Upsilon (Eq. 18);
    // F (t = 1): column i, the sum over j of w S2 S3 Upsilon (Eq. 19)
    for (int lt = 0; lt < 6; ++lt) {
        const int l = lt >> 1, t = lt & 1;
        if (!((em >> (4 * l + t)) & 1)) continue;
        double2* dst = acc + (3 * t + l) * N;
        for (int x = first; x <= hi; x += THREADS) {
            double cr = 0.0, ci = 0.0;
            for (int q = 0; q < nrows; ++q) {
                const int mm = mlo + q, other = mm - x;   // the point's other index
                if (other < 0 || other >= N) continue;
                const int i = t ? x : other;
                const int off = i - max(0, mm - (N - 1));
                const int run = adr[q] + off / PPT;
                if (run < c0 || run > c1) continue;
                const V2 y = ys[(run - c0) * PPT + off % PPT];
                const double w = ws[l * NAD + q] * Sg[other];
                cr += w * (double)y.x;
                ci += w * (double)y.y;
            }
            double2 v = dst[x];
            v.x += cr;
            v.y += ci;
            dst[x] = v;
        }
    }
    // G and H: anti-diagonal m, sum of S1 S2 Upsilon (Eqs. 20, 21)
    if (need_ad) {
        const int q = ((tid - mlo) % THREADS + THREADS) % THREADS;
        if (q < nrows) {
            const int rb = max(c0, adr[q]), re = min(c1 + 1, adr[q + 1]);
            double sr = 0.0, si = 0.0;
            for (int run = rb; run < re; ++run) {
                sr += rp[run - c0].x;
                si += rp[run - c0].y;
            }
            double2 v = acc[6 * N + mlo + q];
            v.x += sr;
            v.y += si;
            acc[6 * N + mlo + q] = v;
        }
    }
}

// The format terms of a square from its accumulated sums (bare, grid weights
// included):
//   E_l = h^3 sum_j S2^2 |row_l(j)|^2,  F_l = h^3 sum_i S1^2 |col_l(i)|^2,
//   G_l = h^3 sum_m w_l S3_l^2 |ad(m)|^2,  H_l = h^4 |sum_m w_l S3_l ad(m)|^2.
__device__ void egn_finish(const int em, const int N, const double h, const double* Sg, const double* wt,
                           const double* s3, const double2* acc, double* red, double* out)
{
    const int tid = threadIdx.x, AD = 2 * N - 1;
    const double h3 = h * h * h;
    double res[3][4];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        res[l][0] = res[l][1] = res[l][2] = res[l][3] = 0.0;
        if ((em >> (4 * l)) & 1) {
            double v = 0.0;
            for (int j = tid; j < N; j += THREADS) {
                const double2 e = acc[l * N + j];
                v += Sg[j] * Sg[j] * (e.x * e.x + e.y * e.y);
            }
            res[l][0] = h3 * block_sum(v, red);
        }
        if ((em >> (4 * l + 1)) & 1) {
            double v = 0.0;
            for (int i = tid; i < N; i += THREADS) {
                const double2 e = acc[(3 + l) * N + i];
                v += Sg[i] * Sg[i] * (e.x * e.x + e.y * e.y);
            }
            res[l][1] = h3 * block_sum(v, red);
        }
        if ((em >> (4 * l + 2)) & 1) {
            double v = 0.0;
            for (int mm = tid; mm < AD; mm += THREADS) {
                const double2 e = acc[6 * N + mm];
                const double w3 = s3[l * AD + mm];
                v += wt[l * AD + mm] * w3 * w3 * (e.x * e.x + e.y * e.y);
            }
            res[l][2] = h3 * block_sum(v, red);
        }
        if ((em >> (4 * l + 3)) & 1) {
            double vr = 0.0, vi = 0.0;
            for (int mm = tid; mm < AD; mm += THREADS) {
                const double2 e = acc[6 * N + mm];
                const double w = wt[l * AD + mm] * s3[l * AD + mm];
                vr += w * e.x;
                vi += w * e.y;
            }
            const double xr = block_sum(vr, red), xi = block_sum(vi, red);
            res[l][3] = h3 * h * (xr * xr + xi * xi);
        }
    }
    if (tid == 0) {
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int t = 0; t < 4; ++t) out[l * 4 + t] = res[l][t];
    }
}

// One work unit: slice group u % n_groups of square u / n_groups.  The
// square's points are cut into runs of PPT consecutive points along an
// anti-diagonal (f1 + f2 constant), ordered by anti-diagonal; a slice is
// THREADS consecutive runs, one per thread.  The points of a thread share
// their gain row g_k(f3), so one LDS read feeds all of them, and a block
// stages only the few rows its slice spans.
// The span, run and live tables are read through restrict-qualified kernel
// parameters: nothing the kernel writes aliases them, so their block-uniform
// reads go through scalar loads.
template <typename R, int MU, int PPT>
__device__ void region_unit(const RegionArgs& a, const int u, const int slot, VecOf<R>* g_vec, double* red,
                            const SpanConst* __restrict__ spans_all, const int* __restrict__ runs,
                            const int* __restrict__ livep_all)
{
    using P = Prec<R>;
    using Vec = typename P::Vec;
    using Seg = typename P::Seg;
    constexpr int KC = P::KC, KP = P::KP, VW = P::VW, KPV = KP / VW;
    // g_vec: g rows of the slice's anti-diagonals, KPV vectors per row

    const int tid = threadIdx.x;
    const int item = u / a.n_groups;
    const int grp = u % a.n_groups;
    const SquareItem it = a.items[item];
    const InstDesc in = a.insts[it.inst];
    const LinkDesc lk = a.links[in.link];
    const int N = a.N, AD = 2 * N - 1;
    const double h = lk.h, df = lk.spacing;
    const double half_grid = 0.5 * (lk.n_ch - 1);
    // absolute offsets of the square (THz): d1 = d1b + f1, d2 = d2b + f2,
    // a + b = sb + f1 + f2, a + b - c = x3b + f1 + f2, c = cabs
    const double d1b = (it.k1 - in.cut) * df - in.f;
    const double d2b = (it.k2 - in.cut) * df - in.f;
    const double sb = (it.k1 + it.k2 - 2.0 * half_grid) * df;
    const double x3b = (it.k1 + it.k2 - in.cut - half_grid) * df - in.f;
    const double cabs = (in.cut - half_grid) * df + in.f;
    const double* wt = a.wt + lk.tab0 + (size_t)in.nf_idx * 3 * AD;
    const double* s3 = a.s3 + lk.tab0 + (size_t)in.nf_idx * 3 * AD;
    const int* livep = livep_all + lk.livep0 + (size_t)in.nf_idx * 3 * (AD + 1);
    const double* Sg = a.Sg + lk.sg0;
    const SpanConst* spans = spans_all + lk.span0;
    const Seg* seg = reinterpret_cast<const Seg*>(a.seg);
    double dacc[3] = {0.0, 0.0, 0.0};

    // a square with coherent sums runs whole in group 0 (its other groups add
    // nothing), with the sums in this block's accumulator slot
    int sl_begin = grp * a.spb, sl_end = min(a.n_slices, (grp + 1) * a.spb);
    double2* acc = nullptr;
    if (it.egn_mask != 0) {
        sl_end = sl_begin;
        if (grp == 0 && slot >= 0) {
            sl_begin = 0;
            sl_end = a.n_slices;
            acc = a.eacc + (size_t)slot * eslot(N);
            // clear the sums this square uses (E rows, F columns per island; the
            // anti-diagonals for G and H), each entry by the thread that owns it
            for (int lt = 0; lt < 6; ++lt)
                if ((it.egn_mask >> (4 * (lt >> 1) + (lt & 1))) & 1)
                    for (int j = tid; j < N; j += THREADS) acc[(3 * (lt & 1) + (lt >> 1)) * N + j] = double2{0.0, 0.0};
            if (it.egn_mask & 0xCCC)
                for (int mm = tid; mm < AD; mm += THREADS) acc[6 * N + mm] = double2{0.0, 0.0};
        }
    }
    for (int sl = sl_begin; sl < sl_end; ++sl) {
        const int c0 = sl * THREADS;
        const int c1 = min(c0 + THREADS, a.n_runs) - 1;       // last run of the slice
        const int mlo = runs[c0] >> RUN_SHIFT, mhi = runs[c1] >> RUN_SHIFT;
        // this thread's run: anti-diagonal m, points i0 .. i0 + PPT - 1 (i <= ihi)
        const bool has = c0 + tid <= c1;
        const int run = runs[has ? c0 + tid : c1];
        const int m = run >> RUN_SHIFT, i0 = run & RUN_MASK;
        const int ihi = min(m, N - 1);
        // a slice is skipped when none of its anti-diagonals is live
        bool live = false;
#pragma unroll
        for (int l = 0; l < 3; ++l)
            if ((it.lmask >> l) & 1) live |= livep[l * (AD + 1) + mhi + 1] - livep[l * (AD + 1) + mlo] > 0;
        if (!live) continue;

        // per point d12 = (f1 - f)(f2 - f) in FP64; a + b and f3 are the run's
        const double ssum = sb + (m + 1 - N) * h;
        double pa[PPT];
        R ur[PPT], ui[PPT];  // Upsilon of each point
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
            const int ip = min(i0 + r, ihi);   // points past the run's end repeat its last
            pa[r] = (d1b + (ip + 0.5 - 0.5 * N) * h) * (d2b + (m - ip + 0.5 - 0.5 * N) * h);
            ur[r] = R(0);
            ui[r] = R(0);
        }

        for (int s = 0; s < lk.n_sp; ++s) {
            const SpanConst sc = spans[s];
            // phases in revolutions are d12 times a per-run factor (Eqs. 22, 24)
            const double fth = fma(ssum, sc.p3r, sc.p2r);
            const double fq = fma(ssum, sc.c3r, sc.c2r);
            // rotation of the span's contribution: gamma Pi e^{i Theta_s} (Eq. 22)
            R gm = spc_r<R>(sc.gamma, sc.f_gamma);
            if (lk.gain_mode == 1) {
                // a real (block-uniform) branch: the empty asm keeps the
                // compiler from evaluating the exponential for every link
                asm volatile("" ::: "memory");
                gm *= exp_fast(R(sc.pi_a - sc.pi_s * ssum + sc.pi_c * cabs));
            }
            // the segment form applies gamma Pi with 1 / |i chi - alpha|^2 below
            const R gr = MU == MU_SEG ? R(1) : gm;
            R rr[PPT], ri[PPT];
#pragma unroll
            for (int r = 0; r < PPT; ++r) {
                R st, ct;
                sincos_phase<R>(pa[r] * fth, &st, &ct);
                rr[r] = gr * ct;
                ri[r] = gr * st;
            }
            if constexpr (MU == MU_MAC) {
                // Maclaurin form, Eqs. 4-6
                const double fx = fma(ssum, sc.c3x, sc.c2x), fl = fma(ssum, sc.c3L, sc.c2L);
                const R al = spc_r<R>(sc.alpha, sc.f_alpha);
                const R c = R(sc.pcr) * R(ssum - cabs) / al;
#pragma unroll
                for (int r = 0; r < PPT; ++r) {
                    const R ch = R(pa[r] * fx);
                    R sl, cl;
                    sincos_phase<R>(pa[r] * fl, &sl, &cl);
                    const R inv1 = R(1) / (al * al + ch * ch);
                    const R inv2 = R(1) / (R(4) * al * al + ch * ch);
                    // eta = (e^{(i chi - a) L} - 1) / (i chi - a)
                    const R emL = spc_r<R>(sc.emL, sc.f_emL), em2L = spc_r<R>(sc.em2L, sc.f_em2L);
                    R vr = emL * cl - R(1), vi = emL * sl;
                    const R er = (-al * vr + ch * vi) * inv1, ei = (-ch * vr - al * vi) * inv1;
                    // (e^{(i chi - 2a) L} - 1) / (i chi - 2a)
                    vr = em2L * cl - R(1);
                    vi = em2L * sl;
                    const R fr = (R(-2) * al * vr + ch * vi) * inv2, fi = (-ch * vr - R(2) * al * vi) * inv2;
                    const R mr = er - c * (er - fr), mi = ei - c * (ei - fi);
                    ur[r] += rr[r] * mr - ri[r] * mi;
                    ui[r] += rr[r] * mi + ri[r] * mr;
                }
                continue;
            }

            // Surrogate table (MU_SUR): mu = eta_6 e^{r / 2} with eta_6 of Eq. 6 (its
            // phase kept), r the ensemble's residual; NaN rows take the segment
            // form below, which then runs for the whole block.
            bool fb[PPT];
#pragma unroll
            for (int r = 0; r < PPT; ++r) fb[r] = MU != MU_SUR;
            if constexpr (MU == MU_SUR) {
                const double fl = fma(ssum, sc.c3L, sc.c2L);
                bool any = false;
#pragma unroll
                for (int r = 0; r < PPT; ++r) {
                    const int ip = min(i0 + r, ihi);
                    float rv = 0.0f;
                    if (has)
                        rv = a.sur_tab[(((size_t)(item - a.sur_item0) * N + (m - ip)) * N + ip) * lk.n_sp + s];
                    fb[r] = rv != rv;
                    any |= fb[r];
                    if (fb[r]) continue;
                    const R al = spc_r<R>(sc.alpha, sc.f_alpha), ch = R(pa[r] * fq) * spc_r<R>(sc.wd, sc.f_wd);
                    R sl, cl;
                    sincos_phase<R>(pa[r] * fl, &sl, &cl);
                    const R emL = spc_r<R>(sc.emL, sc.f_emL);
                    const R vr = emL * cl - R(1), vi = emL * sl;
                    const R inv = recip(al * al + ch * ch);
                    const R g = exp_r(R(0.5) * R(rv));
                    const R mr = (-al * vr + ch * vi) * inv * g, mi = (-ch * vr - al * vi) * inv * g;
                    ur[r] += rr[r] * mr - ri[r] * mi;
                    ui[r] += rr[r] * mi + ri[r] * mr;
                }
                if (!__syncthreads_or(any)) continue;
            }

            // q = e^{(i chi - alpha) Delta}.  Segment form: the span's factor
            // c = rotation * I_0 with I_0 = (q - 1) / (i chi - alpha) multiplies
            // P(q) = sum_k g_k q^k.  Integral form: node n of every segment gives
            // P_n(q) = sum_k g(z_kn) q^k, weighted by
            // W_n = e^{a} (Delta / 2) int_{-1}^{1} l_n(u) e^{a u} du, a = (i chi - alpha) Delta / 2,
            // l_n the Lagrange basis of the nodes (exact product integration of the
            // interpolated gain against the exponential); c = rotation.
            constexpr int NN = MU == MU_INT ? INT_NODES : 1;
            R qi[PPT], cr[PPT], ci[PPT], tq2[PPT];
            R mre[MU == MU_INT ? PPT : 1][4], mim[MU == MU_INT ? PPT : 1][4];
#pragma unroll
            for (int r = 0; r < PPT; ++r) {
                const double tq = pa[r] * fq;   // chi Delta / 2 pi
                R sq, cq;
                sincos_phase<R>(tq, &sq, &cq);
                const R al = spc_r<R>(sc.alpha, sc.f_alpha), ch = R(tq) * spc_r<R>(sc.wd, sc.f_wd);
                const R em = spc_r<R>(sc.em, sc.f_em);
                qi[r] = em * sq;
                tq2[r] = (R(2) * em) * cq;
                if constexpr (MU == MU_INT) {
                    cr[r] = rr[r];
                    ci[r] = ri[r];
                    // a = (i chi - alpha) Delta / 2 and e^{a}; moments m_j = int u^j e^{a u}
                    R sh, chh;
                    sincos_phase<R>(0.5 * tq, &sh, &chh);
                    const R hd = R(M_PI) / R(sc.wd);                       // Delta / 2
                    const R ar = -al * hd, ai = ch * hd;
                    const R eh = exp_r(ar);
                    node_moments(ar, ai, eh * chh, eh * sh, mre[r], mim[r]);
                    // fold e^{a} Delta / 2 into the moments
                    const R fr = hd * eh * chh, fi = hd * eh * sh;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const R tr = mre[r][j] * fr - mim[r][j] * fi;
                        mim[r][j] = mre[r][j] * fi + mim[r][j] * fr;
                        mre[r][j] = tr;
                    }
                } else {
                    const R vr = fma(em, cq, R(-1)), vi = qi[r];
                    const R inv = (MU == MU_SEG ? gm : R(1)) * recip(al * al + ch * ch);
                    const R i0r = (-al * vr + ch * vi) * inv;
                    const R i0i = (-ch * vr - al * vi) * inv;
                    cr[r] = rr[r] * i0r - ri[r] * i0i;
                    ci[r] = rr[r] * i0i + ri[r] * i0r;
                }
            }
            // Goertzel state per point; s = |q|^2 is uniform over the span
            const R ms = spc_r<R>(-(sc.em * sc.em), sc.f_ms);
            const int Kp4 = (sc.K + 3) & ~3;
            const int nrows = mhi - mlo + 1;
            for (int n = 0; n < NN; ++n) {
                const int row0 = sc.off + n * sc.K;
                constexpr bool PEEL = sizeof(R) == 8;
                R b1[PPT], b2[PPT];
                if constexpr (!PEEL) {
#pragma unroll
                    for (int r = 0; r < PPT; ++r) {
                        b1[r] = R(0);
                        b2[r] = R(0);
                    }
                }
                for (int kc1 = Kp4; kc1 > 0; kc1 -= KC) {
                    const int kc0 = kc1 > KC ? kc1 - KC : 0;
                    const int len = kc1 - kc0;
                    __syncthreads();  // previous readers of the staged rows are done
                    // stage g_k(f3) = A_k exp(-zeta_k f3abs) for the slice's anti-diagonals:
                    // an item is VW consecutive segments of a run of SRUN anti-diagonals,
                    // one exp per segment at the run's first anti-diagonal, then the
                    // step ratio exp(-zeta h) down the run, one vector write per row
                    constexpr int SRUN = STAGE_RUN;
                    const int runs = (nrows + SRUN - 1) / SRUN;
                    const int lenv = len / VW;
                    for (int t = tid; t < lenv * runs; t += THREADS) {
                        const int kv = t % lenv, rn = t / lenv;
                        const double x = x3b + (mlo + rn * SRUN + 1 - N) * h;
                        R g[VW], rt[VW];
#pragma unroll
                        for (int e = 0; e < VW; ++e) {
                            const int k = kc0 + kv * VW + e;
                            g[e] = R(0);
                            rt[e] = R(0);
                            if (k < sc.K) {
                                const Seg row = seg[row0 + k];
                                g[e] = row.A * exp_neg(row.zeta, x);
                                rt[e] = row.ratio;
                            }
                        }
                        Vec* dst = g_vec + (rn * SRUN) * KPV + kv;
                        const int nq = min(SRUN, nrows - rn * SRUN);  // rows of this run
#pragma unroll
                        for (int q = 0; q < SRUN; ++q) {
                            if (q >= nq) break;
                            dst[q * KPV] = pack_vec(g);
#pragma unroll
                            for (int e = 0; e < VW; ++e) g[e] *= rt[e];
                        }
                    }
                    __syncthreads();
                    // all points of the thread read one row.  Four segments per step:
                    // b2 takes b_k, then b1 takes b_{k-1}, so the state never moves
                    // between registers; the older state enters the inner product, so
                    // one FMA per segment is on the dependency chain.
                    // threads past the slice's last run skip it: whole waves of a
                    // square's ragged last slice then leave their SIMD to others
                    const Vec* gb = g_vec + (m - mlo) * KPV;
                    int kq = has ? len / 4 - 1 : -1;
                    if (PEEL && kc1 == Kp4) {
                        // the state starts at zero, so the span's first four steps
                        // drop the terms that would multiply it
                        if (kq >= 0) {
                            R g0, g1, g2, g3;
                            load4(gb, kq, g0, g1, g2, g3);
#pragma unroll
                            for (int r = 0; r < PPT; ++r) {
                                b2[r] = g3;
                                b1[r] = fma(tq2[r], g3, g2);
                                b2[r] = fma(tq2[r], b1[r], fma(ms, g3, g1));
                                b1[r] = fma(tq2[r], b2[r], fma(ms, b1[r], g0));
                            }
                            --kq;
                        } else {
#pragma unroll
                            for (int r = 0; r < PPT; ++r) {
                                b1[r] = R(0);
                                b2[r] = R(0);
                            }
                        }
                    }
#pragma unroll 8
                    for (; kq >= 0; --kq) {
                        R g0, g1, g2, g3;
                        load4(gb, kq, g0, g1, g2, g3);
#pragma unroll
                        for (int r = 0; r < PPT; ++r) {
                            b2[r] = fma(tq2[r], b1[r], fma(ms, b2[r], g3));
                            b1[r] = fma(tq2[r], b2[r], fma(ms, b1[r], g2));
                            b2[r] = fma(tq2[r], b1[r], fma(ms, b2[r], g1));
                            b1[r] = fma(tq2[r], b2[r], fma(ms, b1[r], g0));
                        }
                    }
                }
#pragma unroll
                for (int r = 0; r < PPT; ++r) {
                    // P(q) = b_0 - conj(q) b_1;  Upsilon += c W_n P
                    if (!fb[r]) continue;
                    R pr = b1[r] - R(0.5) * tq2[r] * b2[r], pi = qi[r] * b2[r];
                    if constexpr (MU == MU_INT) {
                        R wr, wi;
                        node_weight(n, mre[r], mim[r], wr, wi);
                        const R tr = wr * pr - wi * pi;
                        pi = wr * pi + wi * pr;
                        pr = tr;
                    }
                    // accumulated as two fused steps each
                    ur[r] = fma(cr[r], pr, fma(-ci[r], pi, ur[r]));
                    ui[r] = fma(cr[r], pi, fma(ci[r], pr, ui[r]));
                }
            }
        }

        if (acc)
            egn_slice<R, PPT>(it.egn_mask, N, c0, c1, mlo, mhi, m, i0, ihi, has, ur, ui, Sg, wt, s3, a.adrun, g_vec,
                         acc);

        // GN island sums (Eq. 17)
        if (!has) continue;
        double vs = 0.0;
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
            const int ip = i0 + r;
            if (ip > ihi) continue;
            const double S1 = Sg[ip], S2 = Sg[m - ip];
            const double u2 = (double)ur[r] * (double)ur[r] + (double)ui[r] * (double)ui[r];
            vs += S1 * S1 * S2 * S2 * u2;
        }
#pragma unroll
        for (int l = 0; l < 3; ++l)
            if ((it.lmask >> l) & 1) {
                const double w3 = s3[l * AD + m];
                dacc[l] += wt[l * AD + m] * w3 * w3 * vs;
            }
    }
    double* out = a.partD + (size_t)u * 3;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const double v = block_sum(dacc[l], red);
        if (tid == 0) out[l] = v;
    }
    if (acc) egn_finish(it.egn_mask, N, h, Sg, wt, s3, acc, red, a.partE + (size_t)it.d_index * 12);
}

// Waves per SIMD the register budget is set for: FP32 at most 128 VGPRs (four
// waves), 168 for the FP32 integral form and 8-point runs (three); FP64 168
// for the segment form (three, a few spills beat two waves), otherwise two.
template <typename R, int MU, int PPT>
constexpr int region_min_waves()
{
    if constexpr (sizeof(R) == 4) return (MU == MU_INT || PPT > 4) ? 3 : 4;
    else return MU == MU_SEG ? 3 : 2;
}

template <typename R, int MU, int PPT>
__global__ void __launch_bounds__(THREADS, (region_min_waves<R, MU, PPT>())) region_kernel(RegionArgs a, const SpanConst* __restrict__ spans,
                                                                                   const int* __restrict__ runs,
                                                                                   const int* __restrict__ livep)
{
    __shared__ VecOf<R> g_vec[NAD * (Prec<R>::KP / Prec<R>::VW)];
    __shared__ double red[THREADS / 64];
    static_assert(sizeof(g_vec) >= THREADS * PPT * sizeof(typename Prec<R>::V2) + THREADS * sizeof(double2) +
                                       3 * NAD * sizeof(double) + (NAD + 1) * sizeof(int),
                  "the coherent-sum staging must fit in the gain rows");
    region_unit<R, MU, PPT>(a, a.unit0 + blockIdx.x, -1, g_vec, red, spans, runs, livep);
}

// Persistent blocks on a queue: every block pops unit positions until the
// launch's units are exhausted, so every block reaches the exit.
template <typename R, int MU, int PPT>
__global__ void __launch_bounds__(THREADS, (region_min_waves<R, MU, PPT>())) region_queue_kernel(RegionArgs a, const SpanConst* __restrict__ spans,
                                                                                         const int* __restrict__ runs,
                                                                                         const int* __restrict__ livep)
{
    __shared__ VecOf<R> g_vec[NAD * (Prec<R>::KP / Prec<R>::VW)];
    __shared__ double red[THREADS / 64];
    __shared__ int pos_s;
    // a block can take at most n_units positions, so the loop is bounded even
    // if the counter were not reset
    for (int iter = 0; iter <= a.n_units; ++iter) {
        if (threadIdx.x == 0) pos_s = atomicAdd(a.counter, 1);
        __syncthreads();
        const int pos = pos_s;
        __syncthreads();
        if (pos < 0 || pos >= a.n_units) break;
        region_unit<R, MU, PPT>(a, a.order[a.unit0 + pos], blockIdx.x, g_vec, red, spans, runs, livep);
    }
}

// Resets a queue head with an atomic, so the reset is made where the queue's
// atomics are performed.
__global__ void zero_counter_kernel(int* c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicExch(c, 0);
}

// Per CUT: sigma^2 = sum_f w_f sum_islands P1 P2 P3 [c_D R^3 D + Phi c_E R^2 E + ...],
// summed in a fixed order (Eq. 15), eta = sigma^2 / P^3 (Eq. 11).
__global__ void __launch_bounds__(THREADS) assemble_kernel(AssembleArgs a)
{
    __shared__ double red[THREADS / 64];
    const int q = blockIdx.x, tid = threadIdx.x;
    const double cD = 16.0 / 27.0, cE = 16.0 / 27.0, cF = 32.0 / 81.0, cG = 16.0 / 81.0, cH = 16.0 / 81.0;
    const LinkDesc lk = a.links[a.insts[q * a.n_f].link];
    const double R = lk.rs, R2 = R * R, R3 = R2 * R;
    const double h2 = lk.h * lk.h;
    const double* power = a.power + lk.ch0;
    const double* phi = a.phi + lk.ch0;
    const double* psi = a.psi + lk.ch0;
    double s2 = 0.0, tot[5] = {0, 0, 0, 0, 0};
    int cut = 0;
    for (int n = 0; n < a.n_f; ++n) {
        const InstDesc in = a.insts[q * a.n_f + n];
        cut = in.cut;
        double t[5] = {0, 0, 0, 0, 0};
        for (int sq = in.sq_begin + tid; sq < in.sq_end; sq += THREADS) {
            const SquareItem it = a.items[sq];
            const double* pd = a.partD + (size_t)sq * a.n_groups * 3;
            const double* pe = it.d_index >= 0 ? a.partE + (size_t)it.d_index * 12 : nullptr;
            const bool folded = it.k1 != it.k2;
            for (int l = 0; l < 3; ++l) {
                if (!((it.lmask >> l) & 1)) continue;
                const int k3 = it.k1 + it.k2 - in.cut + (l - 1);
                const double P = power[it.k1] * power[it.k2] * power[k3];
                double D = 0.0;
                for (int g = 0; g < a.n_groups; ++g) D += pd[g * 3 + l];
                t[0] += P * it.mult * cD * R3 * h2 * D;
                if (!pe) continue;
                const double* e = pe + l * 4;
                if (folded) {
                    // the mirror square (k2, k1) has F = this square's E when k3 == k1
                    // and E = this square's F when k3 == k2 (f1 <-> f2 symmetry)
                    if (k3 == it.k1) {
                        t[1] += P * phi[it.k1] * cE * R2 * e[0];
                        t[2] += P * phi[it.k1] * cF * R2 * e[0];
                    }
                    if (k3 == it.k2) {
                        t[2] += P * phi[it.k2] * cF * R2 * e[1];
                        t[1] += P * phi[it.k2] * cE * R2 * e[1];
                    }
                } else {
                    if (k3 == it.k1) t[1] += P * phi[it.k1] * cE * R2 * e[0];
                    if (k3 == it.k2) t[2] += P * phi[it.k2] * cF * R2 * e[1];
                    t[3] += P * phi[it.k1] * cG * R2 * e[2];
                    if (k3 == it.k2) t[4] += P * psi[it.k1] * cH * R * e[3];
                }
            }
        }
        double G = 0.0;
        double tb[5];
        for (int u = 0; u < 5; ++u) {
            tb[u] = block_sum(t[u], red);
            G += tb[u];
        }
        const double wf = a.n_f == 1 ? R : R / a.n_f;
        if (tid == 0 && a.psd) a.psd[(size_t)q * a.n_f + n] = G;
        s2 += wf * G;
        for (int u = 0; u < 5; ++u) tot[u] += wf * tb[u];
    }
    if (tid == 0) {
        const double P = power[cut];
        a.eta[q] = s2 / (P * P * P);
        if (a.sigma2) a.sigma2[q] = s2;
        if (a.terms)
            for (int u = 0; u < 5; ++u) a.terms[(size_t)q * 5 + u] = tot[u];
    }
}

}  // namespace

template <typename R, int MU, int PPT = (sizeof(R) == 4 ? PPT32 : PPT64)>
hipError_t launch_region_t(const RegionArgs& a, int blocks, hipStream_t st)
{
    if (blocks > 0)
        hipLaunchKernelGGL((region_queue_kernel<R, MU, PPT>), dim3(blocks), dim3(THREADS), 0, st, a, a.spans, a.runs,
                           a.livep);
    else
        hipLaunchKernelGGL((region_kernel<R, MU, PPT>), dim3(a.n_units), dim3(THREADS), 0, st, a, a.spans, a.runs,
                           a.livep);
    return hipGetLastError();
}

bool region_ppt_supported(bool fp32, int mu_method, int ppt)
{
    if (ppt == ppt_of(fp32)) return true;
    return fp32 && mu_method == MU_SEG && (ppt == 2 || ppt == 8);
}

hipError_t launch_region(const RegionArgs& a, int blocks, bool fp32, int ppt, hipStream_t st)
{
    if (a.n_units == 0) return hipSuccess;
    if (!region_ppt_supported(fp32, a.mu_method, ppt)) return hipErrorInvalidValue;
    if (a.mu_method == MU_SUR) {
        if (!fp32 || !a.sur_tab) return hipErrorInvalidValue;   // the table path runs the FP32 integrand
        return launch_region_t<float, MU_SUR>(a, blocks, st);
    }
    if (a.mu_method == MU_INT)
        return fp32 ? launch_region_t<float, MU_INT>(a, blocks, st) : launch_region_t<double, MU_INT>(a, blocks, st);
    if (fp32) {
        if (a.mu_method == MU_MAC) return launch_region_t<float, MU_MAC>(a, blocks, st);
        if (ppt == 2) return launch_region_t<float, MU_SEG, 2>(a, blocks, st);
        if (ppt == 8) return launch_region_t<float, MU_SEG, 8>(a, blocks, st);
        return launch_region_t<float, MU_SEG>(a, blocks, st);
    }
    return a.mu_method == MU_SEG ? launch_region_t<double, MU_SEG>(a, blocks, st)
                                 : launch_region_t<double, MU_MAC>(a, blocks, st);
}

hipError_t launch_zero_counter(int* counter, hipStream_t st)
{
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, st, counter);
    return hipGetLastError();
}

// Resident blocks per CU of the queue kernel (occupancy query).
template <typename R, int MU, int PPT = (sizeof(R) == 4 ? PPT32 : PPT64)>
int queue_occupancy()
{
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, region_queue_kernel<R, MU, PPT>, THREADS, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

int region_blocks_per_cu(bool fp32, int mu_method, int ppt)
{
    if (mu_method == MU_SUR) return queue_occupancy<float, MU_SUR>();
    if (mu_method == MU_INT) return fp32 ? queue_occupancy<float, MU_INT>() : queue_occupancy<double, MU_INT>();
    if (fp32) {
        if (mu_method == MU_MAC) return queue_occupancy<float, MU_MAC>();
        if (ppt == 2) return queue_occupancy<float, MU_SEG, 2>();
        if (ppt == 8) return queue_occupancy<float, MU_SEG, 8>();
        return queue_occupancy<float, MU_SEG>();
    }
    return mu_method == MU_SEG ? queue_occupancy<double, MU_SEG>() : queue_occupancy<double, MU_MAC>();
}

hipError_t launch_assemble(const AssembleArgs& a, hipStream_t st)
{
    if (a.n_cut == 0) return hipSuccess;
    hipLaunchKernelGGL(assemble_kernel, dim3(a.n_cut), dim3(THREADS), 0, st, a);
    return hipGetLastError();
}

}  // namespace isrs
