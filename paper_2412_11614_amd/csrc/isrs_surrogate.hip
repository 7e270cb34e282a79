// isrs_surrogate.hip -- learned surrogate of the per-span FWM efficiency on gfx950.
//
// An ensemble of MLPs (16 -> 256 -> 256 -> 256 -> 256 -> 1, SiLU) predicts
// r = ln(|mu_s|^2 / L_eff^2) - ln(|eta_s|^2 / L_eff^2): the ISRS correction of
// the segment closed form (Eqs. 7-10) over the closed form without ISRS
// (Eq. 6).  Training data come from the closed form itself (the paper frames
// the accelerated model as a faster data generator for learning, Sec. IV).
//
// Dense layers run on MFMA: v_mfma_f32_32x32x16_bf16 (BF16 operands, FP32
// accumulation), 64 x 64 output tiles per 256-thread block, 32 x 32 per wave.
// Weights live in FP32 (Adam master copy) with BF16 copies in both layouts
// (W for the backward input gradient, W^T for the forward pass), so every
// MFMA operand of those two products is a contiguous 16-byte load.
// Reductions (losses, bias and weight gradients) use fixed orders, so a run
// is reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/isrs_egn.h"
#include "isrs_internal.h"

using namespace isrs;

namespace {

constexpr int NIN = ISRS_SUR_FEATURES;   // padded input width
constexpr int NH = ISRS_SUR_HIDDEN;
constexpr int NF = 9;                    // physical features
constexpr long OFF_W1 = 0;
constexpr long OFF_B1 = OFF_W1 + (long)NIN * NH;
constexpr long OFF_W2 = OFF_B1 + NH;
constexpr long OFF_B2 = OFF_W2 + (long)NH * NH;
constexpr long OFF_W3 = OFF_B2 + NH;
constexpr long OFF_B3 = OFF_W3 + (long)NH * NH;
constexpr long OFF_W4 = OFF_B3 + NH;
constexpr long OFF_B4 = OFF_W4 + (long)NH * NH;
constexpr long OFF_W5 = OFF_B4 + NH;
constexpr long OFF_B5 = OFF_W5 + NH;
constexpr long NP = OFF_B5 + 1;          // 201,985
constexpr long W_OFF[4] = {OFF_W1, OFF_W2, OFF_W3, OFF_W4};
constexpr long B_OFF[4] = {OFF_B1, OFF_B2, OFF_B3, OFF_B4};
constexpr int MAX_MEMBERS = 16;
constexpr int KSPLIT_ROWS = 512;         // batch rows per split of a weight-gradient product

typedef __attribute__((ext_vector_type(8))) __bf16 bf8;
typedef __attribute__((ext_vector_type(4))) __bf16 bf4;
typedef __attribute__((ext_vector_type(16))) float f16v;

// Feature box (physical units), scaled linearly to [-1, 1]; B_tot of Eq. 25.
#define BOX_LO {-5.0, -5.0, -5.0, 80.0, 0.18, -23.0, 0.10, 0.020, 17.0}
#define BOX_HI {5.0, 5.0, 5.0, 100.0, 0.22, -20.0, 0.16, 0.035, 23.0}
__constant__ double c_lo[NF] = BOX_LO;
__constant__ double c_hi[NF] = BOX_HI;
constexpr double h_lo[NF] = BOX_LO;
constexpr double h_hi[NF] = BOX_HI;
constexpr double BOX_BTOT = 10.0;

// ---------------------------------------------------------------------------
// Counter-based generator (SplitMix64 finaliser, S. Vigna): u = mix(key, i).
// ---------------------------------------------------------------------------
__host__ __device__ inline uint64_t mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__host__ __device__ inline double u01(uint64_t key, uint64_t ctr)
{
    return (double)(mix64(key ^ mix64(ctr)) >> 11) * (1.0 / 9007199254740992.0);
}

// ---------------------------------------------------------------------------
// Closed form of one query point in FP64 (Eqs. 5-10 with the ISRS profile of
// Eq. 25, B_tot = 10 THz, dz = 1 km), and Eq. 6.
// ---------------------------------------------------------------------------
struct Phys {
    double a, b, c, L, adb, b2, b3, cr, pdbm;
};

__device__ inline Phys decode(const float* x)
{
    double v[NF];
    for (int j = 0; j < NF; ++j) v[j] = c_lo[j] + 0.5 * ((double)x[j] + 1.0) * (c_hi[j] - c_lo[j]);
    return {v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8]};
}

__device__ inline double alpha_of(const Phys& p) { return p.adb * (M_LN10 / 10.0); }

// chi of Eq. 24 at (f1, f2, f) in 1/km
__device__ inline double chi_of(const Phys& p)
{
    return 4.0 * M_PI * M_PI * ((p.a - p.c) * (p.b - p.c)) * (p.b2 + M_PI * p.b3 * (p.a + p.b));
}

// ln(|eta|^2 / L_eff^2) with eta = (e^{(i chi - alpha) L} - 1) / (i chi - alpha), Eq. 6
__device__ void eq6(const Phys& p, double* y6)
{
    const double alpha = alpha_of(p), chi = chi_of(p);
    double sl, cl;
    sincos(chi * p.L, &sl, &cl);
    const double eL = exp(-alpha * p.L), den = alpha * alpha + chi * chi;
    const double wr = eL * cl - 1.0, wi = eL * sl;
    const double er = (-alpha * wr + chi * wi) / den, ei = (-chi * wr - alpha * wi) / den;
    const double leff = -expm1(-alpha * p.L) / alpha;
    *y6 = log((er * er + ei * ei) / (leff * leff));
}

// ln(|mu|^2 / L_eff^2) of the segment closed form, Eqs. 7-10, dz = 1 km:
// mu = I_0 sum_k g_k q^k, q = e^{(i chi - alpha) Delta}, I_0 = (q - 1)/(i chi - alpha),
// summed by the Goertzel recurrence b_k = g_k + 2 Re(q) b_{k+1} - |q|^2 b_{k+2},
// sum = b_0 - conj(q) b_1.
__device__ void closed_form(const Phys& p, double* y, double* y6)
{
    const double B = 10.0;
    const double ptot = 1e-3 * pow(10.0, p.pdbm / 10.0);
    const double alpha = alpha_of(p), chi = chi_of(p);
    const double x3 = p.a + p.b - p.c;
    const int K = (int)ceil(p.L / 1.0);
    const double dl = p.L / K;
    const double em = exp(-alpha * dl);
    double sq, cq;
    sincos(chi * dl, &sq, &cq);
    const double qr = em * cq, qi = em * sq;
    const double t = 2.0 * qr, s = em * em;
    double b1 = 0.0, b2 = 0.0;
    for (int k = K - 1; k >= 0; --k) {
        const double z = (k + 0.5) / K * p.L;
        const double X = B * ptot * p.cr * (-expm1(-alpha * z) / alpha);
        const double A = X == 0.0 ? 1.0 : X / (2.0 * sinh(0.5 * X));
        const double g = A * exp(-X / B * x3);   // SRS gain at z_k (Eq. 8 with Eq. 25)
        const double b0 = g + t * b1 - s * b2;
        b2 = b1;
        b1 = b0;
    }
    // after the loop b1 = b_0, b2 = b_1
    const double pr = b1 - qr * b2, pim = qi * b2;
    const double den = alpha * alpha + chi * chi;
    const double vr = qr - 1.0, vi = qi;
    const double i0r = (-alpha * vr + chi * vi) / den, i0i = (-chi * vr - alpha * vi) / den;
    const double mr = i0r * pr - i0i * pim, mi = i0r * pim + i0i * pr;
    const double leff = -expm1(-alpha * p.L) / alpha;
    *y = log((mr * mr + mi * mi) / (leff * leff));
    eq6(p, y6);
}

// Random query point of the sampling box: a channel-pair square of a
// 100-channel, 100 GHz grid (W = 99.84 GHz occupied per channel) whose
// product frequency falls inside a channel, a uniform point of the square,
// and f uniform over the CUT's band.
__device__ void draw(uint64_t key, int64_t i, float* x)
{
    const uint64_t c0 = (uint64_t)i * 256;
    double ph[NF];
    for (int j = 3; j < NF; ++j) ph[j] = c_lo[j] + u01(key, c0 + j) * (c_hi[j] - c_lo[j]);
    const double df = 0.1, W = 0.09984;
    double a = 0, b = 0, c = 0;
    for (int tr = 0; tr < 32; ++tr) {
        const uint64_t c1 = c0 + 16 + 6 * tr;
        const int kc = min(99, (int)(u01(key, c1) * 100.0));
        const int k1 = min(99, (int)(u01(key, c1 + 1) * 100.0));
        const int k2 = min(99, (int)(u01(key, c1 + 2) * 100.0));
        const double x0 = (u01(key, c1 + 3) - 0.5) * W, x1 = (u01(key, c1 + 4) - 0.5) * W;
        const double x2 = (u01(key, c1 + 5) - 0.5) * W;
        a = (k1 - 49.5) * df + x1;
        b = (k2 - 49.5) * df + x2;
        c = (kc - 49.5) * df + x0;
        // f1 + f2 - f = nu_{k1+k2-kc} + x3; the island l holds it when |x3 - l df| <= W/2
        const double x3 = x1 + x2 - x0;
        const int l = (int)rint(x3 / df), k3 = k1 + k2 - kc + l;
        if (k3 >= 0 && k3 < 100 && fabs(x3 - l * df) <= 0.5 * W) break;
    }
    ph[0] = a;
    ph[1] = b;
    ph[2] = c;
    for (int j = 0; j < NF; ++j) x[j] = (float)(2.0 * (ph[j] - c_lo[j]) / (c_hi[j] - c_lo[j]) - 1.0);
    for (int j = NF; j < NIN; ++j) x[j] = 0.0f;
}

__global__ void datagen_kernel(int64_t n, uint64_t key, float* x, float* r, float* y6o)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float xs[NIN];
    draw(key, i, xs);
    for (int j = 0; j < NIN; ++j) x[i * NIN + j] = xs[j];
    double y, y6;
    closed_form(decode(xs), &y, &y6);
    r[i] = (float)(y - y6);
    if (y6o) y6o[i] = (float)y6;
}

// Labels of given query points: r = y - y6 and y6 (closed form, FP64).
__global__ void label_kernel(int64_t n, const float* x, float* r, float* y6o)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double y, y6;
    closed_form(decode(x + i * NIN), &y, &y6);
    r[i] = (float)(y - y6);
    if (y6o) y6o[i] = (float)y6;
}

__global__ void closed_form_kernel(int64_t n, const float* x, float* y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double yy, y6;
    closed_form(decode(x + i * NIN), &yy, &y6);
    y[i] = (float)yy;
}

// ---------------------------------------------------------------------------
// MFMA GEMM: C(m, n) = sum_k A(m, k) B(k, n), A(m, k) = A[m*sam + k*sak],
// B(k, n) = B[k*sbk + n*sbn], K a multiple of 16; blockIdx.z splits K in
// chunks of kchunk rows (partial products written to C + z*cz).
// ---------------------------------------------------------------------------
enum { EPI_BIAS_SILU = 0, EPI_PARTIAL = 1, EPI_DSILU = 2, EPI_BIAS_SILU_H = 3 };

struct GemmArgs {
    const __bf16* A;
    long sam, sak;
    const __bf16* B;
    long sbk, sbn;
    int M, N, K, kchunk;
    float* C;        // fp32 output (Z, partial dW, dZ)
    long ldc, cz;
    __bf16* Ch;      // bf16 output (H = silu(Z), dZ)
    const float* bias;
    const float* Zin;  // EPI_DSILU: pre-activation at (m, n), ldc layout
};

// logistic function with the hardware base-2 exponential and reciprocal (1 ulp
// each; activations are stored in BF16): 1 / (1 + 2^(-z log2 e)), exact limits
// 0 and 1 for large |z|
__device__ __forceinline__ float sigm(float z)
{
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-z * 1.44269504088896341f));
}

template <int EPI>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m0 = blockIdx.y * 64 + (w >> 1) * 32, n0 = blockIdx.x * 64 + (w & 1) * 32;
    const int kbeg = blockIdx.z * g.kchunk, kend = min(g.K, kbeg + g.kchunk);
    const int ra = m0 + (lane & 31), cb = n0 + (lane & 31), kl = 8 * (lane >> 5);
    f16v acc = {};
    for (int k = kbeg; k < kend; k += 16) {
        bf8 av, bv;
        const int kk = k + kl;
        if (ra < g.M) {
            if (g.sak == 1) {
                av = *reinterpret_cast<const bf8*>(g.A + (long)ra * g.sam + kk);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) av[e] = g.A[(long)ra * g.sam + (long)(kk + e) * g.sak];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) av[e] = (__bf16)0.0f;
        }
        if (cb < g.N) {
            if (g.sbk == 1) {
                bv = *reinterpret_cast<const bf8*>(g.B + (long)cb * g.sbn + kk);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) bv[e] = g.B[(long)(kk + e) * g.sbk + (long)cb * g.sbn];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) bv[e] = (__bf16)0.0f;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
    // C layout of the 32 x 32 product: register r of lane l is
    // row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), col = n0 + (lane & 31);
        if (row >= g.M || col >= g.N) continue;
        const long o = (long)row * g.ldc + col;
        const float v = acc[r];
        if constexpr (EPI == EPI_BIAS_SILU || EPI == EPI_BIAS_SILU_H) {
            const float z = v + g.bias[col];
            if constexpr (EPI == EPI_BIAS_SILU) g.C[o] = z;
            g.Ch[o] = (__bf16)(z * sigm(z));
        } else if constexpr (EPI == EPI_PARTIAL) {
            g.C[(long)blockIdx.z * g.cz + o] = v;
        } else {
            const float z = g.Zin[o], sz = sigm(z);
            const float d = v * sz * (1.0f + z * (1.0f - sz));
            g.C[o] = d;
            g.Ch[o] = (__bf16)d;
        }
    }
}

// Network input of a query point: the 9 scaled features and 7 derived ones
// (FP64, then BF16): cos and sin of chi L and of chi Delta (the phases whose
// ripple the closed form carries), ln(1 + |chi| / alpha) / 8 - 1, and
// alpha / |beta|, chi / |beta| with beta = i chi - alpha.
__device__ void features_row(const float* xi, float* f)
{
    const Phys p = decode(xi);
    const double alpha = alpha_of(p), chi = chi_of(p);
    const int K = (int)ceil(p.L / 1.0);
    double sl, cl, sd, cd;
    sincos(chi * p.L, &sl, &cl);
    sincos(chi * (p.L / K), &sd, &cd);
    const double m = sqrt(alpha * alpha + chi * chi);
#pragma unroll
    for (int j = 0; j < NF; ++j) f[j] = xi[j];
    f[9] = (float)cl;
    f[10] = (float)sl;
    f[11] = (float)(log1p(fabs(chi) / alpha) / 8.0 - 1.0);
    f[12] = (float)(alpha / m);
    f[13] = (float)(chi / m);
    f[14] = (float)cd;
    f[15] = (float)sd;
}

__global__ void features_kernel(int rows, const float* x, __bf16* xb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    float f[NIN];
    features_row(x + (long)i * NIN, f);
#pragma unroll
    for (int j = 0; j < NIN; ++j) xb[(long)i * NIN + j] = (__bf16)f[j];
}

// Fused inference: a block takes FB_RT * 32 query points through every
// member's four hidden layers and output layer.  The activations of the tile
// stay in LDS (BF16, rows padded to LDH so the 16-byte row reads of an MFMA
// operand fall in distinct banks); weights stream from L2 as W^T rows.  Wave w
// owns output columns 64 w .. 64 w + 63 of every layer: FB_RT x 2 tiles of
// 32 x 32.  Two blocks share a CU.  (8 row tiles, 256 points per block,
// halves the weight reads per point but leaves one wave per SIMD, its 256
// accumulators in the accumulation registers: 15% slower, the operand loads
// then wait with no other wave to switch to.)
constexpr int FB_RT = 4;
constexpr int FB_M = 32 * FB_RT;
constexpr int FB_MINB = FB_RT > 4 ? 1 : 2;   // resident blocks per CU the registers are budgeted for
constexpr int LDH = NH + 8;
constexpr int LDX = NIN + 8;

// acc[ft][rt]: output features 64 w + 32 ft .. + 31 (rows of the MFMA tile)
// for data rows 32 rt .. + 31 (its columns), i.e. (x W)^T = W^T x^T over K (a
// compile-time count, fully unrolled).  A operand: W^T rows (16 bytes along k,
// from L2); B operand: activation rows of the tile (16 bytes along k, LDS).
template <int K, int LD>
__device__ __forceinline__ void fused_products(const __bf16* src, const __bf16* Wt, int w, int lr, int kh,
                                               f16v (&acc)[2][FB_RT])
{
#pragma unroll
    for (int ft = 0; ft < 2; ++ft)
#pragma unroll
        for (int rt = 0; rt < FB_RT; ++rt) acc[ft][rt] = f16v{};
#pragma unroll
    for (int ks = 0; ks < K / 16; ++ks) {
        const int kk = 16 * ks + kh;
        bf8 av[2];
#pragma unroll
        for (int ft = 0; ft < 2; ++ft) av[ft] = *reinterpret_cast<const bf8*>(Wt + (size_t)(64 * w + 32 * ft + lr) * K + kk);
#pragma unroll
        for (int rt = 0; rt < FB_RT; ++rt) {
            const bf8 bv = *reinterpret_cast<const bf8*>(src + (32 * rt + lr) * LD + kk);
#pragma unroll
            for (int ft = 0; ft < 2; ++ft)
                acc[ft][rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[ft], bv, acc[ft][rt], 0, 0, 0);
        }
    }
}

struct FusedArgs {
    const float* x;
    int64_t n;
    int members;
    float shift, scale;
    float* pred;                        // [members][n]
    const __bf16* wt[MAX_MEMBERS][4];   // W_l^T, [256][k_in]
    const float* p[MAX_MEMBERS];        // FP32 parameters (biases, w5, b5)
};

__global__ void __launch_bounds__(256, FB_MINB) mlp_fused_kernel(FusedArgs a)
{
    __shared__ __attribute__((aligned(16))) __bf16 Hs[FB_M * LDH];
    __shared__ __attribute__((aligned(16))) __bf16 Xs[FB_M * LDX];
    __shared__ float Os[4][FB_M];   // output-layer partial sums, one row per wave
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * FB_M;
    for (int rr = tid; rr < FB_M; rr += 256) {
        float f[NIN];
        if (row0 + rr < a.n) {
            features_row(a.x + (row0 + rr) * NIN, f);
        } else {
#pragma unroll
            for (int j = 0; j < NIN; ++j) f[j] = 0.0f;
        }
#pragma unroll
        for (int j = 0; j < NIN; ++j) Xs[rr * LDX + j] = (__bf16)f[j];
    }
    __syncthreads();
    const int lr = lane & 31, kh = 8 * (lane >> 5);
    for (int m = 0; m < a.members; ++m) {
        const float* pm = a.p[m];
        for (int l = 0; l < 4; ++l) {
            const __bf16* src = l == 0 ? Xs : Hs;
            const __bf16* Wt = a.wt[m][l];
            f16v acc[2][FB_RT];
            if (l == 0)
                fused_products<NIN, LDX>(src, Wt, w, lr, kh, acc);
            else
                fused_products<NH, LDH>(src, Wt, w, lr, kh, acc);
            __syncthreads();  // every wave has read the layer's input
            // register 4 g + e of tile (ft, rt) holds feature 64 w + 32 ft + 8 g + 4 (lane / 32) + e
            // of data row 32 rt + lane % 32: four consecutive features, one 8-byte write
            const float* bias = pm + B_OFF[l];
            if (l < 3) {
#pragma unroll
                for (int ft = 0; ft < 2; ++ft)
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const int f0 = 64 * w + 32 * ft + 8 * g + 4 * (lane >> 5);
                        const float4 bq = *reinterpret_cast<const float4*>(bias + f0);
                        const float bb[4] = {bq.x, bq.y, bq.z, bq.w};
#pragma unroll
                        for (int rt = 0; rt < FB_RT; ++rt) {
                            bf4 hv;
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const float z = acc[ft][rt][4 * g + e] + bb[e];
                                hv[e] = (__bf16)(z * sigm(z));
                            }
                            *reinterpret_cast<bf4*>(Hs + (32 * rt + lr) * LDH + f0) = hv;
                        }
                    }
                __syncthreads();
                continue;
            }
            // last hidden layer: the output layer o = H4 w5 + b5 straight from the
            // accumulators, each activation rounded to BF16 as a stored H4 would be.
            // A lane sums its 32 features of each row; the two half-waves hold the
            // other 32 of the wave's 64, the four waves the rest.
            const float* w5 = pm + OFF_W5;
            float part[FB_RT];
#pragma unroll
            for (int rt = 0; rt < FB_RT; ++rt) part[rt] = 0.0f;
#pragma unroll
            for (int ft = 0; ft < 2; ++ft)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int f0 = 64 * w + 32 * ft + 8 * g + 4 * (lane >> 5);
                    const float4 bq = *reinterpret_cast<const float4*>(bias + f0);
                    const float4 wq = *reinterpret_cast<const float4*>(w5 + f0);
                    const float bb[4] = {bq.x, bq.y, bq.z, bq.w}, ww[4] = {wq.x, wq.y, wq.z, wq.w};
#pragma unroll
                    for (int rt = 0; rt < FB_RT; ++rt)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const float z = acc[ft][rt][4 * g + e] + bb[e];
                            part[rt] = fmaf((float)(__bf16)(z * sigm(z)), ww[e], part[rt]);
                        }
                }
#pragma unroll
            for (int rt = 0; rt < FB_RT; ++rt) part[rt] += __shfl_xor(part[rt], 32, 64);
            if (lane < 32)
#pragma unroll
                for (int rt = 0; rt < FB_RT; ++rt) Os[w][32 * rt + lane] = part[rt];
            __syncthreads();
            for (int rr = tid; rr < FB_M; rr += 256) {
                const float o = ((Os[0][rr] + Os[1][rr]) + (Os[2][rr] + Os[3][rr])) + pm[OFF_B5];
                if (row0 + rr < a.n) a.pred[(int64_t)m * a.n + row0 + rr] = a.shift + a.scale * o;
            }
            // the next writes to Os and Hs come after this member's last barrier
        }
    }
}

// Output layer o = shift + scale (H4 w5 + b5), one wave per row.
__global__ void out_layer_kernel(int rows, const __bf16* H, const float* w5, const float* b5, float shift,
                                 float scale, float* o)
{
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= rows) return;
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < NH / 64; ++j) s += (float)H[(long)row * NH + lane + 64 * j] * w5[lane + 64 * j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) o[row] = shift + scale * (s + b5[0]);
}

// Normalised target t = (r - shift) / scale; d_out = 2 (o - t) / rows;
// dZ4 = d_out w5 silu'(Z4); per-block squared-error sums.
__global__ void out_backward_kernel(int rows, const float* o, const float* r, float shift, float inv_scale,
                                    const float* w5, const float* Z4, float* dout, float* dZ, __bf16* dZh,
                                    float* loss_part)
{
    __shared__ float red[4];
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    float e2 = 0.0f;
    if (row < rows) {
        const float e = o[row] - (r[row] - shift) * inv_scale;
        const float d = 2.0f * e / rows;
        if (lane == 0) dout[row] = d;
        e2 = e * e;
#pragma unroll
        for (int j = 0; j < NH / 64; ++j) {
            const long q = (long)row * NH + lane + 64 * j;
            const float z = Z4[q], sz = sigm(z);
            const float v = d * w5[lane + 64 * j] * sz * (1.0f + z * (1.0f - sz));
            dZ[q] = v;
            dZh[q] = (__bf16)v;
        }
    }
    if (lane == 0) red[threadIdx.x >> 6] = e2;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Column sums of an fp32 [rows x cols] matrix in a fixed order: out[c] =
// sum_r X[r, c]; with H given, the output-layer gradient out[c] = sum_r
// H[r, c] d[r].  A block takes CS_COLS columns; each of its CS_GROUPS row
// groups sums a contiguous run of rows, then the group sums are added in order.
constexpr int CS_COLS = 16, CS_GROUPS = 16;
__global__ void __launch_bounds__(CS_COLS * CS_GROUPS) colsum_kernel(int rows, int cols, const float* X,
                                                                      const __bf16* H, const float* d, float* out)
{
    __shared__ float part[CS_GROUPS][CS_COLS + 1];
    const int cl = threadIdx.x % CS_COLS, rg = threadIdx.x / CS_COLS;
    const int c = blockIdx.x * CS_COLS + cl;
    const int per = (rows + CS_GROUPS - 1) / CS_GROUPS;
    const int r0 = rg * per, r1 = min(rows, r0 + per);
    float s = 0.0f;
    if (c < cols) {
        if (H) {
            for (int r = r0; r < r1; ++r) s += (float)H[(long)r * cols + c] * d[r];
        } else {
            for (int r = r0; r < r1; ++r) s += X[(long)r * cols + c];
        }
    }
    part[rg][cl] = s;
    __syncthreads();
    if (rg == 0 && c < cols) {
        float t = 0.0f;
        for (int g = 0; g < CS_GROUPS; ++g) t += part[g][cl];
        out[c] = t;
    }
}

// Sum of split-K partials in order.
__global__ void split_sum_kernel(long n, int splits, long stride, const float* part, float* out)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += part[z * stride + i];
    out[i] = s;
}

__global__ void adam_kernel(long n, float* p, const float* gr, float* m, float* v, float lr, float b1, float b2,
                            float eps, float c1, float c2)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mm = b1 * m[i] + (1.0f - b1) * g;
    const float vv = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mm;
    v[i] = vv;
    p[i] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// BF16 copies of a weight matrix W [k x n] (fp32): W itself and W^T.
__global__ void weights_bf16_kernel(int k, int n, const float* W, __bf16* Wb, __bf16* Wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k * n) return;
    const int r = i / n, c = i % n;
    const __bf16 v = (__bf16)W[i];
    Wb[i] = v;
    Wt[(long)c * k + r] = v;
}

// Ensemble statistics and the surrogate output before fallback.
__global__ void ensemble_kernel(int64_t n, int members, const float* pred, const float* x, float* mean, float* spread,
                                float* y, double thr_ln, int* flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f, lo = 3.4e38f, hi = -3.4e38f;
    for (int m = 0; m < members; ++m) {
        const float v = pred[(int64_t)m * n + i];
        s += v;
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
    }
    const float mu = s / members, sp = hi - lo;
    if (mean) mean[i] = mu;
    if (spread) spread[i] = sp;
    if (y) {
        double y6;
        const Phys p = decode(x + i * NIN);
        eq6(p, &y6);
        y[i] = (float)(y6 + (double)mu);
    }
    if (flag) flag[i] = (thr_ln < 0.0 || (double)sp > thr_ln) ? 1 : 0;
}

// Mean (pass 0) or sum of squared deviations from *mean (pass 1) of r[0, n),
// one block, fixed summation order.
__global__ void __launch_bounds__(1024) moments_kernel(int64_t n, const float* r, int pass, double* out)
{
    __shared__ double red[1024];
    const double mu = pass ? out[0] : 0.0;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        const double v = (double)r[i] - mu;
        acc += pass ? v * v : v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[pass] = pass ? red[0] : red[0] / (double)n;
}

// Deterministic compaction of flagged indices: per-block counts, one-block
// exclusive scan, per-block ordered scatter.
constexpr int CB = 1024;

__global__ void count_kernel(int64_t n, const int* flag, int* cnt)
{
    __shared__ int s[CB / 64];
    const int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x;
    const int f = i < n ? flag[i] : 0;
    const unsigned long long bal = __ballot(f);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < CB / 64; ++w) t += s[w];
        cnt[blockIdx.x] = t;
    }
}

// Exclusive scan of the per-block counts in one block of SCAN_T threads: each
// thread takes a contiguous run of counts, the run totals are scanned in LDS,
// then each thread writes its run's offsets (integer sums, so exact).
constexpr int SCAN_T = 1024;
__global__ void __launch_bounds__(SCAN_T) scan_kernel(int nb, const int* cnt, int* off, int* total)
{
    __shared__ int part[SCAN_T];
    const int t = threadIdx.x;
    const int per = (nb + SCAN_T - 1) / SCAN_T;
    const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
    int sum = 0;
    for (int b = b0; b < b1; ++b) sum += cnt[b];
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < SCAN_T; d <<= 1) {     // inclusive scan of the run totals
        const int v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int base = t ? part[t - 1] : 0;
    for (int b = b0; b < b1; ++b) {
        off[b] = base;
        base += cnt[b];
    }
    if (t == SCAN_T - 1) *total = part[SCAN_T - 1];
}

__global__ void scatter_kernel(int64_t n, const int* flag, const int* off, int64_t* idx)
{
    __shared__ int s[CB / 64];
    const int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x;
    const int f = i < n ? flag[i] : 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long bal = __ballot(f);
    if (lane == 0) s[w] = __popcll(bal);
    __syncthreads();
    int base = off[blockIdx.x];
    for (int q = 0; q < w; ++q) base += s[q];
    const int rank = __popcll(bal & ((1ull << lane) - 1ull));
    if (f) idx[base + rank] = i;
}

__global__ void fallback_kernel(const int* total, const int64_t* idx, const float* x, float* y)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= *total) return;
    const int64_t i = idx[t];
    double yy, y6;
    closed_form(decode(x + i * NIN), &yy, &y6);
    y[i] = (float)yy;
}

// Query rows of squares [item0, item0 + rows / (N^2 n_sp)) of a plan, one per
// (grid point, span): row ((item - item0) N + j) N + i) n_sp + s, i the f1
// index and j the f2 index of the square.  state: 0 no live island at the
// point, 1 a query inside the sampling box, 2 outside it (closed form).
__global__ void sur_query_kernel(RegionArgs ra, int item0, int64_t rows, int n_sp, float* x, unsigned char* state)
{
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= rows) return;
    const int N = ra.N, AD = 2 * N - 1;
    const int s = (int)(row % n_sp);
    int64_t t = row / n_sp;
    const int i = (int)(t % N);
    t /= N;
    const int j = (int)(t % N);
    const int item = item0 + (int)(t / N);
    const SquareItem it = ra.items[item];
    const InstDesc in = ra.insts[it.inst];
    const LinkDesc lk = ra.links[in.link];
    const SpanConst sc = ra.spans[lk.span0 + s];
    const double* wt = ra.wt + lk.tab0 + (size_t)in.nf_idx * 3 * AD;
    bool live = false;
    for (int l = 0; l < 3; ++l)
        if (((it.lmask >> l) & 1) && wt[l * AD + i + j] != 0.0) live = true;
    float* xr = x + row * NIN;
    if (!live) {
        state[row] = 0;
        for (int q = 0; q < NIN; ++q) xr[q] = 0.0f;
        return;
    }
    const double hg = 0.5 * (lk.n_ch - 1), df = lk.spacing, h = lk.h;
    double ph[NF];
    ph[0] = (it.k1 - hg) * df + (i + 0.5 - 0.5 * N) * h;
    ph[1] = (it.k2 - hg) * df + (j + 0.5 - 0.5 * N) * h;
    ph[2] = (in.cut - hg) * df + in.f;
    ph[3] = sc.L;
    ph[4] = sc.alpha * (10.0 / M_LN10);
    ph[5] = sc.c2x / (4.0 * M_PI * M_PI);
    ph[6] = sc.c3x / (4.0 * M_PI * M_PI * M_PI);
    ph[7] = sc.cr;
    ph[8] = 10.0 * log10(sc.ptot / 1e-3);
    bool inbox = fabs(sc.btot - 10.0) <= 1e-9;
    for (int q = 0; q < NF; ++q) {
        const double v = 2.0 * (ph[q] - c_lo[q]) / (c_hi[q] - c_lo[q]) - 1.0;
        if (!(fabs(v) <= 1.0 + 1e-9)) inbox = false;
        xr[q] = (float)fmin(1.0, fmax(-1.0, v));
    }
    for (int q = NF; q < NIN; ++q) xr[q] = 0.0f;
    state[row] = inbox ? 1 : 2;
}

// Table rows from the ensemble: 0 where no island is live, NaN (closed form)
// outside the box or where the spread exceeds thr_ln (thr_ln < 0: everywhere),
// else the ensemble mean.  Per-block counts of live and fallback rows.
__global__ void sur_combine_kernel(int64_t rows, int members, const float* pred, const unsigned char* state,
                                   double thr_ln, float* tab, int* cnt_live, int* cnt_fb)
{
    __shared__ int sl[4], sf[4];
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int live = 0, fbk = 0;
    if (row < rows) {
        const unsigned char st = state[row];
        float v = 0.0f;
        if (st != 0) {
            live = 1;
            if (st == 2 || thr_ln < 0.0) {
                fbk = 1;
            } else {
                float sum = 0.0f, lo = 3.4e38f, hi = -3.4e38f;
                for (int m = 0; m < members; ++m) {
                    const float p = pred[(int64_t)m * rows + row];
                    sum += p;
                    lo = fminf(lo, p);
                    hi = fmaxf(hi, p);
                }
                if ((double)(hi - lo) > thr_ln) fbk = 1;
                else v = sum / members;
            }
            if (fbk) v = __builtin_nanf("");
        }
        tab[row] = v;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nl = __popcll(__ballot(live)), nf = __popcll(__ballot(fbk));
    if (lane == 0) {
        sl[w] = nl;
        sf[w] = nf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cnt_live[blockIdx.x] = sl[0] + sl[1] + sl[2] + sl[3];
        cnt_fb[blockIdx.x] = sf[0] + sf[1] + sf[2] + sf[3];
    }
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct isrs_surrogate {
    int n_members = 0;
    uint64_t seed = 0;
    int device = 0;
    struct Member {
        float* p = nullptr;  // fp32 params [NP]
        float* m = nullptr;  // Adam moments
        float* v = nullptr;
        __bf16* wb[4] = {};  // W_l [k x n]
        __bf16* wt[4] = {};  // W_l^T [n x k]
        long step = 0;
    };
    std::vector<Member> mem;
    // the network learns t = (r - shift) / scale; set from the first training set
    double shift = 0.0, scale = 1.0;
    int64_t scaled = 0;
    double* mom = nullptr;            // [2] device
    // scratch for a batch of `cap` rows
    int cap = 0;
    __bf16* xb = nullptr;             // [cap x 16]
    float* Z[4] = {};                 // [cap x 256]
    __bf16* H[4] = {};
    float* dZ = nullptr;              // [cap x 256]
    __bf16* dZh = nullptr;
    float* dZ2 = nullptr;
    __bf16* dZh2 = nullptr;
    float* o = nullptr;               // [cap]
    float* dout = nullptr;
    float* loss_part = nullptr;       // [cap / 4]
    float* grad = nullptr;            // [NP]
    float* part = nullptr;            // split-K partials
    size_t part_cap = 0;
    // prediction scratch
    float* pred = nullptr;            // [members x pcap]
    int64_t pcap = 0;
    int* flag = nullptr;
    int* cnt = nullptr;
    int* off = nullptr;
    int* total = nullptr;
    int64_t* idx = nullptr;
    float* cal = nullptr;             // calibration: mean, spread, reference [3 x ccap]
    int64_t ccap = 0;
    int64_t fcap = 0;
    // query rows of the table path
    float* qx = nullptr;
    unsigned char* qstate = nullptr;
    int* qcnt = nullptr;              // [2][blocks]
    int64_t qcap = 0;
};

namespace {

template <typename T>
hipError_t dalloc(T** p, size_t n)
{
    return hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(1, n) * sizeof(T));
}

void dfree(void* p)
{
    if (p) (void)hipFree(p);
}

// frees and clears, so a failed reallocation never leaves a stale pointer
template <typename T>
void release(T*& p)
{
    dfree(p);
    p = nullptr;
}

#define S_TRY(ctx, expr)                                                                                   \
    do {                                                                                                   \
        hipError_t _e = (expr);                                                                            \
        if (_e != hipSuccess)                                                                              \
            return ctx_fail((ctx), _e == hipErrorOutOfMemory ? ISRS_E_NOMEM : ISRS_E_DEVICE,               \
                            (std::string(#expr) + ": " + hipGetErrorString(_e)).c_str());                  \
    } while (0)

// Seeded initialisation on the host: weights U(-s, s), s = sqrt(6 / fan_in)
// (He-uniform), biases 0.  The first layer's fan-in is the 16 network inputs.
void init_params(std::vector<float>& p, uint64_t seed, int member)
{
    p.assign(NP, 0.0f);
    const uint64_t key = mix64(seed ^ (0x5152535455565758ull + (uint64_t)member));
    uint64_t ctr = 0;
    auto fill = [&](long off, int fan_in, long count) {
        const double s = std::sqrt(6.0 / fan_in);
        for (long i = 0; i < count; ++i) p[off + i] = (float)((2.0 * u01(key, ctr++) - 1.0) * s);
    };
    fill(OFF_W1, NIN, (long)NIN * NH);
    fill(OFF_W2, NH, (long)NH * NH);
    fill(OFF_W3, NH, (long)NH * NH);
    fill(OFF_W4, NH, (long)NH * NH);
    fill(OFF_W5, NH, NH);
}

int32_t refresh_bf16(isrs_ctx* c, isrs_surrogate::Member& m, hipStream_t st)
{
    for (int l = 0; l < 4; ++l) {
        const int k = l == 0 ? NIN : NH;
        hipLaunchKernelGGL(weights_bf16_kernel, dim3(blocks_for((int64_t)k * NH, 256)), dim3(256), 0, st, k, NH,
                           m.p + W_OFF[l], m.wb[l], m.wt[l]);
    }
    S_TRY(c, hipGetLastError());
    return ISRS_OK;
}

int32_t ensure_batch(isrs_ctx* c, isrs_surrogate* s, int rows)
{
    if (rows <= s->cap) return ISRS_OK;
    release(s->xb);
    for (int l = 0; l < 4; ++l) {
        release(s->Z[l]);
        release(s->H[l]);
    }
    release(s->dZ);
    release(s->dZh);
    release(s->dZ2);
    release(s->dZh2);
    release(s->o);
    release(s->dout);
    release(s->loss_part);
    s->cap = 0;
    S_TRY(c, dalloc(&s->xb, (size_t)rows * NIN));
    for (int l = 0; l < 4; ++l) {
        S_TRY(c, dalloc(&s->Z[l], (size_t)rows * NH));
        S_TRY(c, dalloc(&s->H[l], (size_t)rows * NH));
    }
    S_TRY(c, dalloc(&s->dZ, (size_t)rows * NH));
    S_TRY(c, dalloc(&s->dZh, (size_t)rows * NH));
    S_TRY(c, dalloc(&s->dZ2, (size_t)rows * NH));
    S_TRY(c, dalloc(&s->dZh2, (size_t)rows * NH));
    S_TRY(c, dalloc(&s->o, (size_t)rows));
    S_TRY(c, dalloc(&s->dout, (size_t)rows));
    S_TRY(c, dalloc(&s->loss_part, (size_t)rows / 4 + 1));
    s->cap = rows;
    return ISRS_OK;
}

GemmArgs gemm(const __bf16* A, long sam, long sak, const __bf16* B, long sbk, long sbn, int M, int N, int K)
{
    GemmArgs g{};
    g.A = A;
    g.sam = sam;
    g.sak = sak;
    g.B = B;
    g.sbk = sbk;
    g.sbn = sbn;
    g.M = M;
    g.N = N;
    g.K = K;
    g.kchunk = K;
    return g;
}

template <int EPI>
void launch_gemm(const GemmArgs& g, int splits, hipStream_t st)
{
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, splits);
    hipLaunchKernelGGL(gemm_kernel<EPI>, grid, dim3(256), 0, st, g);
}

// Forward pass of rows [x (bf16, rows x 16)] through member m; keeps Z, H.
void forward(isrs_surrogate* s, const isrs_surrogate::Member& m, const __bf16* xb, int rows, bool keep_z, float* out,
             bool denorm, hipStream_t st)
{
    const __bf16* in = xb;
    int kin = NIN;
    for (int l = 0; l < 4; ++l) {
        // Z = in [rows x kin] W_l [kin x 256]; W^T rows are contiguous along k
        GemmArgs g = gemm(in, kin, 1, m.wt[l], 1, kin, rows, NH, kin);
        g.C = s->Z[l];
        g.ldc = NH;
        g.Ch = s->H[l];
        g.bias = m.p + B_OFF[l];
        if (keep_z)
            launch_gemm<EPI_BIAS_SILU>(g, 1, st);
        else
            launch_gemm<EPI_BIAS_SILU_H>(g, 1, st);
        in = s->H[l];
        kin = NH;
    }
    hipLaunchKernelGGL(out_layer_kernel, dim3(blocks_for(rows, 4)), dim3(256), 0, st, rows, s->H[3],
                       m.p + OFF_W5, m.p + OFF_B5, denorm ? (float)s->shift : 0.0f, denorm ? (float)s->scale : 1.0f,
                       out);
}

int32_t ensure_part(isrs_ctx* c, isrs_surrogate* s, size_t n)
{
    if (n <= s->part_cap) return ISRS_OK;
    release(s->part);
    s->part_cap = 0;
    S_TRY(c, dalloc(&s->part, n));
    s->part_cap = n;
    return ISRS_OK;
}

// Gradient of the mean squared residual error of one batch into s->grad;
// per-block squared errors into s->loss_part.
int32_t backward(isrs_ctx* c, isrs_surrogate* s, const isrs_surrogate::Member& m, const float* r, int rows,
                 hipStream_t st)
{
    const int splits = std::max(1, rows / KSPLIT_ROWS);
    int32_t rc = ensure_part(c, s, (size_t)splits * NH * NH);
    if (rc) return rc;
    hipLaunchKernelGGL(out_backward_kernel, dim3(blocks_for(rows, 4)), dim3(256), 0, st, rows, s->o, r,
                       (float)s->shift, (float)(1.0 / s->scale), m.p + OFF_W5, s->Z[3], s->dout, s->dZ, s->dZh, s->loss_part);
    // output layer: dw5 = H4^T dout, db5 = sum dout
    hipLaunchKernelGGL(colsum_kernel, dim3(NH / CS_COLS), dim3(CS_COLS * CS_GROUPS), 0, st, rows, NH, nullptr,
                       s->H[3], s->dout, s->grad + OFF_W5);
    hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(CS_COLS * CS_GROUPS), 0, st, rows, 1, s->dout, nullptr, nullptr,
                       s->grad + OFF_B5);
    float* dz = s->dZ;
    __bf16* dzh = s->dZh;
    float* dz_next = s->dZ2;
    __bf16* dzh_next = s->dZh2;
    for (int l = 3; l >= 0; --l) {
        const int kin = l == 0 ? NIN : NH;
        const __bf16* in = l == 0 ? s->xb : s->H[l - 1];
        // dW_l = in^T dZ_l  (reduction over rows, split in chunks, summed in order)
        GemmArgs g = gemm(in, 1, kin, dzh, NH, 1, kin, NH, rows);
        g.kchunk = (rows + splits - 1) / splits;
        g.kchunk = (g.kchunk + 15) / 16 * 16;
        g.C = s->part;
        g.ldc = NH;
        g.cz = (long)kin * NH;
        const int zs = (rows + g.kchunk - 1) / g.kchunk;
        launch_gemm<EPI_PARTIAL>(g, zs, st);
        hipLaunchKernelGGL(split_sum_kernel, dim3(blocks_for((int64_t)kin * NH, 256)), dim3(256), 0, st,
                           (long)kin * NH, zs, (long)kin * NH, s->part, s->grad + W_OFF[l]);
        // db_l = column sums of dZ_l
        hipLaunchKernelGGL(colsum_kernel, dim3(NH / CS_COLS), dim3(CS_COLS * CS_GROUPS), 0, st, rows, NH, dz,
                           nullptr, nullptr, s->grad + B_OFF[l]);
        if (l == 0) break;
        // dZ_{l-1} = (dZ_l W_l^T) * silu'(Z_{l-1});  W_l rows are contiguous along the output index
        GemmArgs gd = gemm(dzh, NH, 1, m.wb[l], 1, NH, rows, NH, NH);
        gd.C = dz_next;
        gd.ldc = NH;
        gd.Ch = dzh_next;
        gd.Zin = s->Z[l - 1];
        launch_gemm<EPI_DSILU>(gd, 1, st);
        std::swap(dz, dz_next);
        std::swap(dzh, dzh_next);
    }
    S_TRY(c, hipGetLastError());
    return ISRS_OK;
}

int32_t pack_rows(isrs_ctx* c, isrs_surrogate* s, const float* x, int64_t row0, int rows, hipStream_t st)
{
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for(rows, 256)), dim3(256), 0, st, rows, x + row0 * NIN, s->xb);
    S_TRY(c, hipGetLastError());
    return ISRS_OK;
}

int32_t ensure_pred(isrs_ctx* c, isrs_surrogate* s, int64_t n)
{
    if (n <= s->pcap) return ISRS_OK;
    release(s->pred);
    release(s->flag);
    release(s->cnt);
    release(s->off);
    release(s->total);
    release(s->idx);
    s->pcap = 0;
    S_TRY(c, dalloc(&s->pred, (size_t)n * s->n_members));
    S_TRY(c, dalloc(&s->flag, (size_t)n));
    const int64_t nb = (n + CB - 1) / CB;
    S_TRY(c, dalloc(&s->cnt, (size_t)nb));
    S_TRY(c, dalloc(&s->off, (size_t)nb));
    S_TRY(c, dalloc(&s->total, 1));
    S_TRY(c, dalloc(&s->idx, (size_t)n));
    s->pcap = n;
    return ISRS_OK;
}

int32_t predict_members(isrs_ctx* c, isrs_surrogate* s, const float* x, int64_t n, hipStream_t st)
{
    int32_t rc = ensure_pred(c, s, n);
    if (rc) return rc;
    FusedArgs fa{};
    fa.x = x;
    fa.n = n;
    fa.members = s->n_members;
    fa.shift = (float)s->shift;
    fa.scale = (float)s->scale;
    fa.pred = s->pred;
    for (int m = 0; m < s->n_members; ++m) {
        for (int l = 0; l < 4; ++l) fa.wt[m][l] = s->mem[m].wt[l];
        fa.p[m] = s->mem[m].p;
    }
    hipLaunchKernelGGL(mlp_fused_kernel, dim3((unsigned)((n + FB_M - 1) / FB_M)), dim3(256), 0, st, fa);
    S_TRY(c, hipGetLastError());
    return ISRS_OK;
}

}  // namespace

extern "C" {

int32_t isrs_surrogate_num_params(int64_t* n)
{
    try {
        if (!n) return ISRS_E_ARG;
        *n = NP;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(nullptr);
    }
}

int32_t isrs_surrogate_create(isrs_ctx* c, int32_t n_members, uint64_t seed, isrs_surrogate** out)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!out || n_members < 1 || n_members > MAX_MEMBERS) return ctx_fail(c, ISRS_E_ARG, "1..16 members");
        *out = nullptr;
        isrs_surrogate* s = new (std::nothrow) isrs_surrogate();
        if (!s) return ctx_fail(c, ISRS_E_NOMEM, "host allocation failed");
        s->n_members = n_members;
        s->seed = seed;
        s->device = ctx_device(c);
        // every failure below releases what was allocated so far
        auto setup = [&]() -> int32_t {
            S_TRY(c, hipSetDevice(s->device));
            hipStream_t st = ctx_stream(c);
            s->mem.resize(n_members);
            std::vector<float> p;
            for (int mi = 0; mi < n_members; ++mi) {
                auto& m = s->mem[mi];
                S_TRY(c, dalloc(&m.p, NP));
                S_TRY(c, dalloc(&m.m, NP));
                S_TRY(c, dalloc(&m.v, NP));
                for (int l = 0; l < 4; ++l) {
                    const size_t k = l == 0 ? NIN : NH;
                    S_TRY(c, dalloc(&m.wb[l], k * NH));
                    S_TRY(c, dalloc(&m.wt[l], k * NH));
                }
                init_params(p, seed, mi);
                S_TRY(c, hipMemcpy(m.p, p.data(), NP * sizeof(float), hipMemcpyHostToDevice));
                S_TRY(c, hipMemset(m.m, 0, NP * sizeof(float)));
                S_TRY(c, hipMemset(m.v, 0, NP * sizeof(float)));
                int32_t rc = refresh_bf16(c, m, st);
                if (rc) return rc;
            }
            S_TRY(c, dalloc(&s->grad, NP));
            S_TRY(c, dalloc(&s->mom, 2));
            S_TRY(c, hipStreamSynchronize(st));
            return ISRS_OK;
        };
        const int32_t rc = setup();
        if (rc) {
            isrs_surrogate_destroy(s);
            return rc;
        }
        *out = s;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_surrogate_destroy(isrs_surrogate* s)
{
    try {
        if (!s) return ISRS_E_ARG;
        (void)hipSetDevice(s->device);
        (void)hipDeviceSynchronize();
        for (auto& m : s->mem) {
            dfree(m.p);
            dfree(m.m);
            dfree(m.v);
            for (int l = 0; l < 4; ++l) {
                dfree(m.wb[l]);
                dfree(m.wt[l]);
            }
        }
        dfree(s->xb);
        for (int l = 0; l < 4; ++l) {
            dfree(s->Z[l]);
            dfree(s->H[l]);
        }
        dfree(s->dZ);
        dfree(s->dZh);
        dfree(s->dZ2);
        dfree(s->dZh2);
        dfree(s->o);
        dfree(s->dout);
        dfree(s->loss_part);
        dfree(s->grad);
        dfree(s->mom);
        dfree(s->part);
        dfree(s->pred);
        dfree(s->flag);
        dfree(s->cnt);
        dfree(s->off);
        dfree(s->total);
        dfree(s->idx);
        dfree(s->cal);
        dfree(s->qx);
        dfree(s->qstate);
        dfree(s->qcnt);
        delete s;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(nullptr);
    }
}

int32_t isrs_surrogate_datagen(isrs_ctx* c, int64_t n, uint64_t seed, float* x, float* r, float* y6)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (n < 1 || !x || !r) return ctx_fail(c, ISRS_E_ARG, "need n >= 1 and output buffers");
        S_TRY(c, hipSetDevice(ctx_device(c)));
        hipLaunchKernelGGL(datagen_kernel, dim3(blocks_for(n, 128)), dim3(128), 0, ctx_stream(c), n, mix64(seed), x,
                           r, y6);
        S_TRY(c, hipGetLastError());
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_surrogate_datagen_batch(isrs_ctx* c, const isrs_batch* b, int32_t n_grid, int64_t n, uint64_t seed,
                                     float* x, float* r, float* y6, int64_t* n_rejected)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!b || n < 1 || !x || !r || n_grid < 1) return ctx_fail(c, ISRS_E_ARG, "need a batch, n >= 1, n_grid >= 1 and outputs");
        const int nl = batch_num_links(b);
        if (nl < 1) return ctx_fail(c, ISRS_E_ARG, "the batch has no links");
        std::vector<LinkView> links(nl);
        std::vector<std::vector<int>> act(nl);
        std::vector<double> pdbm(nl);
        for (int l = 0; l < nl; ++l) {
            links[l] = batch_link_view(b, l);
            double pt = 0.0;
            for (int k = 0; k < links[l].n_ch; ++k)
                if (links[l].power[k] > 0) {
                    act[l].push_back(k);
                    pt += links[l].power[k];
                }
            pdbm[l] = 10.0 * std::log10(pt / 1e-3);
        }
        const uint64_t key = mix64(seed ^ 0x6c696e6b73ull);
        uint64_t ctr = 0;
        auto u = [&]() { return u01(key, ctr++); };
        auto pick = [&](int m) { return std::min(m - 1, (int)(u() * m)); };
        std::vector<float> hx((size_t)n * NIN, 0.0f);
        int64_t rejected = 0;
        for (int64_t q = 0; q < n; ++q) {
            bool done = false;
            for (int tr = 0; tr < 4096 && !done; ++tr) {
                const int l = pick(nl);
                const LinkView& L = links[l];
                if (L.n_cut < 1 || act[l].empty()) continue;
                const int cut = L.cuts[pick(L.n_cut)];
                const int k1 = act[l][pick((int)act[l].size())], k2 = act[l][pick((int)act[l].size())];
                const int i = pick(n_grid), j = pick(n_grid), s_ = pick(L.n_sp);
                const double W = (1.0 + L.rolloff) * L.rs, h = W / n_grid, df = L.spacing;
                const double f1 = (i + 0.5 - 0.5 * n_grid) * h, f2 = (j + 0.5 - 0.5 * n_grid) * h;
                bool island = false;
                for (int li = -1; li <= 1; ++li) {
                    const int k3 = k1 + k2 - cut + li;
                    if (k3 >= 0 && k3 < L.n_ch && L.power[k3] > 0 && std::fabs(f1 + f2 - li * df) <= 0.5 * W) island = true;
                }
                if (!island) continue;
                const double hg = 0.5 * (L.n_ch - 1);
                const isrs_span& sp = L.spans[s_];
                const double ph[NF] = {(k1 - hg) * df + f1, (k2 - hg) * df + f2, (cut - hg) * df, sp.length_km,
                                       sp.alpha_db_km, sp.beta2_ps2_km, sp.beta3_ps3_km, sp.cr_w_km_thz, pdbm[l]};
                bool inbox = std::fabs(L.n_ch * df - BOX_BTOT) <= 1e-9;
                float* xr = hx.data() + (size_t)q * NIN;
                for (int f = 0; f < NF; ++f) {
                    const double v = 2.0 * (ph[f] - h_lo[f]) / (h_hi[f] - h_lo[f]) - 1.0;
                    if (!(std::fabs(v) <= 1.0)) inbox = false;
                    xr[f] = (float)v;
                }
                if (!inbox) {
                    ++rejected;
                    continue;
                }
                done = true;
            }
            if (!done) return ctx_fail(c, ISRS_E_ARG, "the batch has no query points inside the sampling box");
        }
        S_TRY(c, hipSetDevice(ctx_device(c)));
        hipStream_t st = ctx_stream(c);
        S_TRY(c, hipMemcpyAsync(x, hx.data(), hx.size() * sizeof(float), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(label_kernel, dim3(blocks_for(n, 128)), dim3(128), 0, st, n, x, r, y6);
        S_TRY(c, hipGetLastError());
        S_TRY(c, hipStreamSynchronize(st));   // the host rows are released on return
        if (n_rejected) *n_rejected = rejected;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_closed_form_points(isrs_ctx* c, const float* x, int64_t n, float* y)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (n < 1 || !x || !y) return ctx_fail(c, ISRS_E_ARG, "need n >= 1 and buffers");
        S_TRY(c, hipSetDevice(ctx_device(c)));
        hipLaunchKernelGGL(closed_form_kernel, dim3(blocks_for(n, 128)), dim3(128), 0, ctx_stream(c), n, x, y);
        S_TRY(c, hipGetLastError());
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_surrogate_train(isrs_ctx* c, isrs_surrogate* s, const float* x, const float* r, int64_t n,
                             const isrs_train_opts* o, double* loss_out)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!s || !x || !r || !o) return ctx_fail(c, ISRS_E_ARG, "null argument");
        if (o->batch < 64 || o->batch % 64 || o->batch > (1 << 20) || n < o->batch)
            return ctx_fail(c, ISRS_E_ARG, "batch must be a positive multiple of 64, at most n and 2^20");
        if (o->steps < 1 || !(o->lr > 0) || o->member < -1 || o->member >= s->n_members)
            return ctx_fail(c, ISRS_E_ARG, "bad steps, lr or member");
        S_TRY(c, hipSetDevice(s->device));
        hipStream_t st = ctx_stream(c);
        int32_t rc = ensure_batch(c, s, o->batch);
        if (rc) return rc;
        const int rows = o->batch;
        const int lb = (int)blocks_for(rows, 4);
        std::vector<float> lp(lb);
        if (!s->scaled) {
            hipLaunchKernelGGL(moments_kernel, dim3(1), dim3(1024), 0, st, n, r, 0, s->mom);
            hipLaunchKernelGGL(moments_kernel, dim3(1), dim3(1024), 0, st, n, r, 1, s->mom);
            double mo[2];
            S_TRY(c, hipMemcpyAsync(mo, s->mom, sizeof mo, hipMemcpyDeviceToHost, st));
            S_TRY(c, hipStreamSynchronize(st));
            const double sd = std::sqrt(mo[1] / (double)n);
            if (!std::isfinite(mo[0]) || !std::isfinite(sd)) return ctx_fail(c, ISRS_E_NUMERIC, "non-finite targets");
            s->shift = mo[0];
            s->scale = sd > 0.0 ? sd : 1.0;
            s->scaled = 1;
        }
        for (int mi = 0; mi < s->n_members; ++mi) {
            if (o->member >= 0 && mi != o->member) continue;
            auto& m = s->mem[mi];
            double tail = 0.0;
            int tail_n = 0;
            for (int it = 0; it < o->steps; ++it) {
                // member mi walks the data from its own offset
                const int64_t row0 = ((int64_t)(it + (int64_t)mi * 7919) * rows) % (n - rows + 1);
                if ((rc = pack_rows(c, s, x, row0, rows, st))) return rc;
                forward(s, m, s->xb, rows, true, s->o, false, st);
                if ((rc = backward(c, s, m, r + row0, rows, st))) return rc;
                m.step++;
                const float c1 = 1.0f - std::pow(o->beta1, (float)m.step), c2 = 1.0f - std::pow(o->beta2, (float)m.step);
                hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(NP, 256)), dim3(256), 0, st, (long)NP, m.p, s->grad, m.m,
                                   m.v, o->lr, o->beta1, o->beta2, o->eps, c1, c2);
                if ((rc = refresh_bf16(c, m, st))) return rc;
                if (it >= o->steps - 16) {
                    S_TRY(c, hipMemcpyAsync(lp.data(), s->loss_part, lb * sizeof(float), hipMemcpyDeviceToHost, st));
                    S_TRY(c, hipStreamSynchronize(st));
                    double e = 0.0;
                    for (float v : lp) e += v;
                    tail += e / rows * s->scale * s->scale;
                    tail_n++;
                }
            }
            if (loss_out) loss_out[mi] = tail / std::max(1, tail_n);
        }
        S_TRY(c, hipStreamSynchronize(st));
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_surrogate_grad(isrs_ctx* c, isrs_surrogate* s, int32_t member, const float* x, const float* r,
                            int64_t n, float* grads, double* loss)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!s || !x || !r || !grads || member < 0 || member >= s->n_members || n < 64 || n % 64 || n > (1 << 20))
            return ctx_fail(c, ISRS_E_ARG, "bad gradient request (rows: multiple of 64, at most 2^20)");
        S_TRY(c, hipSetDevice(s->device));
        hipStream_t st = ctx_stream(c);
        const int rows = (int)n;
        int32_t rc = ensure_batch(c, s, rows);
        if (rc) return rc;
        if ((rc = pack_rows(c, s, x, 0, rows, st))) return rc;
        forward(s, s->mem[member], s->xb, rows, true, s->o, false, st);
        if ((rc = backward(c, s, s->mem[member], r, rows, st))) return rc;
        S_TRY(c, hipMemcpyAsync(grads, s->grad, NP * sizeof(float), hipMemcpyDeviceToHost, st));
        const int lb = (int)blocks_for(rows, 4);
        std::vector<float> lp(lb);
        S_TRY(c, hipMemcpyAsync(lp.data(), s->loss_part, lb * sizeof(float), hipMemcpyDeviceToHost, st));
        S_TRY(c, hipStreamSynchronize(st));
        if (loss) {
            double e = 0.0;
            for (float v : lp) e += v;
            *loss = e / rows;
        }
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_surrogate_predict(isrs_ctx* c, isrs_surrogate* s, const float* x, int64_t n, float* mean, float* spread)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!s || !x || n < 1) return ctx_fail(c, ISRS_E_ARG, "null argument or n < 1");
        S_TRY(c, hipSetDevice(s->device));
        hipStream_t st = ctx_stream(c);
        int32_t rc = predict_members(c, s, x, n, st);
        if (rc) return rc;
        hipLaunchKernelGGL(ensemble_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, s->n_members, s->pred, x, mean,
                           spread, nullptr, 0.0, nullptr);
        S_TRY(c, hipGetLastError());
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_surrogate_eval_points(isrs_ctx* c, isrs_surrogate* s, const float* x, int64_t n, double thr_db, float* y,
                                   int64_t* n_fallback)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!s || !x || !y || n < 1 || n > (int64_t)1 << 31) return ctx_fail(c, ISRS_E_ARG, "bad query");
        if (std::isnan(thr_db)) return ctx_fail(c, ISRS_E_ARG, "threshold is NaN");
        S_TRY(c, hipSetDevice(s->device));
        hipStream_t st = ctx_stream(c);
        int32_t rc = predict_members(c, s, x, n, st);
        if (rc) return rc;
        // spread of ln|mu|^2 in dB of |mu|^2: 10 log10(e) per ln unit
        const double thr_ln = thr_db < 0 ? -1.0 : thr_db / (10.0 / std::log(10.0));
        hipLaunchKernelGGL(ensemble_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, s->n_members, s->pred, x,
                           nullptr, nullptr, y, thr_ln, s->flag);
        const int64_t nb = (n + CB - 1) / CB;
        hipLaunchKernelGGL(count_kernel, dim3((unsigned)nb), dim3(CB), 0, st, n, s->flag, s->cnt);
        hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(SCAN_T), 0, st, (int)nb, s->cnt, s->off, s->total);
        hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)nb), dim3(CB), 0, st, n, s->flag, s->off, s->idx);
        hipLaunchKernelGGL(fallback_kernel, dim3(blocks_for(n, 128)), dim3(128), 0, st, s->total, s->idx, x, y);
        S_TRY(c, hipGetLastError());
        if (n_fallback) {
            int t = 0;
            S_TRY(c, hipMemcpyAsync(&t, s->total, sizeof(int), hipMemcpyDeviceToHost, st));
            S_TRY(c, hipStreamSynchronize(st));
            *n_fallback = t;
        }
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_surrogate_calibrate(isrs_ctx* c, isrs_surrogate* s, const float* x, int64_t n, double target_db,
                                 double* threshold_db, double* max_err_db, double* accepted_fraction)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!s || !x || !threshold_db || n < 1 || n > (int64_t)1 << 31)
            return ctx_fail(c, ISRS_E_ARG, "null argument or bad n");
        if (!(target_db > 0) || !std::isfinite(target_db)) return ctx_fail(c, ISRS_E_ARG, "target must be > 0");
        S_TRY(c, hipSetDevice(s->device));
        hipStream_t st = ctx_stream(c);
        int32_t rc = predict_members(c, s, x, n, st);
        if (rc) return rc;
        if (n > s->ccap) {
            release(s->cal);
            s->ccap = 0;
            S_TRY(c, dalloc(&s->cal, (size_t)n * 3));
            s->ccap = n;
        }
        float* mean = s->cal;
        float* spread = s->cal + n;
        float* ref = s->cal + 2 * n;
        hipLaunchKernelGGL(ensemble_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, s->n_members, s->pred, x, mean,
                           spread, nullptr, 0.0, nullptr);
        hipLaunchKernelGGL(label_kernel, dim3(blocks_for(n, 128)), dim3(128), 0, st, n, x, ref, nullptr);
        S_TRY(c, hipGetLastError());
        std::vector<float> h((size_t)n * 3);
        S_TRY(c, hipMemcpyAsync(h.data(), s->cal, h.size() * sizeof(float), hipMemcpyDeviceToHost, st));
        S_TRY(c, hipStreamSynchronize(st));
        // errors and spreads in dB of |mu|^2; accept points in order of spread
        // while the largest error so far stays within the target, and stop only
        // between distinct spreads (the gate accepts spread <= threshold)
        const double db = 10.0 / std::log(10.0);
        std::vector<int64_t> order((size_t)n);
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return h[n + a] < h[n + b]; });
        double run = 0.0, best_err = 0.0;
        int64_t best = 0;
        for (int64_t k = 0; k < n; ++k) {
            const int64_t i = order[k];
            const double e = std::fabs((double)h[i] - (double)h[2 * n + i]) * db;
            if (!(e <= target_db) || std::isnan(e)) break;
            run = std::max(run, e);
            if (k + 1 == n || h[n + order[k + 1]] > h[n + i]) {
                best = k + 1;
                best_err = run;
            }
        }
        *threshold_db = best > 0 ? (double)h[n + order[best - 1]] * db : -1.0;
        if (max_err_db) *max_err_db = best_err;
        if (accepted_fraction) *accepted_fraction = (double)best / (double)n;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_surrogate_get_target_scale(const isrs_surrogate* s, double* shift, double* scale)
{
    try {
        if (!s || !shift || !scale) return ISRS_E_ARG;
        *shift = s->shift;
        *scale = s->scale;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(nullptr);
    }
}

int32_t isrs_surrogate_get_params(isrs_surrogate* s, int32_t member, float* p)
{
    try {
        if (!s || !p || member < 0 || member >= s->n_members) return ISRS_E_ARG;
        if (hipSetDevice(s->device) != hipSuccess) return ISRS_E_DEVICE;
        if (hipDeviceSynchronize() != hipSuccess) return ISRS_E_DEVICE;
        if (hipMemcpy(p, s->mem[member].p, NP * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) return ISRS_E_DEVICE;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(nullptr);
    }
}

int32_t isrs_surrogate_set_params(isrs_ctx* c, isrs_surrogate* s, int32_t member, const float* p)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!s || !p || member < 0 || member >= s->n_members) return ctx_fail(c, ISRS_E_ARG, "bad member or params");
        for (long i = 0; i < NP; ++i)
            if (!std::isfinite(p[i])) return ctx_fail(c, ISRS_E_NUMERIC, "non-finite parameter");
        S_TRY(c, hipSetDevice(s->device));
        hipStream_t st = ctx_stream(c);
        S_TRY(c, hipStreamSynchronize(st));
        S_TRY(c, hipMemcpy(s->mem[member].p, p, NP * sizeof(float), hipMemcpyHostToDevice));
        int32_t rc = refresh_bf16(c, s->mem[member], st);
        if (rc) return rc;
        S_TRY(c, hipStreamSynchronize(st));
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_surrogate_save(isrs_surrogate* s, const char* path)
{
    try {
        if (!s || !path) return ISRS_E_ARG;
        if (hipSetDevice(s->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return ISRS_E_DEVICE;
        std::ofstream f(path, std::ios::binary | std::ios::trunc);
        if (!f) return ISRS_E_ARG;
        const char magic[8] = {'I', 'S', 'R', 'S', 'S', 'U', 'R', '1'};
        const int64_t hdr[4] = {s->n_members, (int64_t)s->seed, NP, s->scaled};
        const double sc[2] = {s->shift, s->scale};
        f.write(magic, 8);
        f.write(reinterpret_cast<const char*>(hdr), sizeof hdr);
        f.write(reinterpret_cast<const char*>(sc), sizeof sc);
        std::vector<float> buf(NP);
        for (auto& m : s->mem) {
            f.write(reinterpret_cast<const char*>(&m.step), sizeof m.step);
            for (float* d : {m.p, m.m, m.v}) {
                if (hipMemcpy(buf.data(), d, NP * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) return ISRS_E_DEVICE;
                f.write(reinterpret_cast<const char*>(buf.data()), NP * sizeof(float));
            }
        }
        return f ? ISRS_OK : ISRS_E_ARG;
    } catch (...) {
        return abi_exception(nullptr);
    }
}

int32_t isrs_surrogate_load(isrs_ctx* c, isrs_surrogate* s, const char* path)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!s || !path) return ctx_fail(c, ISRS_E_ARG, "null argument");
        std::ifstream f(path, std::ios::binary);
        if (!f) return ctx_fail(c, ISRS_E_ARG, "cannot open checkpoint");
        char magic[8];
        int64_t hdr[4];
        double sc[2];
        f.read(magic, 8);
        f.read(reinterpret_cast<char*>(hdr), sizeof hdr);
        f.read(reinterpret_cast<char*>(sc), sizeof sc);
        if (!f || std::memcmp(magic, "ISRSSUR1", 8) != 0 || hdr[0] != s->n_members || hdr[2] != NP)
            return ctx_fail(c, ISRS_E_ARG, "checkpoint does not match this surrogate");
        S_TRY(c, hipSetDevice(s->device));
        hipStream_t st = ctx_stream(c);
        S_TRY(c, hipStreamSynchronize(st));
        std::vector<float> buf(NP);
        for (auto& m : s->mem) {
            f.read(reinterpret_cast<char*>(&m.step), sizeof m.step);
            for (float* d : {m.p, m.m, m.v}) {
                f.read(reinterpret_cast<char*>(buf.data()), NP * sizeof(float));
                if (!f) return ctx_fail(c, ISRS_E_ARG, "truncated checkpoint");
                S_TRY(c, hipMemcpy(d, buf.data(), NP * sizeof(float), hipMemcpyHostToDevice));
            }
            int32_t rc = refresh_bf16(c, m, st);
            if (rc) return rc;
        }
        s->seed = (uint64_t)hdr[1];
        s->scaled = hdr[3];
        s->shift = sc[0];
        s->scale = sc[1];
        S_TRY(c, hipStreamSynchronize(st));
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

int32_t isrs_eval_eta_surrogate(isrs_ctx* c, isrs_surrogate* s, const isrs_numerics* nu, const int32_t* cuts,
                                int32_t n_cut, double thr_db, double* eta, double* fallback_fraction)
{
    try {
        if (!c) return ISRS_E_ARG;
        if (!s || !nu || !cuts || !eta) return ctx_fail(c, ISRS_E_ARG, "null argument");
        if (std::isnan(thr_db)) return ctx_fail(c, ISRS_E_ARG, "threshold is NaN");
        S_TRY(c, hipSetDevice(s->device));
        struct Fill : SurrogateFill {
            isrs_surrogate* s;
            double thr_ln;
            int64_t live = 0, fb = 0;
            int32_t fill(isrs_ctx* c, const RegionArgs& ra, int item0, int item1, int n_sp, float* tab,
                         hipStream_t st) override
            {
                const int64_t rows = (int64_t)(item1 - item0) * ra.N * ra.N * n_sp;
                if (rows == 0) return ISRS_OK;
                const unsigned nb = blocks_for(rows, 256);
                if (rows > s->qcap) {
                    release(s->qx);
                    release(s->qstate);
                    release(s->qcnt);
                    s->qcap = 0;
                    S_TRY(c, dalloc(&s->qx, (size_t)rows * NIN));
                    S_TRY(c, dalloc(&s->qstate, (size_t)rows));
                    S_TRY(c, dalloc(&s->qcnt, 2 * (size_t)nb));
                    s->qcap = rows;
                }
                hipLaunchKernelGGL(sur_query_kernel, dim3(nb), dim3(256), 0, st, ra, item0, rows, n_sp, s->qx, s->qstate);
                S_TRY(c, hipGetLastError());
                int32_t rc = predict_members(c, s, s->qx, rows, st);
                if (rc) return rc;
                hipLaunchKernelGGL(sur_combine_kernel, dim3(nb), dim3(256), 0, st, rows, s->n_members, s->pred,
                                   s->qstate, thr_ln, tab, s->qcnt, s->qcnt + nb);
                S_TRY(c, hipGetLastError());
                std::vector<int> h(2 * (size_t)nb);
                S_TRY(c, hipMemcpyAsync(h.data(), s->qcnt, h.size() * sizeof(int), hipMemcpyDeviceToHost, st));
                S_TRY(c, hipStreamSynchronize(st));
                for (unsigned b = 0; b < nb; ++b) {
                    live += h[b];
                    fb += h[nb + b];
                }
                return ISRS_OK;
            }
        } f;
        f.s = s;
        f.thr_ln = thr_db < 0 ? -1.0 : thr_db / (10.0 / std::log(10.0));
        int32_t rc = eval_eta_table(c, nu, cuts, n_cut, f, eta);
        if (rc) return rc;
        if (fallback_fraction) *fallback_fraction = f.live > 0 ? (double)f.fb / (double)f.live : 0.0;
        return ISRS_OK;
    } catch (...) {
        return abi_exception(c);
    }
}

}  // extern "C"
