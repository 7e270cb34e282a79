// isrs_internal.h -- device-side data layout shared by the host layer
// (isrs_api.cpp) and the gfx950 kernels (isrs_kernels.hip).  Not installed;
// the public interface is include/isrs_egn.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/isrs_egn.h"

namespace isrs {

// Region kernel: 256 threads; each owns a run of PPT consecutive points of
// one anti-diagonal of the N x N grid (per precision; 4 in both: 2-point runs
// in FP64 fit four waves per SIMD but ran 4% slower at three and 18% slower at
// four, with twice the slices to stage).  Runs are listed by anti-diagonal,
// and a slice (THREADS consecutive runs) spans at most NAD anti-diagonals for
// every N (59 at most, at N = 30, with 4-point runs; 43 with 2-point runs),
// which bounds the staged LDS rows.
constexpr int THREADS = 256;
constexpr int PPT32 = 4;              // points per run, FP32 integrand
constexpr int PPT64 = 4;              // points per run, FP64
constexpr int ppt_of(bool fp32) { return fp32 ? PPT32 : PPT64; }
constexpr int NAD = 63;               // staged anti-diagonal rows per slice
constexpr int RUN_SHIFT = 13;         // run = m << RUN_SHIFT | first column, N <= 8192
constexpr int RUN_MASK = (1 << RUN_SHIFT) - 1;
constexpr int STAGE_RUN = 8;          // anti-diagonals per staging run (one exp, then a recurrence)

// Forms of the per-span FWM factor run by the region kernel.
constexpr int MU_SEG = 0;             // segment closed form, Eqs. 7-10
constexpr int MU_MAC = 1;             // Maclaurin closed form, Eqs. 2-6
constexpr int MU_INT = 2;             // integral form, Eq. 23, by 4-node product integration per segment
constexpr int MU_SUR = 3;             // surrogate residual table with segment fallback (internal)
constexpr int INT_NODES = 4;
// Gauss-Legendre nodes on [-1, 1] at which the integral form samples the gain
// inside each segment (node n of segment k at z = (k + 1/2 + u_n / 2) Delta).
constexpr double INT_U[INT_NODES] = {-0.86113631159405258, -0.33998104358485626, 0.33998104358485626,
                                     0.86113631159405258};

// Per-span constants, all FP64.  The phase of the segment step, Eq. 9, is
// chi * Delta with chi of Eq. 24; the accumulated phase of Eq. 22 is Theta_s.
// Both are formed in revolutions from d12 = (f1-f)(f2-f) and s = f1 + f2:
//   chi Delta / 2pi = d12 (c2r + c3r s),   Theta_s / 2pi = d12 (p2r + p3r s),
//   chi = d12 (c2x + c3x s)  [rad/km].
struct SpanConst {
    double c2r, c3r;       // 2 pi beta2 Delta,  2 pi^2 beta3 Delta
    double c2x, c3x;       // 4 pi^2 beta2,      4 pi^3 beta3
    double wd;             // 2 pi / Delta: chi = wd * (chi Delta / 2 pi)
    double L, cr, ptot, btot;  // length (km), Cr, total power (W) and bandwidth (THz) of Eq. 25
    double p2r, p3r;       // 2 pi sum_{s'<s} beta2 L,  2 pi^2 sum_{s'<s} beta3 L
    double c2L, c3L;       // 2 pi beta2 L,  2 pi^2 beta3 L  (Maclaurin form)
    double em;             // exp(-alpha Delta)
    double emL, em2L;      // exp(-alpha L), exp(-2 alpha L)
    double alpha;          // 1/km
    double gamma;          // 1/(W km)
    double pcr;            // Ptot Cr (Maclaurin form), 1/(km THz)
    double pi_a, pi_s, pi_c;  // LOSS_ONLY gain: ln Pi_s = pi_a - pi_s (a+b) + pi_c c
    int K;                 // segments
    int off;               // offset of the span's rows in the segment tables
    // FP32 copies for the FP32 integrand (no per-wave conversions)
    float f_alpha, f_em, f_ms, f_wd, f_gamma, f_emL, f_em2L, f_pad;  // f_ms = -em^2
};

// Segment table row k of a span: SRS gain at z_k = A exp(-zeta f3abs)
// (Eq. 8 with Eq. 10) and the step ratio exp(-zeta h) between neighbouring
// anti-diagonals of the grid.  The integral form keeps INT_NODES such tables
// per span (rows off + n K + k), sampled at the nodes inside each segment.
struct SegRow64 {
    double A, zeta, ratio, pad;
};
struct SegRow32 {
    float A, zeta, ratio, pad;
};

// One link (spectrum + spans) of an evaluation; offsets index the
// concatenated tables of all links.
struct LinkDesc {
    int span0, n_sp;      // spans[span0 .. span0 + n_sp)
    int n_ch, gain_mode;
    int ch0;              // power / phi / psi
    int tab0;             // island weight / S(f3) tables: n_f * 3 * (2N-1) per link
    int livep0;           // live prefix counts: n_f * 3 * 2N per link
    int sg0;              // S at the grid points: N per link
    double spacing, h, rs;
};

// One (link, CUT, outer-frequency) instance.
struct InstDesc {
    double f;        // outer frequency offset from the CUT centre, THz
    int link;
    int cut;         // channel index within the link
    int nf_idx;      // outer-frequency sample -> island tables
    int sq_begin;    // its squares in the work list
    int sq_end;
};

// Coherent-sum accumulators of one persistent block, in complex FP64: row
// sums [3 islands][N] (E), column sums [3][N] (F), anti-diagonal sums [2N]
// (G and H).  The slot stride is padded by 24 entries (384 B) so that the
// slots of neighbouring blocks do not all fall into the same L2 sets.
__host__ __device__ constexpr size_t eslot(int N) { return (size_t)8 * N + 24; }

// One channel-pair square of the (f1 <-> f2 folded) work list.
struct SquareItem {
    int inst;
    int k1, k2;
    int lmask;       // bit (l+1): island l has a valid third channel and live points
    int egn_mask;    // bit 4*(l+1) + t, t = 0 E (rows), 1 F (columns), 2 G (anti-diagonals), 3 H (full)
    int pad_;
    int d_index;     // row in the coherent-sum results, -1 if none
    float mult;      // 2 for k1 < k2 (mirror square folded in), else 1
};

// A launch covers work units [unit0, unit0 + n_units); unit u is slice group
// u % n_groups of square u / n_groups.  A square with coherent sums
// (egn_mask != 0) is run whole by its group 0, whose block keeps the sums in
// its accumulator slot; its other groups only write zero partials.  With a
// queue, blocks pop positions from *counter and run unit order[unit0 + pos]
// (a cost-sorted permutation of the launch's units); without one, block b
// runs unit unit0 + b (only for plans without coherent sums).
struct RegionArgs {
    const LinkDesc* links;
    const SpanConst* spans;
    const void* seg;          // SegRow32 or SegRow64 rows
    const double* Sg;
    const double* wt;
    const double* s3;
    const int* livep;
    const InstDesc* insts;
    const SquareItem* items;
    double* partD;            // [units][3]
    double* partE;            // [coherent-sum squares][3 islands][E, F, G, H]
    double2* eacc;            // coherent-sum accumulators, one slot of eslot(N) complex per persistent block
    const int* adrun;         // [2N] first run of each anti-diagonal (run table index), then the run count
    const int* order;         // queue mode: permutation of units, else null
    int* counter;             // queue mode: head counter (zeroed before the launch)
    int unit0;
    int n_units;
    int n_groups;             // slice groups per square
    int spb;                  // slices per group
    int n_slices;             // slices per square
    const int* runs;          // [n_runs] runs of the N x N grid by anti-diagonal
    int n_runs;
    int N;
    int mu_method;            // MU_SEG, MU_MAC, MU_INT or MU_SUR
    const float* sur_tab;     // MU_SUR: ln(|mu|^2 / |eta_6|^2) per (point, span), NaN = closed form;
    int sur_item0;            //   row ((item - sur_item0) * N + j) * N + i) * n_sp + s
};

struct AssembleArgs {
    const LinkDesc* links;
    const InstDesc* insts;
    const SquareItem* items;
    const double* partD;
    const double* partE;
    const double* power;      // concatenated per link
    const double* phi;
    const double* psi;
    double* eta;              // [n_cut]
    double* sigma2;           // [n_cut] or null
    double* terms;            // [n_cut][5] or null
    double* psd;              // [n_cut][n_f] or null
    int n_groups;
    int n_f;
    int n_cut;
};

// Device scratch of the allocation-free evaluation (isrs_eval_eta_dev_noalloc):
// a file-scope array in isrs_kernels.hip, one copy per GPU, held until the
// process ends.  noalloc_scratch() returns this device's copy (the device must
// be current); the address is looked up once per device and kept.
constexpr size_t NOALLOC_BYTES = size_t(64) << 20;
hipError_t noalloc_scratch(int device, void** ptr);

// Kernel launchers (isrs_kernels.hip).  blocks = 0 launches one block per
// unit; blocks > 0 launches that many persistent blocks on the queue.
hipError_t launch_region(const RegionArgs& a, int blocks, bool fp32, int ppt, hipStream_t st);
bool region_ppt_supported(bool fp32, int mu_method, int ppt);   // points per run with a kernel instance
hipError_t launch_zero_counter(int* counter, hipStream_t st);
hipError_t launch_assemble(const AssembleArgs& a, hipStream_t st);
int region_blocks_per_cu(bool fp32, int mu_method, int ppt);

}  // namespace isrs

// Context accessors for the surrogate's host code (isrs_surrogate.hip).
namespace isrs {
hipStream_t ctx_stream(isrs_ctx* c);
int ctx_device(const isrs_ctx* c);
int ctx_num_cu(const isrs_ctx* c);
int32_t ctx_fail(isrs_ctx* c, int32_t code, const char* msg);
int32_t abi_exception(isrs_ctx* c);   // inside a catch handler: status of the current exception

// Evaluation of the context's link with the region kernel reading a residual
// table (mu_method 2): before each launch chunk, fill() writes the table rows
// of squares [item0, item1) and counts live and fallback rows.
struct SurrogateFill {
    virtual ~SurrogateFill() = default;
    virtual int32_t fill(isrs_ctx* c, const RegionArgs& ra, int item0, int item1, int n_sp, float* tab,
                         hipStream_t st) = 0;
};
constexpr int64_t SUR_TAB_ROWS = int64_t(1) << 25;  // table rows per launch chunk

// Read-only view of one link of a batch (host arrays owned by the batch).
struct LinkView {
    int n_ch;
    double spacing, rs, rolloff;
    const double* power;
    const isrs_span* spans;
    int n_sp;
    const int32_t* cuts;
    int n_cut;
};
int batch_num_links(const isrs_batch* b);
LinkView batch_link_view(const isrs_batch* b, int link);
int32_t eval_eta_table(isrs_ctx* c, const isrs_numerics* nu, const int32_t* cuts, int n_cut, SurrogateFill& sf,
                       double* eta_host);
}  // namespace isrs
