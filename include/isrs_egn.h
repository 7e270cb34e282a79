/*
 * isrs_egn.h -- C-ABI of the MI355X (gfx950) ISRS-aware EGN library.
 *
 * The library evaluates, per channel under test (CUT), the nonlinear
 * interference (NLI) of a WDM link with inter-channel stimulated Raman
 * scattering (ISRS) as in "Acceleration and Parallelization Methods for ISRS
 * EGN Model" (arXiv 2412.11614):
 *   - the NLI variance sigma^2 (Eq. 15) summed over the islands of the set
 *     T_kappa (Eq. 16), with the GN term D (Eq. 17) and the modulation-format
 *     terms E, F, G, H (Eqs. 18-21);
 *   - the link function Upsilon (Eq. 22), whose per-span FWM efficiency
 *     factor mu_s (Eq. 23) is taken from the segment closed form (Eqs. 7-10),
 *     or, on request, the Maclaurin closed form (Eqs. 2-6), the integral
 *     form itself (Eq. 23 by product integration), or a learned surrogate
 *     with closed-form fallback;
 *   - the NLI coefficient eta = sigma^2 / P^3 (Eq. 11) and the NLI PSD.
 *
 * Conventions shared by every call
 *   Units: frequencies THz, lengths km, powers W, alpha dB/km, beta2 ps^2/km,
 *   beta3 ps^3/km, gamma 1/(W km), Raman gain slope Cr 1/(W km THz).
 *   Channel k of an n_ch grid sits at (k - (n_ch-1)/2) * spacing from the
 *   grid centre; the ISRS profile (Eq. 25) uses that origin, B_tot =
 *   n_ch * spacing and P_tot = sum of the launch powers.  |S(f)|^2 is the
 *   raised-cosine shape divided by Rs^2.  Each channel-pair square is an
 *   N x N midpoint grid over the channel's spectral support; a point belongs
 *   to island l when |f1 + f2 - f - l*spacing| <= (1+rolloff) Rs / 2.
 *
 *   Every call returns an isrs_status: ISRS_OK (0) or a negative code.
 *   Inputs are validated before any device work; on error nothing is
 *   launched and isrs_last_error() describes the first problem found.
 *   Pointers documented as "host" are read or written by the CPU during
 *   the call; "device" pointers must be device memory of the context's GPU.
 *   The library copies what it needs: callers keep ownership of every
 *   buffer they pass.  No call throws across the boundary.
 *
 *   A context works on one HIP stream: the caller's, or (hip_stream NULL)
 *   a non-blocking stream of its own, which is not ordered with the
 *   caller's work, so device outputs of the *_dev calls are then valid
 *   after a device or stream synchronisation.  It owns device scratch that
 *   it grows on demand and frees in isrs_destroy.  Use one context per host
 *   thread; calls on one context must not overlap.
 */
#ifndef ISRS_EGN_H
#define ISRS_EGN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define ISRS_OK 0
#define ISRS_E_ARG (-1)       /* bad argument: null pointer, size, numerics, CUT index */
#define ISRS_E_SPECTRUM (-2)  /* bad spectrum: non-finite, negative power, (1+ro)Rs > spacing, ... */
#define ISRS_E_LINK (-3)      /* bad span list: non-positive length or loss, non-finite values */
#define ISRS_E_STATE (-4)     /* evaluation before isrs_set_spectrum / isrs_set_link */
#define ISRS_E_DEVICE (-5)    /* no usable gfx950 device, or a HIP runtime error */
#define ISRS_E_NOMEM (-6)     /* device or host allocation failed */
#define ISRS_E_NUMERIC (-7)   /* a result came out non-finite */

/* Amplifier gain reading for the products of Eq. 22. */
#define ISRS_GAIN_EQUALIZED 0 /* gain restores the launch profile: all products are 1 */
#define ISRS_GAIN_LOSS_ONLY 1 /* g_s = exp(alpha_s L_s): products taken literally */

/* Arithmetic of the per-point integrand. */
#define ISRS_PREC_FP64 0         /* everything in FP64 */
#define ISRS_PREC_FP32_PHASE64 1 /* phases reduced in FP64, integrand in FP32, sums in FP64 */

/* FWM efficiency factor per span. */
#define ISRS_MU_SEGMENT 0   /* segment closed form, Eqs. 7-10 */
#define ISRS_MU_MACLAURIN 1 /* Maclaurin closed form, Eqs. 2-6 */
#define ISRS_MU_INTEGRAL 2  /* integral form, Eq. 23: on each of the K = ceil(L / dz) segments the
                             * SRS gain is interpolated at 4 Gauss-Legendre nodes and the product
                             * with exp((i chi - alpha) z) integrated exactly (error O(dz^4) for any
                             * chi); the reference the closed forms approximate */

typedef struct isrs_ctx isrs_ctx;

/* WDM spectrum (the problem statement of Sec. II-B; P, Phi, Psi of Eq. 15).
 * power_w[k] = 0 marks an empty slot.  phi/psi are the format constants of
 * the EGN correction terms (e.g. QPSK -1 / 4, Gaussian 0 / 0).  All arrays
 * are host arrays of n_ch doubles, copied by isrs_set_spectrum. */
typedef struct {
    int32_t n_ch;
    double f_center_thz;     /* informational: absolute grid centre */
    double spacing_thz;      /* channel spacing */
    double symbol_rate_thz;  /* Rs */
    double rolloff;          /* raised-cosine roll-off in [0, 1] */
    const double* power_w;   /* [n_ch] launch power per channel, W */
    const double* phi;       /* [n_ch] */
    const double* psi;       /* [n_ch] */
} isrs_spectrum;

/* One fibre span (parameters of Eqs. 22-25). */
typedef struct {
    double length_km;
    double alpha_db_km;
    double beta2_ps2_km;
    double beta3_ps3_km;
    double gamma_w_km;
    double cr_w_km_thz;
} isrs_span;

/* Discretisation and arithmetic.  n1 == n2 = N is the grid per square;
 * n_f outer samples of f over [-Rs/2, Rs/2] (1: the CUT centre, then
 * sigma^2 = Rs * PSD(0)); K_s = ceil(L_s / dz_km) segments per span
 * (Eq. 7-10, Sec. II-C); egn = 0 keeps only the GN term D. */
typedef struct {
    double dz_km;
    int32_t n1, n2, n_f;
    int32_t egn;
    int32_t precision;  /* ISRS_PREC_* */
    int32_t mu_method;  /* ISRS_MU_* */
} isrs_numerics;

/* Counters and timings of the last evaluation on a context. */
typedef struct {
    double region_ms;       /* summed duration of the region-kernel launches (HIP events) */
    double egn_ms;          /* summed duration of the EGN-sum launches */
    double assemble_ms;     /* per-CUT assembly launch */
    double host_prep_ms;    /* host-side tables and work list */
    int64_t region_launches;
    int64_t n_squares;      /* channel-pair squares evaluated (f1<->f2 folded) */
    int64_t n_delta_squares;/* squares needing the E/F/G/H coherent sums */
    int64_t n_points_live;  /* grid points on live islands, folded squares */
    int64_t horner_steps;   /* sum over live points and spans of K_s */
    double alg_flop;        /* algorithmic FLOP: sum over live point-spans of 8 K_s + 30 */
} isrs_stats;

/* Context lifetime.  device: HIP device ordinal; hip_stream: a hipStream_t
 * to order all work on, or NULL for the library's own stream.  Fails with
 * ISRS_E_DEVICE when the device is absent or not gfx950. */
int32_t isrs_create(isrs_ctx** out, int32_t device, void* hip_stream);
int32_t isrs_destroy(isrs_ctx* ctx);

/* Message of the last failure on ctx ("" if none).  ctx may be NULL, then
 * the message of the last failed isrs_create on this thread. */
const char* isrs_last_error(const isrs_ctx* ctx);

/* Deep-copies the spectrum (Sec. II-B problem statement; P, Phi, Psi of
 * Eq. 15).  Errors: ISRS_E_ARG (null), ISRS_E_SPECTRUM (invalid values). */
int32_t isrs_set_spectrum(isrs_ctx* ctx, const isrs_spectrum* spectrum);

/* Deep-copies n_spans spans (Eqs. 22-25) and the gain reading.
 * Errors: ISRS_E_ARG, ISRS_E_LINK. */
int32_t isrs_set_link(isrs_ctx* ctx, const isrs_span* spans, int32_t n_spans, int32_t gain_mode);

/* Freezes P_tot of the ISRS profile (Eq. 25) at ptot_w (> 0), or restores
 * the sum of launch powers (ptot_w = 0). */
int32_t isrs_set_ptot_override(isrs_ctx* ctx, double ptot_w);

/* NLI coefficient per CUT, Eq. 11 (and sigma^2 of Eq. 15).
 * cuts: host [n_cut] channel indices (active channels).
 * eta: host [n_cut] 1/W^2; sigma2: host [n_cut] W or NULL; terms: host
 * [n_cut*5] or NULL, the D, E, F, G, H contributions to sigma^2 (they sum
 * to sigma^2).  Synchronises the stream before returning.
 * Errors: ISRS_E_ARG, ISRS_E_STATE, ISRS_E_DEVICE, ISRS_E_NOMEM, ISRS_E_NUMERIC. */
int32_t isrs_eval_eta(isrs_ctx* ctx, const isrs_numerics* numerics, const int32_t* cuts, int32_t n_cut,
                      double* eta, double* sigma2, double* terms);

/* As isrs_eval_eta with device outputs (eta_dev [n_cut], sigma2_dev and
 * terms_dev nullable); stream-ordered, does not synchronise and does not
 * check results for finiteness.  cuts stays a host array. */
int32_t isrs_eval_eta_dev(isrs_ctx* ctx, const isrs_numerics* numerics, const int32_t* cuts, int32_t n_cut,
                          double* eta_dev, double* sigma2_dev, double* terms_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation and outputs as isrs_eval_eta_dev, with every device buffer
 * beyond the caller's inputs and outputs (tables, work list, partial sums,
 * coherent-sum accumulators, queue counter) placed in a fixed 64 MiB device
 * array that each GPU holds from library load to process exit.  The call
 * makes no hipMalloc, hipFree or hipHostMalloc; it plans on the host and
 * copies the tables from host memory into that array on the context's stream.
 * Plans with coherent sums get as many persistent blocks as accumulator slots
 * fit after the tables (at least one).  An evaluation whose buffers exceed
 * the 64 MiB fails with ISRS_E_ARG, naming the size it needs; nothing is
 * launched.  Every context on a GPU shares that GPU's array, which keeps the
 * last call's contents: calls that overlap on one GPU (two contexts on
 * different streams) race, so order them.  The surrogate, per-CUT steps and
 * explicit squares are not offered here. */
int32_t isrs_eval_eta_dev_noalloc(isrs_ctx* ctx, const isrs_numerics* numerics, const int32_t* cuts,
                                  int32_t n_cut, double* eta_dev, double* sigma2_dev, double* terms_dev);

/* eta with a sampling step per CUT: dz_km[q] replaces numerics->dz_km for
 * cuts[q] (Sec. III-C: the segment form's step can follow the COI's
 * frequency).  CUTs sharing a step share segment tables.  Outputs, units and
 * errors as isrs_eval_eta; a bad step names its CUT (ISRS_E_ARG). */
int32_t isrs_eval_eta_dz(isrs_ctx* ctx, const isrs_numerics* numerics, const int32_t* cuts, int32_t n_cut,
                         const double* dz_km, double* eta, double* sigma2, double* terms);

/* Error-model step choice: eta of every CUT at each candidate step (on the
 * given numerics, normally a coarse grid) against the smallest candidate;
 * dz_out[q] (host) receives the largest candidate whose |error| is within
 * target_db (the smallest candidate if none is).  err_db_out (host,
 * nullable, [n_cand][n_cut], candidates ascending) receives the errors. */
int32_t isrs_choose_dz(isrs_ctx* ctx, const isrs_numerics* numerics, const int32_t* cuts, int32_t n_cut,
                       const double* candidates, int32_t n_cand, double target_db, double* dz_out,
                       double* err_db_out);

/* NLI PSD at the n_f outer samples of each CUT (Eq. 15 without the outer
 * integral over f): f_thz host [n_cut*n_f] offsets from the CUT centre,
 * psd host [n_cut*n_f] in W/THz.  sigma^2 = sum_f (Rs/n_f) psd. */
int32_t isrs_eval_psd(isrs_ctx* ctx, const isrs_numerics* numerics, const int32_t* cuts, int32_t n_cut,
                      double* f_thz, double* psd_w_per_thz);

/* Island-level values for checking: for CUT `cut` and m squares
 * kappa12 = host [m*2] (k1, k2) pairs, writes host partials[m*15]: for
 * l = -1, 0, 1 the bare integrals D, E, F, G, H of Eqs. 17-21 at f = 0
 * (no R^n prefactors, constants, powers or format factors).  Islands whose
 * third channel is outside the grid or inactive are 0. */
int32_t isrs_eval_islands(isrs_ctx* ctx, const isrs_numerics* numerics, int32_t cut,
                          const int32_t* kappa12, int32_t m, double* partials);

/* Counters of the last evaluation; set profile = 1 to time each launch
 * with HIP events (adds a small host overhead per launch). */
int32_t isrs_set_profiling(isrs_ctx* ctx, int32_t profile);
int32_t isrs_get_stats(const isrs_ctx* ctx, isrs_stats* out);

/* ------------------------------------------------------------------------
 * Batched evaluation of many links in one persistent launch.
 *
 * A batch holds n_links independent links (each its own spectrum, span
 * list and CUT list), concatenated CSR-style.  Evaluation runs every
 * (link, CUT, channel-pair square) of the batch through one cost-sorted
 * work queue (the islands are independent: Sec. II-B), captured in a HIP
 * graph on the first call and replayed by later calls with the same
 * numerics; other numerics rebuild the work list and re-capture.
 * ------------------------------------------------------------------------ */
typedef struct isrs_batch isrs_batch;

typedef struct {
    int32_t n_links;
    const int32_t* ch_offset;      /* [n_links+1] link l owns channels ch_offset[l] .. ch_offset[l+1]-1 */
    const int32_t* span_offset;    /* [n_links+1] link l owns spans span_offset[l] .. span_offset[l+1]-1 */
    const int32_t* cut_offset;     /* [n_links+1] into cuts, or NULL: every active channel is a CUT */
    const int32_t* cuts;           /* concatenated CUT channel indices (local to each link), or NULL */
    const double* spacing_thz;     /* [n_links] */
    const double* symbol_rate_thz; /* [n_links] */
    const double* rolloff;         /* [n_links] */
    const int32_t* gain_mode;      /* [n_links] ISRS_GAIN_*, or NULL for EQUALIZED */
    const double* power_w;         /* [ch_offset[n_links]] launch powers, 0 = inactive */
    const double* phi;             /* [ch_offset[n_links]] */
    const double* psi;             /* [ch_offset[n_links]] */
    const isrs_span* spans;        /* [span_offset[n_links]] */
} isrs_link_batch;

/* Validates and deep-copies a batch (host arrays).  Errors: ISRS_E_ARG,
 * ISRS_E_SPECTRUM / ISRS_E_LINK with the offending link in the message. */
int32_t isrs_batch_create(isrs_ctx* ctx, const isrs_link_batch* batch, isrs_batch** out);
int32_t isrs_batch_destroy(isrs_batch* batch);

/* Number of CUTs of the batch (the length of the eta outputs). */
int32_t isrs_batch_num_cuts(const isrs_batch* batch, int64_t* n_cuts);

/* eta of every CUT of every link (link order, then CUT order), host
 * [n_cuts] 1/W^2; synchronises the context's stream.  The first call with
 * given numerics builds the work list and captures a HIP graph; later calls
 * replay it.  Errors as isrs_eval_eta. */
int32_t isrs_batch_eval(isrs_ctx* ctx, isrs_batch* batch, const isrs_numerics* numerics, double* eta);

/* As isrs_batch_eval with a device output [n_cuts]; stream-ordered. */
int32_t isrs_batch_eval_dev(isrs_ctx* ctx, isrs_batch* batch, const isrs_numerics* numerics, double* eta_dev);

/* Launch-shape autotuner (the islands are independent work of uneven cost,
 * Sec. II-B): times candidate region launches on this batch and keeps the
 * fastest.  Candidates: persistent blocks per CU in {2, 4} on the
 * cost-sorted queue (and, without format terms, one block per work unit);
 * the automatic slice grouping or one slice per unit; region-tile geometry:
 * runs of 2, 4 or 8 points per thread (FP32 segment form; each only where
 * every slice of 256 runs fits the kernel's staged gain rows).  The work list
 * is built once and only re-shaped per candidate.  The choice is cached in
 * the JSON file at cache_path (nullable), keyed by architecture, grid size,
 * segment-count and span-count buckets, precision and FWM form; a cached
 * entry is reused without timing. */
int32_t isrs_autotune(isrs_ctx* ctx, isrs_batch* batch, const isrs_numerics* numerics, const char* cache_path);

/* Launch shape in use on a batch: mode 0 = one block per unit, 1 = queue;
 * blocks_per_cu, sort (1 = cost-sorted), slices (of 256 point runs) per unit
 * and points_per_run (0 before the first plan: the precision's default).
 * Every output pointer is nullable. */
int32_t isrs_batch_get_tuning(const isrs_batch* batch, int32_t* mode, int32_t* blocks_per_cu, int32_t* sort,
                              int32_t* slices, int32_t* points_per_run);

/* ------------------------------------------------------------------------
 * Learned surrogate of the per-span FWM efficiency (an MLP ensemble).
 *
 * Query point (one span of one link at one (f1, f2, f)): 16 floats, of
 * which entries 0..8 hold 9 physical features scaled linearly from the
 * sampling box to [-1, 1] (entries 9..15 are ignored):
 *   f1, f2, f      absolute frequencies from the grid centre, [-5, 5] THz
 *   L              span length, [80, 100] km
 *   alpha          [0.18, 0.22] dB/km
 *   beta2, beta3   [-23, -20] ps^2/km, [0.10, 0.16] ps^3/km
 *   Cr             [0.020, 0.035] 1/(W km THz)
 *   Ptot           [17, 23] dBm (ISRS profile of Eq. 25, B_tot = 10 THz)
 * Network input: those 9 values and 7 derived in FP64 from them, with chi of
 * Eq. 24, Delta = L / ceil(L / 1 km) and |beta| = sqrt(alpha^2 + chi^2):
 * cos(chi L), sin(chi L), ln(1 + |chi| / alpha) / 8 - 1, alpha / |beta|,
 * chi / |beta|, cos(chi Delta), sin(chi Delta).
 * Target: y = ln(|mu_s|^2 / L_eff^2) of the segment closed form (Eqs. 7-10,
 * dz = 1 km).  The network learns the residual r = y - y6 over the closed
 * form without ISRS (Eq. 6); predictions are y6 + r.
 * Network per member: 16 -> 256 -> 256 -> 256 -> 256 -> 1, SiLU, BF16
 * weights and activations with FP32 accumulation on MFMA, FP32 master
 * weights and Adam.
 * ------------------------------------------------------------------------ */
typedef struct isrs_surrogate isrs_surrogate;

typedef struct {
    int32_t steps;       /* optimiser steps per member */
    int32_t batch;       /* minibatch rows, multiple of 64 */
    float lr;            /* Adam step size */
    float beta1, beta2, eps;
    int32_t member;      /* member to train, -1 = all */
} isrs_train_opts;

#define ISRS_SUR_FEATURES 16  /* padded input width */
#define ISRS_SUR_HIDDEN 256

/* Creates an ensemble of n_members (1..16) with seeded initial weights. */
int32_t isrs_surrogate_create(isrs_ctx* ctx, int32_t n_members, uint64_t seed, isrs_surrogate** out);
int32_t isrs_surrogate_destroy(isrs_surrogate* sur);

/* Draws n query points from the feature box (a channel-pair square of a
 * 100-channel, 100 GHz grid whose product f1 + f2 - f falls in a channel, a
 * uniform point of it, f uniform over the CUT's band; span parameters
 * uniform) with a counter-based generator (SplitMix64) keyed by seed, and
 * labels them with the closed form in FP64.  x_dev: device [n*16] scaled features;
 * r_dev: device [n] residual targets; y6_dev: device [n] or NULL. */
int32_t isrs_surrogate_datagen(isrs_ctx* ctx, int64_t n, uint64_t seed, float* x_dev, float* r_dev,
                               float* y6_dev);

/* As isrs_surrogate_datagen, with the query points drawn from the links of a
 * batch (the query distribution the surrogate meets in the loop): a link,
 * one of its CUTs, a pair of its active channels, a midpoint of the
 * n_grid x n_grid square lying on a live island (Eq. 16), and a span, each
 * uniform (SplitMix64 counters keyed by seed); f is the CUT centre and Ptot
 * the link's total launch power.  Outputs as for isrs_surrogate_datagen
 * (device buffers owned by the caller).  Draws outside the sampling box (or
 * from links whose B_tot is not 10 THz) are redrawn and counted in
 * n_rejected (host, nullable).  Fails with ISRS_E_ARG when 4096 draws in a
 * row are rejected, with nothing written.  The points are drawn on the host
 * and copied up; the call returns after the labels are written (it
 * synchronizes the context's stream). */
int32_t isrs_surrogate_datagen_batch(isrs_ctx* ctx, const isrs_batch* batch, int32_t n_grid, int64_t n,
                                     uint64_t seed, float* x_dev, float* r_dev, float* y6_dev, int64_t* n_rejected);

/* Adam on the mean squared error of the normalised residual
 * t = (r - shift) / scale for opts->steps minibatches per member (rows drawn
 * in order, wrapping).  shift and scale are the mean and standard deviation
 * of r_dev[0, n) at the first training call, kept for the surrogate's life
 * (and in checkpoints); the network's raw output o predicts t, and
 * predictions are shift + scale * o.  loss_out (host, nullable) receives each
 * trained member's mean loss over its last 16 steps, in units of r^2. */
int32_t isrs_surrogate_train(isrs_ctx* ctx, isrs_surrogate* sur, const float* x_dev, const float* r_dev, int64_t n,
                             const isrs_train_opts* opts, double* loss_out);

/* Ensemble prediction of the residual: mean_dev and spread_dev (max - min
 * over members, in ln units), device [n]; either may be NULL. */
int32_t isrs_surrogate_predict(isrs_ctx* ctx, isrs_surrogate* sur, const float* x_dev, int64_t n, float* mean_dev,
                               float* spread_dev);

/* y = ln(|mu|^2 / L_eff^2) for n query points: the ensemble where its
 * spread is at most spread_db_threshold (in dB of |mu|^2), the closed form
 * (FP64, Eqs. 7-10) elsewhere.  y_dev device [n]; n_fallback (host,
 * nullable) counts the closed-form points.  threshold < 0: all closed form. */
int32_t isrs_surrogate_eval_points(isrs_ctx* ctx, isrs_surrogate* sur, const float* x_dev, int64_t n,
                                   double spread_db_threshold, float* y_dev, int64_t* n_fallback);

/* Calibrates the fallback gate on n labelled query points x_dev (device
 * [n*16], e.g. from isrs_surrogate_datagen_batch): each point's error is the
 * ensemble mean against the closed form (FP64, Eqs. 7-10), in dB of
 * |mu|^2, and the spread the gate compares.  threshold_db (host) receives
 * the largest spread threshold for which every calibration point the gate
 * accepts (spread <= threshold) is within target_db of the closed form, or
 * -1 when none is (all points then fall back); max_err_db and
 * accepted_fraction (host, nullable) receive the largest accepted error and
 * the accepted share.  Synchronises the context's stream.  The ensemble's
 * spread is not an error bound by itself; this call measures the map from
 * one to the other on data of the intended query distribution. */
int32_t isrs_surrogate_calibrate(isrs_ctx* ctx, isrs_surrogate* sur, const float* x_dev, int64_t n, double target_db,
                                 double* threshold_db, double* max_err_db, double* accepted_fraction);

/* Closed form only, same query points and output as above. */
int32_t isrs_closed_form_points(isrs_ctx* ctx, const float* x_dev, int64_t n, float* y_dev);

/* Parameters of one member as FP32 host arrays in the order W1 [16x256],
 * b1 [256], W2, b2, W3, b3, W4 [256x256] each with b, w5 [256], b5 [1]
 * (row-major, input index first).  n_params = 201,985. */
int32_t isrs_surrogate_num_params(int64_t* n_params);
int32_t isrs_surrogate_get_target_scale(const isrs_surrogate* sur, double* shift, double* scale);
int32_t isrs_surrogate_get_params(isrs_surrogate* sur, int32_t member, float* params);
int32_t isrs_surrogate_set_params(isrs_ctx* ctx, isrs_surrogate* sur, int32_t member, const float* params);

/* Gradient of mean((o - t)^2) over n rows (no update), t the normalised
 * residual above, same layout as the parameters; grads host [n_params],
 * loss host (normalised units). */
int32_t isrs_surrogate_grad(isrs_ctx* ctx, isrs_surrogate* sur, int32_t member, const float* x_dev,
                            const float* r_dev, int64_t n, float* grads, double* loss);

/* eta (Eq. 11) of the context's link with the surrogate in the loop: for
 * every grid point and span, |mu_s| comes from the ensemble and the phase
 * from Eq. 6 (mu = eta_6 exp(r/2), r the predicted residual), coherently
 * summed over spans as in Eq. 22.  Where the ensemble spread exceeds
 * spread_db_threshold (dB of |mu|^2; < 0: everywhere), where a query lies
 * outside the sampling box, or when B_tot is not 10 THz, the segment closed
 * form (Eqs. 7-10) is used.  FP32 integrand, FP64 phases and sums; numerics
 * and errors as isrs_eval_eta.  eta host [n_cut]; fallback_fraction (host,
 * nullable) receives the share of live (point, span) pairs that took the
 * closed form. */
int32_t isrs_eval_eta_surrogate(isrs_ctx* ctx, isrs_surrogate* sur, const isrs_numerics* numerics,
                                const int32_t* cuts, int32_t n_cut, double spread_db_threshold, double* eta,
                                double* fallback_fraction);

/* Checkpoint: weights, Adam moments, step counters and seed. */
int32_t isrs_surrogate_save(isrs_surrogate* sur, const char* path);
int32_t isrs_surrogate_load(isrs_ctx* ctx, isrs_surrogate* sur, const char* path);

/* Pure host checks used by the set/eval calls (no device needed). */
int32_t isrs_validate_spectrum(const isrs_spectrum* spectrum);
int32_t isrs_validate_link(const isrs_span* spans, int32_t n_spans, int32_t gain_mode);
int32_t isrs_validate_numerics(const isrs_numerics* numerics);

/* Library version string. */
const char* isrs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ISRS_EGN_H */
