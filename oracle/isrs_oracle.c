/*
 * isrs_oracle.c -- plain FP64 CPU reference of the ISRS-aware EGN model.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file.  It shares no code, header,
 * table or helper with the GPU library; the two sides only receive the same
 * input arrays.
 *
 * What it computes (paper: "Acceleration and Parallelization Methods for ISRS
 * EGN Model", arXiv 2412.11614):
 *   - ISRS power profile rho_s(z, f) and SRS gain (Appendix A, Eqs. 13-14,
 *     Appendix B Eq. 25), the power-transfer figure (Eq. 12);
 *   - the FWM efficiency factor mu_s (Eq. 23) three ways:
 *       ORC_MU_INTEGRAL : the integral itself, by adaptive oscillatory
 *                         quadrature (the paper's reference method);
 *       ORC_MU_SEGMENT  : the segment closed form, Eqs. 7-10, summed term by
 *                         term exactly as written;
 *       ORC_MU_MACLAURIN: the Maclaurin closed form, Eqs. 4-6;
 *   - the link function Upsilon (Eq. 22) with the phase of Eq. 24;
 *   - per-island integrals D, E, F, G, H (Eqs. 17-21) on a midpoint grid over
 *     each channel-pair square, the island set T_kappa (Eq. 16), the NLI
 *     variance (Eq. 15) and the NLI coefficient eta (Eq. 11).
 *
 * Readings of points the paper leaves open (all documented with the design):
 *   channel k sits at (k - (n_ch-1)/2) * spacing from the grid centre; offsets
 *   and integration limits use the channel spacing, prefactors R^n use the
 *   symbol rate; |S(f)|^2 is the raised-cosine shape / Rs^2 (so Rs * int |S|^2
 *   = 1); the outer integral over f is sampled at n_f midpoints (n_f = 1: the
 *   CUT centre, sigma^2 = Rs * G(0)); each square (k1, k2) is an N x N
 *   midpoint grid over [-W/2, W/2]^2 with W = (1 + rolloff) Rs, and a point
 *   belongs to island l when |f1 + f2 - f - l*spacing| <= W/2; on an exact
 *   boundary it is shared half/half between the two islands and S takes its
 *   inside limit; amplifier gain either restores the launch profile exactly
 *   (EQUALIZED: all gain products in Eq. 22 are 1) or only the span loss
 *   (LOSS_ONLY: g_s = exp(alpha_s L_s), products taken literally).
 *
 * Units: THz, ps, km, W.  THz * ps = 1, so the phase coefficient is rad/km.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_MU_INTEGRAL 0
#define ORC_MU_SEGMENT 1
#define ORC_MU_MACLAURIN 2

#define ORC_GAIN_EQUALIZED 0
#define ORC_GAIN_LOSS_ONLY 1

#define ORC_MAX_SPANS 256
#define CC_N 16            /* Chebyshev degree per piece of the smooth envelope */
#define GL_N 64            /* Gauss-Legendre nodes for moments at small |w|     */
#define W_SMALL 20.0       /* below this |w| the moments use Gauss-Legendre     */
#define MAX_PIECES 256
#define TIE_EPS 1e-9       /* island-boundary tie tolerance, in grid steps      */

/* Inputs, laid out exactly like the Python-side arrays. */
typedef struct {
    double length, alpha_db, beta2, beta3, gamma, cr;
} orc_span;

typedef struct {
    int n_ch;
    double spacing, rs, rolloff;
    const double *power, *phi, *psi;
} orc_spectrum;

typedef struct {
    int n_grid, n_f;
    double dz;
    int egn, mu_method, gain_mode;
    double ptot_override;
} orc_numerics;

/* ------------------------------------------------------------------------ */
/* Basic physics                                                             */
/* ------------------------------------------------------------------------ */

/* dB/km -> 1/km: power attenuation alpha = alpha_dB / (10 log10 e). */
double orc_alpha_lin(double alpha_db) { return alpha_db / (10.0 / log(10.0)); }

/* Effective length L_eff(z) = (1 - exp(-alpha z)) / alpha (Eqs. 1, 13). */
double orc_leff(double alpha, double z) { return -expm1(-alpha * z) / alpha; }

/* SRS gain, Eq. 14, written with X = B Ptot Cr L_eff(z):
 *   SRS_G = X exp(-X f / B) / (2 sinh(X / 2)),  and 1 at X = 0. */
double orc_srs_gain(double X, double f, double B)
{
    if (X == 0.0) return 1.0;
    return X * exp(-X * f / B) / (2.0 * sinh(0.5 * X));
}

/* Normalised power profile rho(z, f), Eqs. 13 / 25. */
double orc_rho(double alpha, double cr, double ptot, double B, double z, double f)
{
    double X = B * ptot * cr * orc_leff(alpha, z);
    return orc_srs_gain(X, f, B) * exp(-alpha * z);
}

/* Power transfer between the outermost channels, Eq. 12, in dB
 * (the factor 4.3 read as 10 log10 e). */
double orc_delta_rho_db(double ptot, double cr, double alpha, double L, double B)
{
    return 10.0 / log(10.0) * ptot * cr * orc_leff(alpha, L) * B;
}

/* Phase coefficient of Eq. 24 / Eq. 5 (rad/km) for absolute frequencies
 * a = f1, b = f2, c = f measured from the grid centre. */
static double phase_coef(double beta2, double beta3, double a, double b, double c)
{
    double d12 = (a - c) * (b - c);   /* formed first: symmetric in a <-> b */
    return 4.0 * M_PI * M_PI * d12 * (beta2 + M_PI * beta3 * (a + b));
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1, 1] (Newton on P_n from Chebyshev guesses).    */
/* ------------------------------------------------------------------------ */
static double gl_x[GL_N], gl_w[GL_N];
static int gl_ready = 0;

static double legendre_pair(double x, double* pnm1)
{
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= GL_N; k++) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    *pnm1 = p0;
    return p1;
}

static void gl_init(void)
{
    if (gl_ready) return;
    for (int i = 0; i < GL_N; i++) {
        double x = cos(M_PI * (i + 0.75) / (GL_N + 0.5)), pn, pm, dp;
        for (int it = 0; it < 100; it++) {
            pn = legendre_pair(x, &pm);
            dp = GL_N * (x * pn - pm) / (x * x - 1.0);
            double dx = pn / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        pn = legendre_pair(x, &pm);
        dp = GL_N * (x * pn - pm) / (x * x - 1.0);
        gl_x[i] = x;
        gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    gl_ready = 1;
}

void orc_gl_rule(double* x, double* w)
{
    gl_init();
    memcpy(x, gl_x, sizeof gl_x);
    memcpy(w, gl_w, sizeof gl_w);
}

/* ------------------------------------------------------------------------ */
/* Modified Chebyshev moments  M_k(w) = int_{-1}^{1} T_k(t) exp(w t) dt      */
/* ------------------------------------------------------------------------ */

/* Gauss-Legendre evaluation: accurate for |w| <= W_SMALL (and well beyond). */
static void moments_gl(cplx w, int n, cplx* M)
{
    gl_init();
    for (int k = 0; k <= n; k++) M[k] = 0;
    for (int q = 0; q < GL_N; q++) {
        double t = gl_x[q];
        cplx e = gl_w[q] * cexp(w * t);
        double T0 = 1.0, T1 = t;
        M[0] += e * T0;
        if (n >= 1) M[1] += e * T1;
        for (int k = 2; k <= n; k++) {
            double T2 = 2.0 * t * T1 - T0;
            M[k] += e * T2;
            T0 = T1;
            T1 = T2;
        }
    }
}

/* Forward recurrence from integration by parts, stable for k < |w|:
 *   M_0 = (E+ - E-) / w,  M_1 = (E+ + E-) / w - M_0 / w,
 *   M_2 = 2 (E+ - E-) / w - 4 M_1 / w - M_0,
 *   M_{k+1} = -2 D_k / (w (k-1)) - 2 (k+1) M_k / w + (k+1)/(k-1) M_{k-1},
 * with E+- = exp(+-w) and D_k = E+ - (-1)^(k+1) E-.  It follows from
 * 2 T_k = T'_{k+1}/(k+1) - T'_{k-1}/(k-1) and
 * int T'_m exp(w t) = T_m exp(w t) |_{-1}^{1} - w M_m. */
static void moments_rec(cplx w, int n, cplx* M)
{
    cplx ep = cexp(w), em = cexp(-w);
    M[0] = (ep - em) / w;
    if (n >= 1) M[1] = (ep + em) / w - M[0] / w;
    if (n >= 2) M[2] = 2.0 * (ep - em) / w - 4.0 * M[1] / w - M[0];
    for (int k = 2; k < n; k++) {
        cplx Dk = (k % 2 == 1) ? (ep - em) : (ep + em);   /* (-1)^(k+1) */
        M[k + 1] = -2.0 * Dk / (w * (double)(k - 1)) - 2.0 * (k + 1) * M[k] / w
                   + ((double)(k + 1) / (double)(k - 1)) * M[k - 1];
    }
}

void orc_moments(double wre, double wim, int n, int method, double* out /* [2(n+1)] */)
{
    cplx M[64];
    cplx w = wre + I * wim;
    if (n > 63) n = 63;
    if (method == 0) moments_gl(w, n, M); else moments_rec(w, n, M);
    for (int k = 0; k <= n; k++) { out[2 * k] = creal(M[k]); out[2 * k + 1] = cimag(M[k]); }
}

static void moments(cplx w, int n, cplx* M)
{
    if (cabs(w) <= W_SMALL) moments_gl(w, n, M);
    else moments_rec(w, n, M);
}

/* ------------------------------------------------------------------------ */
/* Adaptive Chebyshev envelope of the smooth factor of the mu integrand.    */
/* The integrand of Eq. 23 is SRS_G(z, x) * exp((i chi - alpha) z) (Eq. 1).  */
/* SRS_G does not oscillate; it is interpolated piecewise at Chebyshev-      */
/* Lobatto points, with bisection until the last two coefficients vanish     */
/* to 1e-13 of the largest.  Each piece times exp(beta z) is then integrated */
/* exactly through the moments above, so the cost does not grow with chi.    */
/* ------------------------------------------------------------------------ */
typedef struct {
    double zc, hw;
    double c[CC_N + 1];
} cc_piece;

typedef struct {
    int n;
    cc_piece p[MAX_PIECES];
} envelope;

typedef struct {
    double alpha, cr, ptot, B, x;
} env_fn;

static double env_eval(const env_fn* e, double z)
{
    double X = e->B * e->ptot * e->cr * orc_leff(e->alpha, z);
    return orc_srs_gain(X, e->x, e->B);
}

static double cc_cos[CC_N + 1][CC_N + 1];   /* cos(pi j k / CC_N) */
static int cc_ready = 0;

static void cc_init(void)
{
    if (cc_ready) return;
    for (int j = 0; j <= CC_N; j++)
        for (int k = 0; k <= CC_N; k++) cc_cos[j][k] = cos(M_PI * (double)((j * k) % (2 * CC_N)) / CC_N);
    cc_ready = 1;
}

static void cheb_coeffs(const env_fn* e, double zc, double hw, double* c)
{
    double v[CC_N + 1];
    for (int j = 0; j <= CC_N; j++) v[j] = env_eval(e, zc + hw * cc_cos[j][1]);
    for (int k = 0; k <= CC_N; k++) {
        double s = 0.0;
        for (int j = 0; j <= CC_N; j++) {
            double t = v[j] * cc_cos[j][k];
            if (j == 0 || j == CC_N) t *= 0.5;
            s += t;
        }
        s *= 2.0 / CC_N;
        if (k == 0 || k == CC_N) s *= 0.5;
        c[k] = s;
    }
}

static void envelope_add(envelope* env, const env_fn* e, double z0, double z1, int depth)
{
    double zc = 0.5 * (z0 + z1), hw = 0.5 * (z1 - z0);
    double c[CC_N + 1];
    cheb_coeffs(e, zc, hw, c);
    double big = 0.0;
    for (int k = 0; k <= CC_N; k++) big = fmax(big, fabs(c[k]));
    double tail = fabs(c[CC_N - 1]) + fabs(c[CC_N]);
    if (tail > 1e-13 * big && depth < 20 && env->n + 2 <= MAX_PIECES) {
        envelope_add(env, e, z0, zc, depth + 1);
        envelope_add(env, e, zc, z1, depth + 1);
        return;
    }
    cc_piece* p = &env->p[env->n++];
    p->zc = zc;
    p->hw = hw;
    memcpy(p->c, c, sizeof c);
}

static void envelope_build(envelope* env, double alpha, double cr, double ptot, double B,
                           double x, double L)
{
    env_fn e = {alpha, cr, ptot, B, x};
    env->n = 0;
    envelope_add(env, &e, 0.0, L, 0);
}

/* int_0^L SRS_G(z, x) exp(beta z) dz over the envelope's pieces. */
static cplx envelope_integrate(const envelope* env, cplx beta)
{
    cplx total = 0;
    cplx M[CC_N + 1];
    for (int q = 0; q < env->n; q++) {
        const cc_piece* p = &env->p[q];
        moments(beta * p->hw, CC_N, M);
        cplx s = 0;
        for (int k = 0; k <= CC_N; k++) s += p->c[k] * M[k];
        total += p->hw * cexp(beta * p->zc) * s;
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* FWM efficiency factor mu_s(f1, f2, f)                                    */
/* ------------------------------------------------------------------------ */

/* Segment closed form, Eqs. 8-10, term by term. */
static cplx mu_segment(double alpha, double cr, double ptot, double B, double L, double dz,
                       double x, double chi)
{
    int K = (int)ceil(L / dz);
    if (K < 1) K = 1;
    cplx beta = -alpha + I * chi;
    cplx sum = 0;
    for (int k = 0; k < K; k++) {
        double zk = (k + 0.5) / K * L;                       /* Eq. 10 */
        double X = B * ptot * cr * orc_leff(alpha, zk);
        double g = orc_srs_gain(X, x, B);                    /* SRS gain at z_k, Eq. 8 */
        cplx Ik = (cexp(beta * ((k + 1.0) / K * L)) - cexp(beta * ((double)k / K * L))) / beta; /* Eq. 9 */
        sum += g * Ik;
    }
    return sum;
}

/* Maclaurin closed form, Eqs. 4-6. */
static cplx mu_maclaurin(double alpha, double cr, double ptot, double L, double x, double chi)
{
    cplx b1 = I * chi - alpha, b2 = I * chi - 2.0 * alpha;
    cplx eta = (cexp(b1 * L) - 1.0) / b1;                    /* Eq. 6 */
    return eta - ptot * cr * x / alpha * (eta - (cexp(b2 * L) - 1.0) / b2);   /* Eq. 4 */
}

/* mu for one span at absolute frequencies (a, b, c); env may be NULL. */
static cplx mu_span(const orc_span* s, double ptot, double B, int method, double dz,
                    double a, double b, double c, const envelope* env)
{
    double alpha = orc_alpha_lin(s->alpha_db);
    double chi = phase_coef(s->beta2, s->beta3, a, b, c);
    double x = a + b - c;
    if (method == ORC_MU_SEGMENT) return mu_segment(alpha, s->cr, ptot, B, s->length, dz, x, chi);
    if (method == ORC_MU_MACLAURIN) return mu_maclaurin(alpha, s->cr, ptot, s->length, x, chi);
    envelope local;
    if (!env) {
        envelope_build(&local, alpha, s->cr, ptot, B, x, s->length);
        env = &local;
    }
    return envelope_integrate(env, -alpha + I * chi);
}

void orc_mu(const orc_span* s, double ptot, double B, int method, double dz, double a, double b,
            double c, double* out)
{
    gl_init();
    cc_init();
    cplx m = mu_span(s, ptot, B, method, dz, a, b, c, NULL);
    out[0] = creal(m);
    out[1] = cimag(m);
}

/* Link function Upsilon, Eq. 22. */
static cplx upsilon(const orc_span* sp, int n_sp, double ptot, double B, int method, double dz,
                    int gain_mode, double a, double b, double c, envelope* const* envs)
{
    cplx ups = 0;
    double theta_lin = 0.0;   /* sum_{s'<s} (beta2 L + pi (a+b) beta3 L) */
    for (int s = 0; s < n_sp; s++) {
        cplx mu = mu_span(&sp[s], ptot, B, method, dz, a, b, c, envs ? envs[s] : NULL);
        double theta = 4.0 * M_PI * M_PI * ((a - c) * (b - c)) * theta_lin;
        double gain = 1.0;
        if (gain_mode == ORC_GAIN_LOSS_ONLY) {
            for (int q = 0; q < s; q++) {
                double al = orc_alpha_lin(sp[q].alpha_db), L = sp[q].length;
                double g = exp(al * L);
                gain *= pow(g, 1.5) * sqrt((orc_rho(al, sp[q].cr, ptot, B, L, a)
                                            * orc_rho(al, sp[q].cr, ptot, B, L, b))
                                           * orc_rho(al, sp[q].cr, ptot, B, L, a + b - c));
            }
            for (int q = s; q < n_sp; q++) {
                double al = orc_alpha_lin(sp[q].alpha_db), L = sp[q].length;
                double g = exp(al * L);
                gain *= sqrt(g) * sqrt(orc_rho(al, sp[q].cr, ptot, B, L, c));
            }
        }
        ups += sp[s].gamma * mu * cexp(I * theta) * gain;
        theta_lin += sp[s].beta2 * sp[s].length + M_PI * (a + b) * sp[s].beta3 * sp[s].length;
    }
    return ups;
}

void orc_upsilon(const orc_span* sp, int n_sp, double ptot, double B, int method, double dz,
                 int gain_mode, double a, double b, double c, double* out)
{
    gl_init();
    cc_init();
    cplx u = upsilon(sp, n_sp, ptot, B, method, dz, gain_mode, a, b, c, NULL);
    out[0] = creal(u);
    out[1] = cimag(u);
}

/* ------------------------------------------------------------------------ */
/* Channel spectrum                                                          */
/* ------------------------------------------------------------------------ */

/* Raised-cosine PSD shape, 1 in the flat part, integral = Rs. */
static double rc_shape(double x, double rs, double ro)
{
    double ax = fabs(x);
    double lo = 0.5 * (1.0 - ro) * rs, hi = 0.5 * (1.0 + ro) * rs;
    if (ax <= lo) return 1.0;
    if (ax > hi) return 0.0;
    return 0.5 * (1.0 + cos(M_PI * (ax - lo) / (ro * rs)));
}

/* Field spectrum S(x) = sqrt(shape) / Rs, so Rs * int |S|^2 = 1. */
static double S_of(double x, double rs, double ro) { return sqrt(rc_shape(x, rs, ro)) / rs; }

/* Limit of S from inside the support (used on island-boundary ties). */
static double S_inside(double x, double rs, double ro)
{
    if (ro == 0.0) return 1.0 / rs;
    return S_of(x, rs, ro);
}

double orc_S(double x, double rs, double ro) { return S_of(x, rs, ro); }

/* ------------------------------------------------------------------------ */
/* Island integrals of one channel-pair square                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_spectrum* sp;
    const orc_span* spans;
    int n_sp;
    const orc_numerics* nu;
    double ptot, B;
} model;

static double model_ptot(const orc_spectrum* sp, const orc_numerics* nu)
{
    if (nu->ptot_override > 0.0) return nu->ptot_override;
    double p = 0.0;
    for (int k = 0; k < sp->n_ch; k++) p += sp->power[k];
    return p;
}

static double nu_ch(const orc_spectrum* sp, int k) { return (k - 0.5 * (sp->n_ch - 1)) * sp->spacing; }

/* Island membership (Eq. 16 with the grid reading): on the anti-diagonal
 * f1 + f2 = (m + 1 - N) h of an N x N square, island l holds the points with
 * |f3| <= W/2, f3 = f1 + f2 - f - l * spacing.  wt[l+1] = 1 inside, 1/2 on an
 * exact boundary (the cell is split between two islands), 0 outside; S3 is
 * S(f3) (its inside limit on a boundary).  Returns 1 if any island has a
 * nonzero contribution. */
static int antidiag_islands(const orc_spectrum* sp, int N, const int* valid, int m, double f,
                            double* wt, double* S3)
{
    const double rs = sp->rs, ro = sp->rolloff, W = (1.0 + ro) * rs, h = W / N;
    const double r = sp->spacing / h;
    int sidx = m + 1 - N, any = 0;
    for (int l = -1; l <= 1; l++) {
        wt[l + 1] = 0.0;
        S3[l + 1] = 0.0;
        if (!valid[l + 1]) continue;
        double u = (double)sidx - f / h - l * r;       /* f3 / h */
        double au = fabs(u), half = 0.5 * N;
        if (au < half - TIE_EPS) {
            wt[l + 1] = 1.0;
            S3[l + 1] = S_of(u * h, rs, ro);
        } else if (au <= half + TIE_EPS) {
            wt[l + 1] = 0.5;
            S3[l + 1] = S_inside(u * h, rs, ro);
        }
        if (wt[l + 1] > 0.0 && S3[l + 1] != 0.0) any = 1;
    }
    return any;
}

static void square_valid(const orc_spectrum* sp, int cut, int k1, int k2, int* valid)
{
    for (int l = -1; l <= 1; l++) {
        int k3 = k1 + k2 - cut + l;
        valid[l + 1] = (k3 >= 0 && k3 < sp->n_ch && sp->power[k3] > 0.0);
    }
}

/* Largest |(f1 - f)(f2 - f)| over the grid points of all islands of CUT
 * `cut` at f = 0 (absolute frequencies), for the domain-geometry check. */
double orc_domain_max_d1d2(const orc_spectrum* sp, int n_grid, int cut)
{
    const int N = n_grid;
    const double W = (1.0 + sp->rolloff) * sp->rs, h = W / N;
    double best = 0.0;
    for (int k1 = 0; k1 < sp->n_ch; k1++)
        for (int k2 = 0; k2 < sp->n_ch; k2++) {
            if (!(sp->power[k1] > 0 && sp->power[k2] > 0)) continue;
            int valid[3];
            square_valid(sp, cut, k1, k2, valid);
            for (int m = 0; m <= 2 * N - 2; m++) {
                double wt[3], S3[3];
                if (!antidiag_islands(sp, N, valid, m, 0.0, wt, S3)) continue;
                int i0 = m - (N - 1) > 0 ? m - (N - 1) : 0;
                int i1 = m < N - 1 ? m : N - 1;
                for (int i = i0; i <= i1; i++) {
                    int j = m - i;
                    double d1 = nu_ch(sp, k1) + (-0.5 * W + (i + 0.5) * h) - nu_ch(sp, cut);
                    double d2 = nu_ch(sp, k2) + (-0.5 * W + (j + 0.5) * h) - nu_ch(sp, cut);
                    best = fmax(best, fabs(d1 * d2));
                }
            }
        }
    return best;
}

double orc_phase_coef(double beta2, double beta3, double a, double b, double c)
{
    return phase_coef(beta2, beta3, a, b, c);
}

/* Bare integrals of the three islands l = -1, 0, 1 of square (k1, k2) for CUT
 * `cut` at outer frequency f:  out[(l+1)*5 + t], t = D, E, F, G, H with
 *   D = sum_pts  w |S1|^2 |S2|^2 |S3|^2 |Ups|^2                      (Eq. 17)
 *   E = sum_f2   h |S2|^2 | sum_f1 w S1 S3 Ups |^2                   (Eq. 18)
 *   F = sum_f1   h |S1|^2 | sum_f2 w S2 S3 Ups |^2                   (Eq. 19)
 *   G = sum_nu   w |S3|^2 | sum_{f1+f2=nu} h S1 S2 Ups |^2           (Eq. 20)
 *   H = | sum_pts w S1 S2 S3 Ups |^2                                  (Eq. 21)
 * (second inner integrals of Eqs. 18-21 are the conjugates of the first; S is
 * real).  Without the R^n prefactors, the 16/27 ... constants, powers and
 * format factors.  Islands whose third channel is outside the grid or
 * inactive stay zero. */
static void square_terms(const model* md, int cut, int k1, int k2, double f, double* out)
{
    const orc_spectrum* sp = md->sp;
    const int N = md->nu->n_grid;
    const double rs = sp->rs, ro = sp->rolloff, W = (1.0 + ro) * rs, h = W / N;
    const int n_sp = md->n_sp;
    const int method = md->nu->mu_method;

    memset(out, 0, 15 * sizeof(double));
    int valid[3];
    square_valid(sp, cut, k1, k2, valid);
    if (!valid[0] && !valid[1] && !valid[2]) return;

    cplx* rows = calloc(3 * N, sizeof(cplx));
    cplx* cols = calloc(3 * N, sizeof(cplx));
    cplx* adsum = calloc(3 * (2 * N - 1), sizeof(cplx));
    double* adw = calloc(3 * (2 * N - 1), sizeof(double));
    double* ads3 = calloc(3 * (2 * N - 1), sizeof(double));
    cplx hsum[3] = {0, 0, 0};
    double* Sg = malloc(N * sizeof(double));
    for (int i = 0; i < N; i++) Sg[i] = S_of(-0.5 * W + (i + 0.5) * h, rs, ro);

    envelope** envs = NULL;
    if (method == ORC_MU_INTEGRAL) {
        envs = malloc(n_sp * sizeof(envelope*));
        for (int s = 0; s < n_sp; s++) envs[s] = malloc(sizeof(envelope));
    }

    const double c = nu_ch(sp, cut) + f;
    for (int m = 0; m <= 2 * N - 2; m++) {
        double wt[3], S3[3];
        if (!antidiag_islands(sp, N, valid, m, f, wt, S3)) continue;
        int sidx = m + 1 - N;
        double x = nu_ch(sp, k1) + nu_ch(sp, k2) - nu_ch(sp, cut) + sidx * h - f;  /* a + b - c */
        if (envs)
            for (int s = 0; s < n_sp; s++)
                envelope_build(envs[s], orc_alpha_lin(md->spans[s].alpha_db), md->spans[s].cr,
                               md->ptot, md->B, x, md->spans[s].length);
        int i0 = m - (N - 1) > 0 ? m - (N - 1) : 0;
        int i1 = m < N - 1 ? m : N - 1;
        for (int i = i0; i <= i1; i++) {
            int j = m - i;
            double f1 = -0.5 * W + (i + 0.5) * h, f2 = -0.5 * W + (j + 0.5) * h;
            double a = nu_ch(sp, k1) + f1, b = nu_ch(sp, k2) + f2;
            cplx ups = upsilon(md->spans, n_sp, md->ptot, md->B, method, md->nu->dz,
                               md->nu->gain_mode, a, b, c, envs);
            double S1 = Sg[i], S2 = Sg[j];
            for (int l = 0; l < 3; l++) {
                if (wt[l] == 0.0) continue;
                double w = wt[l];
                double u2 = creal(ups) * creal(ups) + cimag(ups) * cimag(ups);
                out[l * 5 + 0] += h * h * w * S1 * S1 * S2 * S2 * S3[l] * S3[l] * u2;
                rows[l * N + j] += h * w * S1 * S3[l] * ups;
                cols[l * N + i] += h * w * S2 * S3[l] * ups;
                adsum[l * (2 * N - 1) + m] += h * S1 * S2 * ups;
                hsum[l] += h * h * w * S1 * S2 * S3[l] * ups;
            }
        }
        for (int l = 0; l < 3; l++) {
            adw[l * (2 * N - 1) + m] = wt[l];
            ads3[l * (2 * N - 1) + m] = S3[l];
        }
    }
    for (int l = 0; l < 3; l++) {
        double E = 0, F = 0, G = 0;
        for (int j = 0; j < N; j++) {
            cplx v = rows[l * N + j];
            E += h * Sg[j] * Sg[j] * (creal(v) * creal(v) + cimag(v) * cimag(v));
        }
        for (int i = 0; i < N; i++) {
            cplx v = cols[l * N + i];
            F += h * Sg[i] * Sg[i] * (creal(v) * creal(v) + cimag(v) * cimag(v));
        }
        for (int m = 0; m <= 2 * N - 2; m++) {
            cplx v = adsum[l * (2 * N - 1) + m];
            double s3 = ads3[l * (2 * N - 1) + m];
            G += h * adw[l * (2 * N - 1) + m] * s3 * s3 * (creal(v) * creal(v) + cimag(v) * cimag(v));
        }
        out[l * 5 + 1] = E;
        out[l * 5 + 2] = F;
        out[l * 5 + 3] = G;
        out[l * 5 + 4] = creal(hsum[l]) * creal(hsum[l]) + cimag(hsum[l]) * cimag(hsum[l]);
    }
    if (envs) {
        for (int s = 0; s < n_sp; s++) free(envs[s]);
        free(envs);
    }
    free(Sg);
    free(rows);
    free(cols);
    free(adsum);
    free(adw);
    free(ads3);
}

static int check_inputs(const orc_spectrum* sp, const orc_span* spans, int n_sp, const orc_numerics* nu)
{
    if (!sp || !spans || !nu) return -1;
    if (sp->n_ch < 1 || n_sp < 1 || n_sp > ORC_MAX_SPANS || nu->n_grid < 1 || nu->n_f < 1) return -1;
    if (!(sp->rs > 0) || !(sp->spacing > 0) || sp->rolloff < 0 || sp->rolloff > 1) return -1;
    if ((1.0 + sp->rolloff) * sp->rs > sp->spacing * (1.0 + 1e-12)) return -1;
    if (!(nu->dz > 0)) return -1;
    for (int s = 0; s < n_sp; s++)
        if (!(spans[s].length > 0) || !(spans[s].alpha_db > 0) || spans[s].cr < 0) return -1;
    return 0;
}

int orc_square_terms(const orc_spectrum* sp, const orc_span* spans, int n_sp,
                     const orc_numerics* nu, int cut, int k1, int k2, double f, double* out)
{
    if (check_inputs(sp, spans, n_sp, nu)) return -1;
    model md = {sp, spans, n_sp, nu, model_ptot(sp, nu), sp->n_ch * sp->spacing};
    gl_init();
    cc_init();
    square_terms(&md, cut, k1, k2, f, out);
    return 0;
}

/* sigma^2, eta, the five summed contributions and the PSD samples of one CUT,
 * Eqs. 15, 16 and 11.  Squares are evaluated in parallel; their results are
 * stored and summed in a fixed order, so the answer does not depend on the
 * thread count. */
int orc_eval_cut(const orc_spectrum* sp, const orc_span* spans, int n_sp, const orc_numerics* nu,
                 int cut, double* sigma2, double* eta, double* terms5, double* psd)
{
    if (check_inputs(sp, spans, n_sp, nu)) return -1;
    if (cut < 0 || cut >= sp->n_ch || !(sp->power[cut] > 0)) return -1;
    gl_init();
    cc_init();
    model md = {sp, spans, n_sp, nu, model_ptot(sp, nu), sp->n_ch * sp->spacing};
    const int nc = sp->n_ch;
    const double R = sp->rs;
    const double cD = 16.0 / 27.0, cE = 16.0 / 27.0, cF = 32.0 / 81.0, cG = 16.0 / 81.0, cH = 16.0 / 81.0;
    double tot[5] = {0, 0, 0, 0, 0};
    double s2 = 0.0;
    double* sq = malloc((size_t)nc * nc * 15 * sizeof(double));
    for (int n = 0; n < nu->n_f; n++) {
        double f = (nu->n_f == 1) ? 0.0 : -0.5 * R + (n + 0.5) * R / nu->n_f;
#pragma omp parallel for schedule(dynamic, 1)
        for (int q = 0; q < nc * nc; q++) {
            int k1 = q / nc, k2 = q % nc;
            double* o = sq + (size_t)q * 15;
            if (sp->power[k1] > 0 && sp->power[k2] > 0) square_terms(&md, cut, k1, k2, f, o);
            else memset(o, 0, 15 * sizeof(double));
        }
        double Gf = 0.0;
        double tf[5] = {0, 0, 0, 0, 0};
        for (int q = 0; q < nc * nc; q++) {
            int k1 = q / nc, k2 = q % nc;
            if (!(sp->power[k1] > 0 && sp->power[k2] > 0)) continue;
            for (int l = -1; l <= 1; l++) {
                int k3 = k1 + k2 - cut + l;
                if (k3 < 0 || k3 >= nc || !(sp->power[k3] > 0)) continue;
                const double* o = sq + (size_t)q * 15 + (l + 1) * 5;
                double P = sp->power[k1] * sp->power[k2] * sp->power[k3];
                double t[5];
                t[0] = cD * R * R * R * o[0];
                t[1] = (nu->egn && k3 == k1) ? sp->phi[k1] * cE * R * R * o[1] : 0.0;
                t[2] = (nu->egn && k3 == k2) ? sp->phi[k2] * cF * R * R * o[2] : 0.0;
                t[3] = (nu->egn && k1 == k2) ? sp->phi[k1] * cG * R * R * o[3] : 0.0;
                t[4] = (nu->egn && k1 == k2 && k3 == k2) ? sp->psi[k1] * cH * R * o[4] : 0.0;
                for (int u = 0; u < 5; u++) {
                    tf[u] += P * t[u];
                    Gf += P * t[u];
                }
            }
        }
        double wf = (nu->n_f == 1) ? R : R / nu->n_f;
        if (psd) psd[n] = Gf;
        s2 += wf * Gf;
        for (int u = 0; u < 5; u++) tot[u] += wf * tf[u];
    }
    free(sq);
    if (sigma2) *sigma2 = s2;
    if (eta) *eta = s2 / (sp->power[cut] * sp->power[cut] * sp->power[cut]);
    if (terms5) for (int u = 0; u < 5; u++) terms5[u] = tot[u];
    return 0;
}

/* Format constants from constellation points: Phi = mu4/mu2^2 - 2,
 * Psi = mu6/mu2^3 - 9 mu4/mu2^2 + 12 (EGN model). */
void orc_format_constants(const double* re, const double* im, int n, double* phi, double* psi)
{
    double m2 = 0, m4 = 0, m6 = 0;
    for (int k = 0; k < n; k++) {
        double p = re[k] * re[k] + im[k] * im[k];
        m2 += p;
        m4 += p * p;
        m6 += p * p * p;
    }
    m2 /= n;
    m4 /= n;
    m6 /= n;
    *phi = m4 / (m2 * m2) - 2.0;
    *psi = m6 / (m2 * m2 * m2) - 9.0 * m4 / (m2 * m2) + 12.0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
