/*
 * sfq_oracle.c -- plain, slow CPU oracle for the strong-field QED Monte Carlo step
 * (Montefiori & Tamburini, "SFQEDtoolkit", arXiv:2301.07684).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls this file;
 * only the test-suite, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no code, header, table or constant generator with the GPU library.
 *
 * Everything is computed from the plain definitions in double precision (the chi radicand in
 * long double):
 *   - K_nu(x)  = int_0^inf exp(-x cosh t) cosh(nu t) dt                     (textbook integral rep.)
 *   - Ki_nu(x) = int_x^inf K_nu(y) dy = int_0^inf exp(-x cosh t) cosh(nu t)/cosh t dt
 *   - rates      : paper Sec. 4.1 Eq. (wtilde) and Sec. 4.2 Eq. (wtilde_pair), by adaptive quadrature
 *   - spectra/CDF: paper Sec. 4.3 Eq. (pe_eff_int_2) and Sec. 4.4 Eq. (tilde_I_pp)
 *   - sampling   : inverse transform sampling, paper Sec. 4.3 Eq. (ITS_base)/(again) and
 *                  Sec. 4.4 Eq. (again_pp), solved by Brent's root finder
 *   - decisions  : optical-depth method (paper Sec. 2, Eq. (any_event)) or local method (Sec. 2)
 *   - beyond-LCFA: paper Sec. 5, Eqs. (fl)-(condit), (gammaLCFA), (rej_cond)
 *   - the momentum push of the PIC cycle the step sits in (paper Fig. 7): the Boris scheme,
 *     in long double (the paper names no pusher; see orc_boris_push)
 *   - Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11), written from
 *     the published round definition.
 * No tabulation, no caching across calls, no approximation scheme of its own.
 *
 * Adaptive quadrature: Gauss-Legendre rule of order ORC_GL_N whose nodes are computed at first
 * use by Newton iteration on the Legendre three-term recurrence; an interval is accepted when
 * the rule on the whole interval and the sum of the rule on its two halves agree to the
 * requested tolerance.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------------------------------ */
/* Physical constants (CODATA 2018): fine-structure constant and reduced Compton wavelength.  */
/* ------------------------------------------------------------------------------------------ */
double orc_alpha(void) { return 7.2973525693e-3; }
double orc_lambda_compton(void) { return 3.8615926796e-13; } /* metres, hbar/(m_e c) */
double orc_speed_of_light(void) { return 299792458.0; }

/* ------------------------------------------------------------------------------------------ */
/* Gauss-Legendre nodes by Newton iteration on P_n (three-term recurrence).                  */
/* ------------------------------------------------------------------------------------------ */
#define ORC_GL_N 12
static double gl_x[ORC_GL_N], gl_w[ORC_GL_N];
static int gl_ready = 0;

static void gl_init(void)
{
    if (gl_ready) return;
#pragma omp critical(orc_gl_init)
    {
        if (!gl_ready) {
            const int n = ORC_GL_N;
            for (int i = 0; i < n; ++i) {
                double x = cos(ORC_PI * (i + 0.75) / (n + 0.5)); /* standard starting guess */
                double dp = 0.0;
                for (int it = 0; it < 100; ++it) {
                    double p0 = 1.0, p1 = x;
                    for (int k = 2; k <= n; ++k) {
                        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                        p0 = p1;
                        p1 = p2;
                    }
                    /* p1 = P_n(x), p0 = P_{n-1}(x); derivative from the standard identity */
                    dp = n * (x * p1 - p0) / (x * x - 1.0);
                    double dx = p1 / dp;
                    x -= dx;
                    if (fabs(dx) < 1e-17) break;
                }
                gl_x[i] = x;
                gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
            }
            gl_ready = 1;
        }
    }
}

/* Public accessors so the test-suite can pin the rule itself (exactness on monomials). */
int orc_gl_order(void) { return ORC_GL_N; }
void orc_gl_rule(double* x, double* w)
{
    gl_init();
    for (int i = 0; i < ORC_GL_N; ++i) { x[i] = gl_x[i]; w[i] = gl_w[i]; }
}

typedef double (*orc_fn)(double t, const void* ctx);

static double gl_apply(orc_fn f, const void* ctx, double a, double b)
{
    double c = 0.5 * (a + b), h = 0.5 * (b - a), s = 0.0;
    for (int i = 0; i < ORC_GL_N; ++i) s += gl_w[i] * f(c + h * gl_x[i], ctx);
    return s * h;
}

/* Globally adaptive integration over [a,b]: the interval list starts from `pieces` equal
 * sub-intervals; each interval carries the rule on its two halves (the value used) and the
 * difference from the rule on the whole interval (the error estimate of the coarser rule, so
 * an upper bound for the error of the value used).  The interval with the largest estimate is
 * bisected until the summed estimate is below rel * sum|values| or ORC_MAX_IV intervals exist. */
#define ORC_MAX_IV 600
typedef struct { double a, b, l, r, err; } orc_iv;

static void iv_fill(orc_fn f, const void* ctx, orc_iv* v, double a, double b, double whole)
{
    double m = 0.5 * (a + b);
    v->a = a; v->b = b;
    v->l = gl_apply(f, ctx, a, m);
    v->r = gl_apply(f, ctx, m, b);
    v->err = fabs(v->l + v->r - whole);
}

static double integrate(orc_fn f, const void* ctx, double a, double b, double rel, int pieces)
{
    gl_init();
    if (!(b > a)) return 0.0;
    orc_iv iv[ORC_MAX_IV];
    if (pieces > ORC_MAX_IV / 4) pieces = ORC_MAX_IV / 4;
    int n = 0;
    double h = (b - a) / pieces;
    for (int k = 0; k < pieces; ++k) {
        double lo = a + k * h, hi = (k == pieces - 1) ? b : a + (k + 1) * h;
        iv_fill(f, ctx, &iv[n++], lo, hi, gl_apply(f, ctx, lo, hi));
    }
    for (;;) {
        double err = 0.0, mag = 0.0, emax = -1.0;
        int imax = 0;
        for (int i = 0; i < n; ++i) {
            err += iv[i].err;
            mag += fabs(iv[i].l) + fabs(iv[i].r);
            if (iv[i].err > emax) { emax = iv[i].err; imax = i; }
        }
        if (err <= rel * mag || n >= ORC_MAX_IV) break;
        orc_iv p = iv[imax];
        double m = 0.5 * (p.a + p.b);
        if (!(m > p.a && m < p.b)) break;
        iv_fill(f, ctx, &iv[imax], p.a, m, p.l);
        iv_fill(f, ctx, &iv[n++], m, p.b, p.r);
    }
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += iv[i].l + iv[i].r;
    return s;
}

/* ------------------------------------------------------------------------------------------ */
/* Modified Bessel functions of the second kind and their tail integrals, exponentially       */
/* scaled: Ks(nu,x) = e^x K_nu(x), Kis(nu,x) = e^x int_x^inf K_nu.  The factor e^{-x cosh t}  */
/* is written e^{-x} e^{-x (cosh t - 1)} with cosh t - 1 = 2 sinh^2(t/2).                      */
/* ------------------------------------------------------------------------------------------ */
#define ORC_INNER_REL 1e-14

typedef struct { double nu, x; } bk_ctx;

static double k_integrand(double t, const void* c)
{
    const bk_ctx* k = (const bk_ctx*)c;
    double sh = sinh(0.5 * t);
    return exp(-k->x * 2.0 * sh * sh) * cosh(k->nu * t);
}

static double ki_integrand(double t, const void* c)
{
    const bk_ctx* k = (const bk_ctx*)c;
    double sh = sinh(0.5 * t);
    return exp(-k->x * 2.0 * sh * sh) * cosh(k->nu * t) / cosh(t);
}

/* Upper limit beyond which the integrand is < e^-60 of its size near the peak. */
static double bk_upper(double nu, double x)
{
    double T = acosh(1.0 + 60.0 / x) + 2.0 * nu + 2.0;
    return T < 100.0 ? T : 100.0;
}

double orc_bessel_k_scaled(double nu, double x)
{
    if (!(x > 0.0)) return INFINITY;
    bk_ctx c = {nu, x};
    return integrate(k_integrand, &c, 0.0, bk_upper(nu, x), ORC_INNER_REL, 8);
}

double orc_bessel_ki_scaled(double nu, double x)
{
    if (x < 0.0) return NAN;
    bk_ctx c = {nu, x};
    double T = (x > 0.0) ? bk_upper(nu, x) : 100.0;
    return integrate(ki_integrand, &c, 0.0, T, ORC_INNER_REL, 12);
}

double orc_bessel_k(double nu, double x) { return exp(-x) * orc_bessel_k_scaled(nu, x); }
double orc_bessel_ki(double nu, double x) { return exp(-x) * orc_bessel_ki_scaled(nu, x); }

/* ------------------------------------------------------------------------------------------ */
/* Total rates, paper Sec. 4.1 Eq. (wtilde) and Sec. 4.2 Eq. (wtilde_pair).                    */
/* ------------------------------------------------------------------------------------------ */
#define ORC_OUTER_REL 1e-12

/* W~_rad(chi) = int_0^inf (45 (v chi)^2 + 42 v chi + 20)/(2 + 3 v chi)^3 K_{2/3}(v) dv,
 * with v = t^3 (removes the v^{-2/3} endpoint singularity) and upper bound v = 700
 * (the paper's footnote to Eq. (wtilde): the remainder underflows). */
typedef struct { double chi; } chi_ctx;

static double wrad_integrand(double t, const void* c)
{
    double chi = ((const chi_ctx*)c)->chi;
    double v = t * t * t;
    double vc = v * chi;
    double rat = (45.0 * vc * vc + 42.0 * vc + 20.0) / pow(2.0 + 3.0 * vc, 3);
    return rat * orc_bessel_k(2.0 / 3.0, v) * 3.0 * t * t;
}

double orc_wtilde_rad(double chi)
{
    if (chi < 0.0) return NAN;
    chi_ctx c = {chi};
    return integrate(wrad_integrand, &c, 0.0, cbrt(700.0), ORC_OUTER_REL, 24);
}

/* W~_pair(chi) = int_0^1 (9 - v^2)/(3 (1 - v^2)) K_{2/3}(8/(3 chi (1 - v^2))) dv.
 * Computed as e^{-eta0} times the integral of the same integrand multiplied by e^{eta0},
 * eta0 = 8/(3 chi), so that the exponentially small values for small chi do not underflow;
 * orc_wtilde_pair_scaled returns e^{eta0} W~_pair. */
static double wpair_scaled_integrand(double v, const void* c)
{
    double chi = ((const chi_ctx*)c)->chi;
    double om = 1.0 - v * v;
    if (om <= 0.0) return 0.0;
    double eta0 = 8.0 / (3.0 * chi);
    double eta = eta0 / om;
    double d = eta0 * v * v / om; /* eta - eta0 */
    return (9.0 - v * v) / (3.0 * om) * exp(-d) * orc_bessel_k_scaled(2.0 / 3.0, eta);
}

double orc_wtilde_pair_scaled(double chi)
{
    if (!(chi > 0.0)) return 0.0;
    chi_ctx c = {chi};
    return integrate(wpair_scaled_integrand, &c, 0.0, 1.0, ORC_OUTER_REL, 32);
}

double orc_wtilde_pair(double chi)
{
    if (!(chi > 0.0)) return 0.0;
    return exp(-8.0 / (3.0 * chi)) * orc_wtilde_pair_scaled(chi);
}

/* Normalised rates W = R / omega_r, paper Eqs. (pe_rate_3) and (pp_tot_real).
 * lr_over_lc = lambda_r / lambda_C.  The pair rate is zero below chi = 0.01, where the paper
 * neglects it (Sec. 4.2, text after Eq. (low_chi)); with bw_fast it is zero below chi = 0.3
 * (App. A, function 7). */
double orc_rate_compton(double gamma, double chi, double lr_over_lc)
{
    if (!(gamma > 0.0) || !(chi > 0.0)) return 0.0;
    return orc_alpha() / (sqrt(3.0) * ORC_PI) * lr_over_lc * chi / gamma * orc_wtilde_rad(chi);
}

double orc_rate_breit_wheeler(double gamma, double chi, double lr_over_lc, int bw_fast)
{
    double chi_min = bw_fast ? 0.3 : 0.01;
    if (!(gamma > 0.0) || !(chi >= chi_min)) return 0.0;
    return orc_alpha() / (sqrt(3.0) * ORC_PI) * lr_over_lc / gamma * orc_wtilde_pair(chi);
}

/* ------------------------------------------------------------------------------------------ */
/* Photon-emission spectrum in the w variable, paper Sec. 4.3 Eqs. (subs_altri), (pe_eff_int_2).*/
/* ------------------------------------------------------------------------------------------ */
/* dI~_pe/dw = 9 w^2/(2 (1+s)^3) { [1 + (1+s)^2] K_{2/3}(w^3) - (1+s) Ki_{1/3}(w^3) },
 * s = 3 chi w^3 / 2. */
double orc_photon_spectrum_w(double w, double chi)
{
    if (!(w > 0.0)) return 0.0;
    double x = w * w * w;
    double s = 1.5 * chi * x;
    double op = 1.0 + s;
    double k23 = orc_bessel_k(2.0 / 3.0, x);
    double ki13 = orc_bessel_ki(1.0 / 3.0, x);
    return 9.0 * w * w / (2.0 * op * op * op) * ((1.0 + op * op) * k23 - op * ki13);
}

/* The same integrand written with K_{5/3}: using K_{1/3} + K_{5/3} = -2 K'_{2/3},
 *   (1+s)^{-1}[(1 + (1+s)^2) K_{2/3} - (1+s) Ki_{1/3}] = Ki_{5/3} + (xi^2/(1-xi)) K_{2/3},
 * xi = s/(1+s).  Used only as an independent check of the transcription and of positivity. */
double orc_photon_spectrum_w_k53(double w, double chi)
{
    if (!(w > 0.0)) return 0.0;
    double x = w * w * w;
    double s = 1.5 * chi * x;
    double op = 1.0 + s;
    double xi = s / op;
    double k23 = orc_bessel_k(2.0 / 3.0, x);
    double ki53 = orc_bessel_ki(5.0 / 3.0, x);
    return 9.0 * w * w / (2.0 * op * op) * (ki53 + xi * xi * op * k23);
}

static double photon_spec_cb(double w, const void* c)
{
    return orc_photon_spectrum_w(w, ((const chi_ctx*)c)->chi);
}

/* I~_pe(wbar, chi) = int_0^wbar dI~_pe/dw dw */
double orc_photon_cdf(double wbar, double chi)
{
    if (!(wbar > 0.0)) return 0.0;
    chi_ctx c = {chi};
    return integrate(photon_spec_cb, &c, 0.0, wbar, ORC_OUTER_REL, 16);
}

/* Upper tail int_wbar^inf, integrated directly (no subtraction from the total).  The
 * integrand carries e^{-w^3}; beyond w^3 = wbar^3 + 60 it is below e^-60 of its value at
 * wbar, and beyond w^3 = 700 it underflows. */
double orc_photon_ccdf(double wbar, double chi)
{
    if (wbar < 0.0) wbar = 0.0;
    double xb = wbar * wbar * wbar;
    double xe = xb + 60.0;
    if (xe > 700.0) xe = 700.0;
    if (xb >= xe) return 0.0;
    chi_ctx c = {chi};
    return integrate(photon_spec_cb, &c, wbar, cbrt(xe), ORC_OUTER_REL, 24);
}

/* ------------------------------------------------------------------------------------------ */
/* Pair-creation spectrum in the v variable, paper Sec. 4.4 Eqs. (subs_pair), (tilde_I_pp).    */
/* All pair CDF values are returned multiplied by e^{eta0}, eta0 = 8/(3 chi), like             */
/* orc_wtilde_pair_scaled; the inversion equation is homogeneous in that factor.              */
/* ------------------------------------------------------------------------------------------ */
/* dI~_pp/dv = 2 (1+v^2)/(1-v^2) K_{2/3}(eta_v) + Ki_{1/3}(eta_v),  eta_v = 8/(3 chi (1 - v^2)) */
double orc_pair_spectrum_v_scaled(double v, double chi)
{
    double om = 1.0 - v * v;
    if (!(om > 0.0) || !(chi > 0.0)) return 0.0;
    double eta0 = 8.0 / (3.0 * chi);
    double eta = eta0 / om;
    double d = eta0 * v * v / om;
    double e = exp(-d);
    return e * (2.0 * (1.0 + v * v) / om * orc_bessel_k_scaled(2.0 / 3.0, eta) +
                orc_bessel_ki_scaled(1.0 / 3.0, eta));
}

static double pair_spec_cb(double v, const void* c)
{
    return orc_pair_spectrum_v_scaled(v, ((const chi_ctx*)c)->chi);
}

double orc_pair_cdf_scaled(double vbar, double chi)
{
    if (!(vbar > 0.0)) return 0.0;
    if (vbar > 1.0) vbar = 1.0;
    chi_ctx c = {chi};
    return integrate(pair_spec_cb, &c, 0.0, vbar, ORC_OUTER_REL, 16);
}

double orc_pair_ccdf_scaled(double vbar, double chi)
{
    if (vbar < 0.0) vbar = 0.0;
    if (vbar >= 1.0) return 0.0;
    chi_ctx c = {chi};
    return integrate(pair_spec_cb, &c, vbar, 1.0, ORC_OUTER_REL, 24);
}

/* ------------------------------------------------------------------------------------------ */
/* Brent's root finder (Brent 1973: bisection, secant and inverse quadratic interpolation).   */
/* ------------------------------------------------------------------------------------------ */
typedef double (*orc_root_fn)(double x, const void* ctx);

static double brent(orc_root_fn f, const void* ctx, double a, double b, double fa, double fb,
                    double rtol)
{
    if (fa == 0.0) return a;
    if (fb == 0.0) return b;
    double c = a, fc = fa, d = b - a, e = d;
    for (int it = 0; it < 300; ++it) {
        if ((fb > 0.0) == (fc > 0.0)) { c = a; fc = fa; d = b - a; e = d; }
        if (fabs(fc) < fabs(fb)) { a = b; b = c; c = a; fa = fb; fb = fc; fc = fa; }
        double tol = 2.0 * 1.1e-16 * fabs(b) + 0.5 * rtol * fabs(b) + 1e-300;
        double m = 0.5 * (c - b);
        if (fabs(m) <= tol || fb == 0.0) return b;
        if (fabs(e) >= tol && fabs(fa) > fabs(fb)) {
            double s = fb / fa, p, q;
            if (a == c) { /* secant */
                p = 2.0 * m * s;
                q = 1.0 - s;
            } else { /* inverse quadratic interpolation */
                double qq = fa / fc, r = fb / fc;
                p = s * (2.0 * m * qq * (qq - r) - (b - a) * (r - 1.0));
                q = (qq - 1.0) * (r - 1.0) * (s - 1.0);
            }
            if (p > 0.0) q = -q; else p = -p;
            if (2.0 * p < fmin(3.0 * m * q - fabs(tol * q), fabs(e * q))) {
                e = d;
                d = p / q;
            } else { d = m; e = m; }
        } else { d = m; e = m; }
        a = b;
        fa = fb;
        b += (fabs(d) > tol) ? d : (m > 0.0 ? tol : -tol);
        fb = f(b, ctx);
    }
    return b;
}

/* ------------------------------------------------------------------------------------------ */
/* Inverse transform sampling.                                                                 */
/* ------------------------------------------------------------------------------------------ */
#define ORC_ROOT_RTOL 2e-15

typedef struct { double chi, level; } its_ctx;

static double ph_lower(double w, const void* c)
{
    const its_ctx* k = (const its_ctx*)c;
    return orc_photon_cdf(w, k->chi) - k->level;
}
static double ph_upper(double w, const void* c)
{
    const its_ctx* k = (const its_ctx*)c;
    return orc_photon_ccdf(w, k->chi) - k->level;
}

/* Solve I~_pe(wbar, chi) = r W~_rad(chi) (paper Eq. (again)).  For r <= 1/2 the CDF itself is
 * used; for r > 1/2 the equivalent upper-tail form int_wbar^inf = (1 - r) W~_rad, so that no
 * digits are lost near r -> 1.  Returns wbar. */
double orc_photon_wbar(double chi, double r)
{
    if (!(r > 0.0) || !(r < 1.0) || !(chi > 0.0)) return NAN;
    double W = orc_wtilde_rad(chi);
    /* slope of I~_pe at w = 0: 9 Gamma(2/3) / 2^{1/3} (paper Eq. (pe_eff_int_approx_w_small));
     * since the spectrum is largest at w = 0 the linear form is a lower bound for wbar. */
    double k0 = 9.0 * tgamma(2.0 / 3.0) / cbrt(2.0);
    if (r <= 0.5) {
        its_ctx c = {chi, r * W};
        double lo = r * W / k0, flo = ph_lower(lo, &c);
        if (flo >= 0.0) { /* only by rounding at tiny r */
            double hi0 = lo;
            lo = 0.5 * lo;
            flo = ph_lower(lo, &c);
            double fhi0 = ph_lower(hi0, &c);
            return brent(ph_lower, &c, lo, hi0, flo, fhi0, ORC_ROOT_RTOL);
        }
        double hi = 2.0 * lo, fhi = ph_lower(hi, &c);
        while (fhi < 0.0) { lo = hi; flo = fhi; hi *= 2.0; fhi = ph_lower(hi, &c); }
        return brent(ph_lower, &c, lo, hi, flo, fhi, ORC_ROOT_RTOL);
    } else {
        its_ctx c = {chi, (1.0 - r) * W};
        double lo = 0.0, flo = W - c.level;
        double hi = 0.5, fhi = ph_upper(hi, &c);
        while (fhi > 0.0) { lo = hi; flo = fhi; hi *= 1.5; fhi = ph_upper(hi, &c); }
        return brent(ph_upper, &c, lo, hi, flo, fhi, ORC_ROOT_RTOL);
    }
}

/* Photon energy from (gamma_e, chi_e, r): wbar from the ITS equation, then
 * s = 3 chi wbar^3 / 2, gamma_photon = gamma s/(1+s) (paper Eq. (subs_altri)); the emitter keeps
 * gamma - gamma_photon = gamma/(1+s) (collinear recoil by energy conservation). */
void orc_sample_photon(double gamma, double chi, double r, double* gamma_photon,
                       double* gamma_emitter, double* wbar_out)
{
    double wb = orc_photon_wbar(chi, r);
    double s = 1.5 * chi * wb * wb * wb;
    if (gamma_photon) *gamma_photon = gamma * (s / (1.0 + s));
    if (gamma_emitter) *gamma_emitter = gamma / (1.0 + s);
    if (wbar_out) *wbar_out = wb;
}

static double pp_lower(double v, const void* c)
{
    const its_ctx* k = (const its_ctx*)c;
    return orc_pair_cdf_scaled(v, k->chi) - k->level;
}
static double pp_upper(double v, const void* c)
{
    const its_ctx* k = (const its_ctx*)c;
    return orc_pair_ccdf_scaled(v, k->chi) - k->level;
}

/* Solve I~_pp(vbar, chi) = |r'| W~_pair(chi), r' = 2 r - 1 (paper Eq. (again_pp)); for
 * |r'| > 1/2 the upper-tail form int_vbar^1 = (1 - |r'|) W~_pair is solved instead. */
double orc_pair_vbar(double chi, double r)
{
    if (!(r > 0.0) || !(r < 1.0) || !(chi > 0.0)) return NAN;
    double rp = 2.0 * r - 1.0;
    double q = fabs(rp);
    if (q == 0.0) return 0.0;
    double W = orc_wtilde_pair_scaled(chi);
    if (q <= 0.5) {
        its_ctx c = {chi, q * W};
        return brent(pp_lower, &c, 0.0, 1.0, -c.level, W - c.level, ORC_ROOT_RTOL);
    } else {
        its_ctx c = {chi, (1.0 - q) * W};
        return brent(pp_upper, &c, 0.0, 1.0, W - c.level, -c.level, ORC_ROOT_RTOL);
    }
}

/* Electron energy gamma (1 + sgn(r') vbar)/2 and positron energy gamma (1 - sgn(r') vbar)/2
 * (paper Eq. (return_to_nrg)); sgn(0) = +1, irrelevant since vbar(0) = 0. */
void orc_sample_pair(double gamma, double chi, double r, double* gamma_electron,
                     double* gamma_positron, double* vbar_out)
{
    double vb = orc_pair_vbar(chi, r);
    double sg = (2.0 * r - 1.0) < 0.0 ? -1.0 : 1.0;
    if (gamma_electron) *gamma_electron = 0.5 * gamma * (1.0 + sg * vb);
    if (gamma_positron) *gamma_positron = 0.5 * gamma * (1.0 - sg * vb);
    if (vbar_out) *vbar_out = vb;
}

/* ------------------------------------------------------------------------------------------ */
/* Quantum parameter chi, paper Sec. 4 Eq. (chi_exact), in normalised units:                  */
/*   chi = gamma (lambda_C/lambda_r) sqrt((E + beta x B)^2 - (beta . E)^2),  beta = p/gamma,  */
/* gamma = sqrt(1 + p^2) for leptons and |p| for photons.  Long double; radicand clamped at 0. */
/* ------------------------------------------------------------------------------------------ */
double orc_chi(int is_photon, const double p[3], const double E[3], const double B[3],
               double lc_over_lr)
{
    long double px = p[0], py = p[1], pz = p[2];
    long double p2 = px * px + py * py + pz * pz;
    long double g = is_photon ? sqrtl(p2) : sqrtl(1.0L + p2);
    if (g == 0.0L) return 0.0;
    long double bx = px / g, by = py / g, bz = pz / g;
    long double ex = E[0], ey = E[1], ez = E[2];
    long double fx = ex + (by * B[2] - bz * B[1]);
    long double fy = ey + (bz * B[0] - bx * B[2]);
    long double fz = ez + (bx * B[1] - by * B[0]);
    long double be = bx * ex + by * ey + bz * ez;
    long double rad = fx * fx + fy * fy + fz * fz - be * be;
    if (rad < 0.0L) rad = 0.0L;
    return (double)(g * (long double)lc_over_lr * sqrtl(rad));
}

/* ------------------------------------------------------------------------------------------ */
/* Boris push (J. P. Boris, Proc. 4th Conf. Num. Sim. Plasmas, 1970), the leapfrog momentum     */
/* update of the PIC cycle (paper Fig. 7): for charge q (units of |e|, mass m_e) in normalised  */
/* units dp/dt = q (E + p x B / gamma): half an electric kick, a rotation about B by the        */
/* half-angle vector t = q dt B / (2 gamma^-), and the other half electric kick.               */
/* ------------------------------------------------------------------------------------------ */
void orc_boris_push(double q, const double p[3], const double E[3], const double B[3], double dt,
                    double out[3])
{
    const long double h = 0.5L * (long double)q * (long double)dt;
    long double um[3], t[3], s[3], up[3], uq[3];
    for (int k = 0; k < 3; ++k) um[k] = (long double)p[k] + h * (long double)E[k];
    const long double g = sqrtl(1.0L + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int k = 0; k < 3; ++k) t[k] = h * (long double)B[k] / g;
    const long double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int k = 0; k < 3; ++k) s[k] = 2.0L * t[k] / (1.0L + t2);
    up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    uq[0] = um[0] + (up[1] * s[2] - up[2] * s[1]);
    uq[1] = um[1] + (up[2] * s[0] - up[0] * s[2]);
    uq[2] = um[2] + (up[0] * s[1] - up[1] * s[0]);
    for (int k = 0; k < 3; ++k) out[k] = (double)(uq[k] + h * (long double)E[k]);
}

void orc_boris_push_batch(double q, long n, const double* px, const double* py, const double* pz,
                          const double* ex, const double* ey, const double* ez, const double* bx,
                          const double* by, const double* bz, double dt, double* ox, double* oy,
                          double* oz)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        const double p[3] = {px[i], py[i], pz[i]}, E[3] = {ex[i], ey[i], ez[i]},
                     B[3] = {bx[i], by[i], bz[i]};
        double o[3];
        orc_boris_push(q, p, E, B, dt, o);
        ox[i] = o[0];
        oy[i] = o[1];
        oz[i] = o[2];
    }
}

double orc_gamma(int is_photon, const double p[3])
{
    long double p2 = (long double)p[0] * p[0] + (long double)p[1] * p[1] + (long double)p[2] * p[2];
    return (double)(is_photon ? sqrtl(p2) : sqrtl(1.0L + p2));
}

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011).  One round on (x0,x1,x2,x3) with key (k0,k1):           */
/*   (hi0,lo0) = 0xD2511F53 * x0,  (hi1,lo1) = 0xCD9E8D57 * x2 (64-bit products),              */
/*   out = (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0);                                           */
/* the key is advanced by (0x9E3779B9, 0xBB67AE85) between rounds.                             */
/* ------------------------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t m0 = (uint64_t)0xD2511F53u * x0;
        uint64_t m1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0 = (uint32_t)(m1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)m1;
        uint32_t y2 = (uint32_t)(m0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)m0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Draw layout: key = (seed mod 2^32, seed >> 32); counter = (uid mod 2^32, uid >> 32, step,
 * purpose).  The four output words form two 64-bit words a = x0:x1 and b = x2:x3. */
void orc_draw(uint64_t seed, uint64_t uid, uint32_t step, uint32_t purpose, uint64_t* a,
              uint64_t* b)
{
    uint32_t ctr[4] = {(uint32_t)uid, (uint32_t)(uid >> 32), step, purpose};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    *a = ((uint64_t)o[0] << 32) | o[1];
    *b = ((uint64_t)o[2] << 32) | o[3];
}

/* Uniform in the open interval (0,1): ((a >> 12) + 1/2) 2^-52, exact in double. */
double orc_uniform(uint64_t a) { return ((double)(a >> 12) + 0.5) * 0x1p-52; }

/* Optical depth from a uniform: tau = -ln(1 - r) (paper Sec. 2, text after Eq. (any_event)). */
double orc_optical_depth(uint64_t a) { return -log(1.0 - orc_uniform(a)); }

/* ------------------------------------------------------------------------------------------ */
/* The Monte Carlo step for one particle.                                                       */
/* ------------------------------------------------------------------------------------------ */
enum { ORC_ELECTRON = 0, ORC_POSITRON = 1, ORC_PHOTON = 2 };
enum { ORC_P_INIT = 0, ORC_P_EMIT = 1, ORC_P_CHILD = 2, ORC_P_CHILD2 = 3, ORC_P_LOCAL = 4 };
enum { ORC_OPTICAL_DEPTH = 0, ORC_LOCAL = 1 };

typedef struct {
    double dt;          /* time step in units of 1/omega_r */
    double lc_over_lr;  /* lambda_C / lambda_r */
    uint64_t seed;
    uint32_t step;
    int32_t decision;   /* ORC_OPTICAL_DEPTH or ORC_LOCAL */
    int32_t bw_fast;
    int32_t pad;
} orc_step_cfg;

/* Per-particle result of one step.  Products are written into prod[0..1]:
 *   lepton emitter : prod[0] = photon
 *   converting photon: prod[0] = electron, prod[1] = positron                               */
typedef struct {
    double px, py, pz, tau;
    uint64_t uid, parent;
    double gamma;
    int32_t species, valid;
} orc_product;

typedef struct {
    double chi, gamma, rate;
    double tau_out;
    double px, py, pz;
    int32_t emitted, alive_out, clamped, pad;
    double r_energy; /* the energy uniform, for diagnostics */
    double xi_or_v;  /* photon: gamma_photon/gamma; pair: vbar */
    orc_product prod[2];
} orc_result;

/* Emission decision (paper Sec. 2).  Optical depth: tau_d <- tau_d - W dt, event iff the new
 * tau_d < 0 (the remaining optical depth is stored in *tau either way; after an event the caller
 * overwrites it with a fresh -ln(1 - r)).  Local: event iff W dt > r with r from draw purpose
 * ORC_P_LOCAL; *tau is not touched. */
int orc_decide(const orc_step_cfg* cfg, double W, uint64_t uid, double* tau)
{
    if (cfg->decision == ORC_OPTICAL_DEPTH) {
        double t = *tau - W * cfg->dt;
        *tau = t;
        return t < 0.0;
    }
    uint64_t a, b;
    orc_draw(cfg->seed, uid, cfg->step, ORC_P_LOCAL, &a, &b);
    return W * cfg->dt > orc_uniform(a);
}

/* Decisions only, for a given rate per particle: after an optical-depth event the particle's
 * tau is re-drawn from purpose ORC_P_EMIT word b, as in the full step.  For statistics tests. */
void orc_decide_batch(const orc_step_cfg* cfg, long n, const double* W, double* tau,
                      const uint64_t* uid, int32_t* emitted)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        int e = orc_decide(cfg, W[i], uid[i], &tau[i]);
        emitted[i] = e;
        if (e && cfg->decision == ORC_OPTICAL_DEPTH) {
            uint64_t a, b;
            orc_draw(cfg->seed, uid[i], cfg->step, ORC_P_EMIT, &a, &b);
            tau[i] = orc_optical_depth(b);
        }
    }
}

/* Scale a momentum vector to the magnitude belonging to energy g (lepton: sqrt(g^2-1),
 * photon: g), keeping its direction (paper App. A, function 17, collinear momentum).
 * A lepton with g <= 1 is left at rest and reported as clamped. */
static int collinear(const double pin[3], double pn, double g, int photon, double out[3])
{
    double mag;
    int clamped = 0;
    if (photon) mag = g;
    else if (g > 1.0) mag = sqrt((g - 1.0) * (g + 1.0));
    else { mag = 0.0; clamped = 1; }
    double f = (pn > 0.0) ? mag / pn : 0.0;
    out[0] = pin[0] * f; out[1] = pin[1] * f; out[2] = pin[2] * f;
    return clamped;
}

void orc_step_one(const orc_step_cfg* cfg, int species, const double p[3], const double E[3],
                  const double B[3], double tau, uint64_t uid, int alive, orc_result* res)
{
    memset(res, 0, sizeof(*res));
    res->px = p[0]; res->py = p[1]; res->pz = p[2];
    res->tau_out = tau;
    res->alive_out = alive;
    if (!alive) return;
    int photon = (species == ORC_PHOTON);
    double gamma = orc_gamma(photon, p);
    double chi = orc_chi(photon, p, E, B, cfg->lc_over_lr);
    double lr_over_lc = 1.0 / cfg->lc_over_lr;
    double W = photon ? orc_rate_breit_wheeler(gamma, chi, lr_over_lc, cfg->bw_fast)
                      : orc_rate_compton(gamma, chi, lr_over_lc);
    res->chi = chi;
    res->gamma = gamma;
    res->rate = W;

    int emit = orc_decide(cfg, W, uid, &res->tau_out);
    if (!emit) return;
    res->emitted = 1;

    uint64_t e_a, e_b, c_a, c_b;
    orc_draw(cfg->seed, uid, cfg->step, ORC_P_EMIT, &e_a, &e_b);
    orc_draw(cfg->seed, uid, cfg->step, ORC_P_CHILD, &c_a, &c_b);
    double r = orc_uniform(e_a);
    res->r_energy = r;
    double pn = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);

    if (!photon) {
        double gph, gem, wb;
        orc_sample_photon(gamma, chi, r, &gph, &gem, &wb);
        res->xi_or_v = gph / gamma;
        double pnew[3], pph[3];
        res->clamped = collinear(p, pn, gem, 0, pnew);
        collinear(p, pn, gph, 1, pph);
        res->px = pnew[0]; res->py = pnew[1]; res->pz = pnew[2];
        if (cfg->decision == ORC_OPTICAL_DEPTH) res->tau_out = orc_optical_depth(e_b);
        orc_product* q = &res->prod[0];
        q->px = pph[0]; q->py = pph[1]; q->pz = pph[2];
        q->tau = orc_optical_depth(c_a);
        q->uid = c_b;
        q->parent = uid;
        q->gamma = gph;
        q->species = ORC_PHOTON;
        q->valid = 1;
    } else {
        double ge, gp, vb;
        orc_sample_pair(gamma, chi, r, &ge, &gp, &vb);
        res->xi_or_v = vb;
        uint64_t d_a, d_b;
        orc_draw(cfg->seed, uid, cfg->step, ORC_P_CHILD2, &d_a, &d_b);
        double pe[3], pp[3];
        int c1 = collinear(p, pn, ge, 0, pe);
        int c2 = collinear(p, pn, gp, 0, pp);
        res->clamped = c1 + c2;
        res->alive_out = 0;
        orc_product* q = &res->prod[0];
        q->px = pe[0]; q->py = pe[1]; q->pz = pe[2];
        q->tau = orc_optical_depth(e_b);
        q->uid = c_b;
        q->parent = uid;
        q->gamma = ge;
        q->species = ORC_ELECTRON;
        q->valid = 1;
        q = &res->prod[1];
        q->px = pp[0]; q->py = pp[1]; q->pz = pp[2];
        q->tau = orc_optical_depth(c_a);
        q->uid = d_a;
        q->parent = uid;
        q->gamma = gp;
        q->species = ORC_POSITRON;
        q->valid = 1;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Beyond-LCFA photon emission, paper Sec. 5.                                                   */
/* ------------------------------------------------------------------------------------------ */
/* State per lepton: Fperp[3] = F_{L,perp}^{(n-1)}, dF[3] = F^{(n-1)} - F^{(n-2)}, just_created.
 * Inputs: p_prev = p^{(n-1/2)}, p_push = p_L^{(n+1/2)}, dt, tau_c = lambda_C/lambda_r.
 * Returns the flag of the condition below Eq. (condit); outputs gamma^{(n)}, chi^{(n)},
 * delta^{(n)}.  A particle flagged just_created stores F_perp and dF = 0 (Sec. 5 sets
 * F^{(n-2)} = F^{(n-1)} = F^{(n)}) and reports no emission. */
int orc_blcfa_update(const double p_prev[3], const double p_push[3], double dt, double tau_c,
                     double Fperp[3], double dF[3], int* just_created, double* gamma_out,
                     double* chi_out, double* delta_out, int* first_step)
{
    double FL[3], pL[3];
    for (int k = 0; k < 3; ++k) {
        FL[k] = (p_push[k] - p_prev[k]) / dt;          /* Eq. (fl) */
        pL[k] = 0.5 * (p_push[k] + p_prev[k]);
    }
    double p2 = pL[0] * pL[0] + pL[1] * pL[1] + pL[2] * pL[2];
    double g2 = 1.0 + p2;
    double g = sqrt(g2);                              /* Eq. (gammaBLCFA) */
    double fp = FL[0] * pL[0] + FL[1] * pL[1] + FL[2] * pL[2];
    double Fp[3];
    for (int k = 0; k < 3; ++k) Fp[k] = FL[k] - fp / g2 * pL[k];   /* Eq. (fl_perp) */
    double F2 = Fp[0] * Fp[0] + Fp[1] * Fp[1] + Fp[2] * Fp[2];
    double chi = tau_c * g * sqrt(F2);                /* Eq. (chi_p) */
    *gamma_out = g;
    *chi_out = chi;
    *delta_out = 0.0;
    if (first_step) *first_step = 0;
    if (*just_created) {
        for (int k = 0; k < 3; ++k) { Fperp[k] = Fp[k]; dF[k] = 0.0; }
        *just_created = 0;
        if (first_step) *first_step = 1;
        return 0;
    }
    double d1[3], d2[3];
    for (int k = 0; k < 3; ++k) {
        double diff = Fp[k] - Fperp[k];               /* F^(n) - F^(n-1) */
        d1[k] = diff / dt;                            /* first derivative */
        d2[k] = (diff - dF[k]) / (dt * dt);           /* second derivative */
    }
    double dd = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
    double fd = fabs(Fp[0] * d2[0] + Fp[1] * d2[1] + Fp[2] * d2[2]);
    double delta = tau_c * tau_c * (dd + fd);          /* Eq. (condit) */
    for (int k = 0; k < 3; ++k) { dF[k] = Fp[k] - Fperp[k]; Fperp[k] = Fp[k]; }
    *delta_out = delta;
    const double zeta = 2.220446049250313e-16;
    return (g2 * delta / (zeta * zeta) > chi * chi * F2) && (chi > zeta);
}

/* gamma_{gamma,LCFA} of Eq. (gammaLCFA) with tau/tau_C = 2 pi sqrt(F_perp^2 / delta). */
double orc_blcfa_threshold(const double Fperp[3], double delta, double gamma, double chi)
{
    double F2 = Fperp[0] * Fperp[0] + Fperp[1] * Fperp[1] + Fperp[2] * Fperp[2];
    double tau_ratio = 2.0 * ORC_PI * sqrt(F2 / delta);
    double arg = chi / (8.0 * gamma) * tau_ratio;
    return 0.7 * gamma / (1.0 + 4.0 / (3.0 * ORC_PI * chi) * sinh(3.0 * asinh(arg)));
}

/* The LCFA photon-energy distribution in gamma_photon (paper Eq. (pe_dp)) up to factors that
 * do not depend on gamma_photon:  (1/(1+u)) [(1 + (1+u)^2) K_{2/3}(z) - (1+u) Ki_{1/3}(z)],
 * u = g_ph/(gamma - g_ph), z = 2u/(3 chi). */
double orc_photon_pdf_energy(double g_ph, double gamma, double chi)
{
    if (!(g_ph > 0.0) || !(g_ph < gamma)) return 0.0;
    double u = g_ph / (gamma - g_ph);
    double z = 2.0 * u / (3.0 * chi);
    double op = 1.0 + u;
    return ((1.0 + op * op) * orc_bessel_k(2.0 / 3.0, z) - op * orc_bessel_ki(1.0 / 3.0, z)) / op;
}

/* Acceptance of Eq. (rej_cond): a sample gbar above the threshold is kept; below it, it is
 * kept iff r2 * pdf(gbar) <= pdf(threshold).  Returns 1 if accepted. */
int orc_blcfa_accept(double gbar, double limit, double gamma, double chi, double r2)
{
    if (gbar > limit) return 1;
    return r2 * orc_photon_pdf_energy(gbar, gamma, chi) <=
           orc_photon_pdf_energy(limit, gamma, chi);
}

/* One beyond-LCFA step of a lepton (paper Sec. 5 with the local decision of Sec. 2).
 * p_prev = p^{(n-1/2)}, p_push = p_L^{(n+1/2)}; the state (Fperp, dF, just_created) is updated.
 * Readings where the paper is silent: a particle that was just created stores its force and
 * cannot emit; when the condition below Eq. (condit) fails, a particle with chi > zeta emits by
 * the LCFA (threshold 0) and one with chi <= zeta does not emit; the energy of the emitted photon
 * is taken from the pushed momentum, gamma' = sqrt(1 + p_push^2) - gamma_photon, and the
 * emitter keeps its direction.  Draws: P_LOCAL a decides, P_EMIT a samples the energy, P_LOCAL b
 * accepts (Eq. (rej_cond)); the photon product takes P_CHILD (a: optical depth, b: uid). */
void orc_step_blcfa_one(const orc_step_cfg* cfg, const double p_prev[3], const double p_push[3],
                        double Fperp[3], double dF[3], int* just_created, uint64_t uid,
                        orc_result* res)
{
    memset(res, 0, sizeof(*res));
    res->px = p_push[0]; res->py = p_push[1]; res->pz = p_push[2];
    res->alive_out = 1;
    double gamma, chi, delta;
    int first;
    const double tau_c = cfg->lc_over_lr;
    int flag = orc_blcfa_update(p_prev, p_push, cfg->dt, tau_c, Fperp, dF, just_created, &gamma,
                                &chi, &delta, &first);
    double W = orc_rate_compton(gamma, chi, 1.0 / cfg->lc_over_lr);
    res->chi = chi;
    res->gamma = gamma;
    res->rate = W;
    if (first) return;
    uint64_t la, lb;
    orc_draw(cfg->seed, uid, cfg->step, ORC_P_LOCAL, &la, &lb);
    if (!(W * cfg->dt > orc_uniform(la))) return;
    double limit;
    const double zeta = 2.220446049250313e-16;
    if (flag) {
        limit = orc_blcfa_threshold(Fperp, delta, gamma, chi);
        if (!(limit < 0.75 * gamma)) return;
    } else if (chi > zeta) {
        limit = 0.0;
    } else {
        return;
    }
    uint64_t e_a, e_b, c_a, c_b;
    orc_draw(cfg->seed, uid, cfg->step, ORC_P_EMIT, &e_a, &e_b);
    orc_draw(cfg->seed, uid, cfg->step, ORC_P_CHILD, &c_a, &c_b);
    double r = orc_uniform(e_a);
    res->r_energy = r;
    double gph, gem, wb;
    orc_sample_photon(gamma, chi, r, &gph, &gem, &wb);
    res->xi_or_v = gph / gamma;
    if (!orc_blcfa_accept(gph, limit, gamma, chi, orc_uniform(lb))) {
        res->clamped = -1; /* marks a rejection */
        return;
    }
    res->emitted = 1;
    double pn = sqrt(p_push[0] * p_push[0] + p_push[1] * p_push[1] + p_push[2] * p_push[2]);
    double g_after = sqrt(1.0 + pn * pn) - gph;
    double pnew[3], pph[3];
    res->clamped = collinear(p_push, pn, g_after, 0, pnew);
    collinear(p_push, pn, gph, 1, pph);
    res->px = pnew[0]; res->py = pnew[1]; res->pz = pnew[2];
    orc_product* q = &res->prod[0];
    q->px = pph[0]; q->py = pph[1]; q->pz = pph[2];
    q->tau = orc_optical_depth(c_a);
    q->uid = c_b;
    q->parent = uid;
    q->gamma = gph;
    q->species = ORC_PHOTON;
    q->valid = 1;
}

/* ------------------------------------------------------------------------------------------ */
/* Batched entry points (OpenMP over particles) used by the Python wrapper.                   */
/* ------------------------------------------------------------------------------------------ */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_wtilde_rad_batch(long n, const double* chi, double* out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (long i = 0; i < n; ++i) out[i] = orc_wtilde_rad(chi[i]);
}

void orc_wtilde_pair_scaled_batch(long n, const double* chi, double* out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (long i = 0; i < n; ++i) out[i] = orc_wtilde_pair_scaled(chi[i]);
}

void orc_rates_batch(long n, int is_photon, const double* gamma, const double* chi,
                     double lr_over_lc, int bw_fast, double* out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (long i = 0; i < n; ++i)
        out[i] = is_photon ? orc_rate_breit_wheeler(gamma[i], chi[i], lr_over_lc, bw_fast)
                           : orc_rate_compton(gamma[i], chi[i], lr_over_lc);
}

void orc_chi_batch(long n, int is_photon, const double* px, const double* py, const double* pz,
                   const double* ex, const double* ey, const double* ez, const double* bx,
                   const double* by, const double* bz, double lc_over_lr, double* gamma_out,
                   double* chi_out)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double p[3] = {px[i], py[i], pz[i]}, E[3] = {ex[i], ey[i], ez[i]},
               B[3] = {bx[i], by[i], bz[i]};
        if (gamma_out) gamma_out[i] = orc_gamma(is_photon, p);
        chi_out[i] = orc_chi(is_photon, p, E, B, lc_over_lr);
    }
}

void orc_sample_photon_batch(long n, const double* gamma, const double* chi, const double* r,
                             double* gph, double* gem, double* wbar)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < n; ++i)
        orc_sample_photon(gamma[i], chi[i], r[i], gph ? gph + i : 0, gem ? gem + i : 0,
                          wbar ? wbar + i : 0);
}

void orc_sample_pair_batch(long n, const double* gamma, const double* chi, const double* r,
                           double* ge, double* gp, double* vbar)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < n; ++i)
        orc_sample_pair(gamma[i], chi[i], r[i], ge ? ge + i : 0, gp ? gp + i : 0,
                        vbar ? vbar + i : 0);
}

void orc_step_batch(const orc_step_cfg* cfg, int species, long n, const double* px,
                    const double* py, const double* pz, const double* ex, const double* ey,
                    const double* ez, const double* bx, const double* by, const double* bz,
                    const double* tau, const uint64_t* uid, const uint8_t* alive, orc_result* out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < n; ++i) {
        double p[3] = {px[i], py[i], pz[i]}, E[3] = {ex[i], ey[i], ez[i]},
               B[3] = {bx[i], by[i], bz[i]};
        orc_step_one(cfg, species, p, E, B, tau[i], uid[i], alive ? alive[i] : 1, &out[i]);
    }
}

/* state arrays component-major: Fperp[k*n + i] */
void orc_step_blcfa_batch(const orc_step_cfg* cfg, long n, const double* pxp, const double* pyp,
                          const double* pzp, const double* px, const double* py, const double* pz,
                          double* Fperp, double* dF, uint8_t* just_created, const uint64_t* uid,
                          orc_result* out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < n; ++i) {
        double pp[3] = {pxp[i], pyp[i], pzp[i]}, pu[3] = {px[i], py[i], pz[i]};
        double F[3] = {Fperp[i], Fperp[n + i], Fperp[2 * n + i]};
        double D[3] = {dF[i], dF[n + i], dF[2 * n + i]};
        int jc = just_created[i];
        orc_step_blcfa_one(cfg, pp, pu, F, D, &jc, uid[i], &out[i]);
        for (int k = 0; k < 3; ++k) { Fperp[k * n + i] = F[k]; dF[k * n + i] = D[k]; }
        just_created[i] = (uint8_t)jc;
    }
}

long orc_result_size(void) { return (long)sizeof(orc_result); }
long orc_product_size(void) { return (long)sizeof(orc_product); }
