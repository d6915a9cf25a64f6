// sfq_device.h -- device-side arithmetic of the QED Monte Carlo step for gfx950.
//
// Method: Montefiori & Tamburini, arXiv:2301.07684 (SFQEDtoolkit).  What is computed here:
//   chi              Sec. 4 Eq. (chi_exact), rewritten as a sum of squares (no cancellation)
//   rates            Sec. 4.1 Eq. (pe_rate_3), Sec. 4.2 Eq. (pp_tot_real), from tables of
//                    W~_rad(chi) and e^{8/(3chi)} W~_pair(chi)/chi (Chebyshev, Clenshaw: App. B)
//   photon energy    Sec. 4.3 Eq. (again): tabulated inverse wbar(r, chi) -> Eq. (subs_altri)
//   pair energies    Sec. 4.4 Eqs. (again_pp), (return_to_nrg): tabulated inverse in
//                    y = eta_v - eta0 -> v -> electron/positron energies
//   photon spectrum  Sec. 4 Eq. (pe_dp) from tables of K_{2/3} and Ki_{1/3} (beyond-LCFA ratio)
//   Philox4x32-10    Salmon et al., SC'11
// The tables are produced by the package's table generator; their geometry is fixed here.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfq {

// ---------------------------------------------------------------------------------------------
// Table geometry (identical to the generator's; checked when the table file is loaded).
// ---------------------------------------------------------------------------------------------
constexpr int RATE_DEG = 20;
constexpr int CHI_OCT_LO = -6, CHI_OCT_HI = 16;
constexpr int N_CHI_SEG = 1 + (CHI_OCT_HI - CHI_OCT_LO);
constexpr int PAIR_OCT_LO = -7;
constexpr int N_PAIR_SEG = CHI_OCT_HI - PAIR_OCT_LO;
constexpr int KA_DEG = 20, N_KA = 4;
constexpr int KB_DEG = 18, KB_OCT_LO = 1, KB_OCT_HI = 18;
constexpr int INV_NC = 16, INV_NR = 12;
constexpr int N_LO_SEG = 4;
constexpr int T_OCT_LO = -1, T_OCT_HI = 6;
constexpr int N_HI_SEG = 2 * (T_OCT_HI - T_OCT_LO);
constexpr int N_R_SEG = N_LO_SEG + N_HI_SEG;
constexpr int INV_PATCH = INV_NR * INV_NC;

constexpr int RAD_SIZE = N_CHI_SEG * RATE_DEG;
constexpr int PAIR_SIZE = N_PAIR_SEG * RATE_DEG;
constexpr int KA_SIZE = N_KA * 2 * KA_DEG;
constexpr int KB_SIZE = (KB_OCT_HI - KB_OCT_LO) * 2 * KB_DEG;
constexpr int PHINV_SIZE = N_CHI_SEG * N_R_SEG * INV_PATCH;
constexpr int PPINV_SIZE = N_PAIR_SEG * N_R_SEG * INV_PATCH;

// ---------------------------------------------------------------------------------------------
// Physical constants (CODATA 2018) and derived numbers.
// ---------------------------------------------------------------------------------------------
constexpr double ALPHA = 7.2973525693e-3;
constexpr double LAMBDA_C = 3.8615926796e-13;  // reduced Compton wavelength hbar/(m c), metres
constexpr double C_LIGHT = 299792458.0;
constexpr double PI = 3.14159265358979323846;
constexpr double SQRT2 = 1.4142135623730951;
constexpr double ZETA = 2.220446049250313e-16;  // the "nearly negligible number" of Sec. 5
// large-chi forms used only above the tables (chi >= 2^16)
constexpr double WRAD_ASYM_C1 = 7.9471626165891861;   // 14 pi Gamma(2/3) 3^{2/3}/(9 sqrt 3)
constexpr double WRAD_ASYM_C2 = 4.5344984105855446;   // 5 pi / (2 sqrt 3)
constexpr double WPAIR_ASYM_C = 2.0656216916754387;   // 5 sqrt(pi) Gamma(2/3)^2 (3/4)^{2/3}/(7 Gamma(7/6))

// ---------------------------------------------------------------------------------------------
// Philox4x32-10
// ---------------------------------------------------------------------------------------------
struct Draw {
    uint64_t a, b;
};

__device__ __forceinline__ Draw philox_draw(uint64_t seed, uint64_t uid, uint32_t step,
                                            uint32_t purpose)
{
    uint32_t x0 = (uint32_t)uid, x1 = (uint32_t)(uid >> 32), x2 = step, x3 = purpose;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = 0xD2511F53u * x0, hi0 = __umulhi(0xD2511F53u, x0);
        const uint32_t lo1 = 0xCD9E8D57u * x2, hi1 = __umulhi(0xCD9E8D57u, x2);
        const uint32_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Draw d;
    d.a = ((uint64_t)x0 << 32) | x1;
    d.b = ((uint64_t)x2 << 32) | x3;
    return d;
}

// uniform in (0,1): ((a >> 12) + 1/2) 2^-52, exact in double
__device__ __forceinline__ double uniform53(uint64_t a)
{
    return fma((double)(a >> 12), 0x1p-52, 0x1p-53);
}

__device__ __forceinline__ double optical_depth(uint64_t a) { return -log(1.0 - uniform53(a)); }

// ---------------------------------------------------------------------------------------------
// chi and gamma.  With n = p/|p|, E_par = n.E, E_perp = E - E_par n, f = E_perp + n x B and
// d = gamma - |p| = m^2/(gamma + |p|) (m = 1 leptons, 0 photons):
//   (gamma E + p x B)^2 - (p.E)^2 = | |p| f + d E_perp |^2 + m^2 E_par^2,
// a sum of squares, so chi has no catastrophic cancellation for nearly co-propagating
// particles (where gamma E + p x B -> E/(gamma+|p|)).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void gamma_chi(bool photon, double px, double py, double pz, double ex,
                                          double ey, double ez, double bx, double by, double bz,
                                          double lc_over_lr, double& gamma, double& chi)
{
    const double p2 = fma(px, px, fma(py, py, pz * pz));
    const double pn = sqrt(p2);
    gamma = photon ? pn : sqrt(1.0 + p2);
    if (pn == 0.0) {  // at rest: chi = lc |E| for a lepton, 0 for a photon
        chi = photon ? 0.0 : lc_over_lr * sqrt(fma(ex, ex, fma(ey, ey, ez * ez)));
        return;
    }
    // correctly rounded quotients: an axis-aligned momentum gives an exact unit vector, so the
    // exactly co-propagating case (E_perp + n x B = 0) cancels exactly
    const double nx = px / pn, ny = py / pn, nz = pz / pn;
    const double epar = fma(nx, ex, fma(ny, ey, nz * ez));
    const double eqx = fma(-epar, nx, ex), eqy = fma(-epar, ny, ey), eqz = fma(-epar, nz, ez);
    const double fx = eqx + (ny * bz - nz * by);
    const double fy = eqy + (nz * bx - nx * bz);
    const double fz = eqz + (nx * by - ny * bx);
    const double d = photon ? 0.0 : 1.0 / (gamma + pn);
    const double vx = fma(pn, fx, d * eqx), vy = fma(pn, fy, d * eqy), vz = fma(pn, fz, d * eqz);
    double rad = fma(vx, vx, fma(vy, vy, vz * vz));
    if (!photon) rad = fma(epar, epar, rad);
    chi = lc_over_lr * sqrt(rad);
}

// ---------------------------------------------------------------------------------------------
// Clenshaw's recurrence (App. B): f = sum_{k<N} c_k T_k(X), c_0 full weight.
// ---------------------------------------------------------------------------------------------
template <int N, typename T, typename P>
__device__ __forceinline__ T clenshaw(const P* c, T X)
{
    T b1 = T(0), b2 = T(0);
    const T X2 = X + X;
#pragma unroll
    for (int k = N - 1; k >= 1; --k) {
        const T bn = fma(X2, b1, T(c[k]) - b2);
        b2 = b1;
        b1 = bn;
    }
    return fma(X, b1, T(c[0]) - b2);
}

// chi segment: 0 for chi < 2^CHI_OCT_LO (linear in chi), else the octave; X in [-1, 1].
// Returns true if chi is beyond the last octave (X is then clamped to 1).
__device__ __forceinline__ bool chi_segment(double chi, int& seg, double& X)
{
    if (chi < 0x1p-6) {
        seg = 0;
        X = fma(chi, 0x1p7, -1.0);
        return false;
    }
    const uint64_t bits = (uint64_t)__double_as_longlong(chi);
    const int e = (int)((bits >> 52) & 0x7ff) - 1023;
    const double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) |
                                                      0x3FF0000000000000ull));
    seg = e - CHI_OCT_LO + 1;
    X = fma(2.0, m, -3.0);
    if (seg > N_CHI_SEG - 1) {
        seg = N_CHI_SEG - 1;
        X = 1.0;
        return true;
    }
    return false;
}

__device__ __forceinline__ bool chi_segment(float chi, int& seg, float& X)
{
    if (chi < 0x1p-6f) {
        seg = 0;
        X = fmaf(chi, 0x1p7f, -1.0f);
        return false;
    }
    const uint32_t bits = (uint32_t)__float_as_int(chi);
    const int e = (int)((bits >> 23) & 0xff) - 127;
    const float m = __int_as_float((int)((bits & 0x007FFFFFu) | 0x3F800000u));
    seg = e - CHI_OCT_LO + 1;
    X = fmaf(2.0f, m, -3.0f);
    if (seg > N_CHI_SEG - 1) {
        seg = N_CHI_SEG - 1;
        X = 1.0f;
        return true;
    }
    return false;
}

// octave of chi for the pair tables (chi >= 2^PAIR_OCT_LO); clamps at both ends
template <typename T>
__device__ __forceinline__ bool pair_segment(T chi, int& seg, T& X)
{
    int e;
    const T m2 = frexp(chi, &e);  // chi = m2 2^e, m2 in [0.5, 1)
    int o = e - 1;
    T Xl = fma(T(4), m2, T(-3));  // 2 (2 m2) - 3
    bool out = false;
    if (o < PAIR_OCT_LO) { o = PAIR_OCT_LO; Xl = T(-1); }
    if (o > CHI_OCT_HI - 1) { o = CHI_OCT_HI - 1; Xl = T(1); out = true; }
    seg = o - PAIR_OCT_LO;
    X = Xl;
    return out;
}

// ---------------------------------------------------------------------------------------------
// Rates.  `rad` and `pair` point to the (LDS-staged) coefficient tables.
// ---------------------------------------------------------------------------------------------
// W~_rad(chi) (Sec. 4.1, Eq. (wtilde)); sets *ood when chi is beyond the tables
template <typename T, typename P>
__device__ __forceinline__ T wtilde_rad(const P* rad, T chi, bool* ood)
{
    int seg;
    T X;
    if (chi_segment(chi, seg, X)) {
        *ood = true;
        return T(WRAD_ASYM_C1) * pow(chi, T(-1.0 / 3.0)) - T(WRAD_ASYM_C2) / chi;
    }
    return clenshaw<RATE_DEG>(rad + seg * RATE_DEG, X);
}

// W~_pair(chi) (Sec. 4.2, Eq. (wtilde_pair)) for chi >= 2^PAIR_OCT_LO
template <typename T, typename P>
__device__ __forceinline__ T wtilde_pair(const P* pair, T chi, bool* ood)
{
    int seg;
    T X;
    if (pair_segment(chi, seg, X)) {
        *ood = true;
        return T(WPAIR_ASYM_C) * pow(chi, T(2.0 / 3.0));
    }
    const T P_ = clenshaw<RATE_DEG>(pair + seg * RATE_DEG, X);
    return chi * P_ * exp(T(-8.0 / 3.0) / chi);
}

// ---------------------------------------------------------------------------------------------
// Inverse-CDF tables.  r-segment from r in (0, 1): lower region r <= 1/2 in N_LO_SEG equal
// segments (local variable linear in r); upper region r > 1/2 by half-octaves of
// t = -ln(1 - r) (t in [2^e, 2^e sqrt2) or [2^e sqrt2, 2^{e+1})).
// ---------------------------------------------------------------------------------------------
struct RSeg {
    int seg;
    double X;
    bool upper;
};

__device__ __forceinline__ RSeg r_segment(double r)
{
    RSeg s;
    if (r <= 0.5) {
        int k = (int)(r * (2 * N_LO_SEG));
        k = k > N_LO_SEG - 1 ? N_LO_SEG - 1 : (k < 0 ? 0 : k);
        s.seg = k;
        s.X = fma(r, 4.0 * N_LO_SEG, -(2.0 * k + 1.0));
        s.upper = false;
        return s;
    }
    const double t = -log(1.0 - r);  // 1 - r is exact for r >= 1/2
    int e;
    const double m2 = frexp(t, &e);   // t = m2 2^e, m2 in [0.5, 1)
    int o = e - 1;
    const double m = 2.0 * m2;        // t = m 2^o, m in [1, 2)
    const int half = m >= SQRT2 ? 1 : 0;
    if (o < T_OCT_LO) o = T_OCT_LO;   // not reached: t >= ln 2
    if (o > T_OCT_HI - 1) o = T_OCT_HI - 1;
    const double a = ldexp(half ? SQRT2 : 1.0, o);
    const double b = ldexp(half ? 2.0 : SQRT2, o);
    s.seg = N_LO_SEG + 2 * (o - T_OCT_LO) + half;
    s.X = (2.0 * t - a - b) / (b - a);
    s.upper = true;
    return s;
}

// 2D patch evaluation: inner Clenshaw along chi for every r row, then along r (App. B,
// Eqs. (back_rec_2d), (start_cl_2)).
template <typename T, typename P>
__device__ __forceinline__ T patch_eval(const P* c, T Xc, T Xr)
{
    T d[INV_NR];
#pragma unroll
    for (int i = 0; i < INV_NR; ++i) d[i] = clenshaw<INV_NC>(c + i * INV_NC, Xc);
    return clenshaw<INV_NR>(d, Xr);
}

// Photon sample: returns s = 3 chi wbar^3 / 2 (Eq. (subs_altri)); the photon takes the energy
// fraction s/(1+s) and the emitter keeps 1/(1+s).
__device__ __forceinline__ double photon_s64(const double* tab, double chi, double r, bool* ood)
{
    int cs;
    double Xc;
    if (chi_segment(chi, cs, Xc)) *ood = true;
    const RSeg rs = r_segment(r);
    const double f = patch_eval(tab + (cs * N_R_SEG + rs.seg) * INV_PATCH, Xc, rs.X);
    double xbar;
    if (rs.upper) {
        xbar = exp(f);               // the table holds ln(wbar^3)
    } else {
        const double w = f * r;      // the table holds wbar / r
        xbar = w * w * w;
    }
    return 1.5 * chi * xbar;
}

__device__ __forceinline__ float photon_s32(const float* tab, double chi_d, double r, bool* ood)
{
    const float chi = (float)chi_d;
    int cs;
    float Xc;
    if (chi_segment(chi, cs, Xc)) *ood = true;
    const RSeg rs = r_segment(r);     // segment selection and t in double (exact 1 - r)
    const float f = patch_eval(tab + (cs * N_R_SEG + rs.seg) * INV_PATCH, Xc, (float)rs.X);
    float xbar;
    if (rs.upper) {
        xbar = expf(f);
    } else {
        const float w = f * (float)r;
        xbar = w * w * w;
    }
    return 1.5f * chi * xbar;
}

// Pair sample: returns y = eta_v - eta0 for |r'| = |2r - 1| (the table variable), from which
// v^2 = y/(y + eta0) and 1 - v^2 = eta0/(y + eta0).
__device__ __forceinline__ double pair_y64(const double* tab, double chi, double q, bool* ood)
{
    int cs;
    double Xc;
    if (pair_segment(chi, cs, Xc)) *ood = true;
    const RSeg rs = r_segment(q);
    const double f = patch_eval(tab + (cs * N_R_SEG + rs.seg) * INV_PATCH, Xc, rs.X);
    if (rs.upper) return exp(f);     // ln y
    const double u = f * q;          // sqrt(y) / q
    return u * u;
}

__device__ __forceinline__ float pair_y32(const float* tab, double chi_d, double q, bool* ood)
{
    const float chi = (float)chi_d;
    int cs;
    float Xc;
    if (pair_segment(chi, cs, Xc)) *ood = true;
    const RSeg rs = r_segment(q);
    const float f = patch_eval(tab + (cs * N_R_SEG + rs.seg) * INV_PATCH, Xc, (float)rs.X);
    if (rs.upper) return expf(f);
    const float u = f * (float)q;
    return u * u;
}

// ---------------------------------------------------------------------------------------------
// Bessel pieces of the photon spectrum (for the beyond-LCFA acceptance ratio): returns
// (K_{2/3}(x), Ki_{1/3}(x)) times e^{x} for x >= 2 (scaled) or unscaled for x < 2; *scaled
// tells which.  x must be > 0 and < 2^KB_OCT_HI.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void bessel_pieces(const double* ka, const double* kb, double x,
                                              double& k23, double& ki13, bool& scaled)
{
    constexpr double WS = 1.2599210498948732;  // 2^{1/3}
    if (x < 2.0) {
        const double w = cbrt(x);
        int s = (int)(w * (N_KA / WS));
        s = s > N_KA - 1 ? N_KA - 1 : (s < 0 ? 0 : s);
        const double a = WS * s / N_KA;
        const double X = (2.0 * w - a - (a + WS / N_KA)) / (WS / N_KA);
        const double* c = ka + s * 2 * KA_DEG;
        k23 = clenshaw<KA_DEG>(c, X) / (w * w);
        ki13 = clenshaw<KA_DEG>(c + KA_DEG, X);
        scaled = false;
        return;
    }
    int e;
    const double m2 = frexp(x, &e);
    int o = e - 1;
    if (o > KB_OCT_HI - 1) o = KB_OCT_HI - 1;
    const double a = ldexp(1.0, o);
    const double X = (2.0 * x - 3.0 * a) / a;
    (void)m2;
    const double* c = kb + (o - KB_OCT_LO) * 2 * KB_DEG;
    const double sq = rsqrt(x);
    k23 = sq * clenshaw<KB_DEG>(c, X);
    ki13 = sq * clenshaw<KB_DEG>(c + KB_DEG, X);
    scaled = true;
}

// log of the LCFA photon spectrum in photon energy (Eq. (pe_dp)) up to terms independent of
// the photon energy g (gamma_e fixed):  log{ (1/(1+u)) [(1+(1+u)^2) K_{2/3}(z) - (1+u) Ki_{1/3}(z)] },
// u = g/(gamma - g), z = 2u/(3 chi).  Logarithms keep the ratio of Eq. (rej_cond) finite when
// both values underflow.
__device__ __forceinline__ double log_photon_pdf(const double* ka, const double* kb, double g,
                                                 double gamma, double chi)
{
    const double u = g / (gamma - g);
    const double z = 2.0 * u / (3.0 * chi);
    if (!(z > 0.0)) return INFINITY;     // the spectrum diverges as g^{-2/3} at g -> 0
    if (!(z < 0x1p17)) return -INFINITY;
    double k, ki;
    bool scaled;
    bessel_pieces(ka, kb, z, k, ki, scaled);
    const double op = 1.0 + u;
    const double v = ((1.0 + op * op) * k - op * ki) / op;
    return log(v) - (scaled ? z : 0.0);
}

}  // namespace sfq
