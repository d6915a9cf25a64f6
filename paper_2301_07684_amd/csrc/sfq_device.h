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
constexpr int RATE_DEG = 16;
// The truncated evaluation form (an accuracy/speed dial, the analogue of the paper's choice of
// coefficient counts, Sec. 4.5): the leading RATE_DEG_TRUNC terms of each rate segment and the
// leading INV_TRUNC x INV_TRUNC coefficients of each inverse patch, from the same tables.
constexpr int RATE_DEG_TRUNC = 10;
constexpr int INV_TRUNC = 5;
constexpr int CHI_OCT_LO = -6, CHI_OCT_HI = 16;
constexpr int N_CHI_SEG = 1 + (CHI_OCT_HI - CHI_OCT_LO);
constexpr int PAIR_OCT_LO = -7;
constexpr int N_PAIR_SEG = CHI_OCT_HI - PAIR_OCT_LO;
constexpr int KA_DEG = 20, N_KA = 4;
constexpr int KB_DEG = 18, KB_OCT_LO = 1, KB_OCT_HI = 18;
constexpr int INV_NC = 8, INV_NR = 8;
constexpr int SUB = 4;                  // quarter-octave segments of the inverse tables
constexpr int INV_CHI_OCT_LO = -10;
constexpr int N_INV_CHI = 1 + SUB * (CHI_OCT_HI - INV_CHI_OCT_LO);
constexpr int N_PAIR_INV_CHI = SUB * (CHI_OCT_HI - PAIR_OCT_LO);
constexpr int N_LO_SEG = 8;
constexpr int T_OCT_LO = -1, T_OCT_HI = 6;
constexpr int N_HI_SEG = SUB * (T_OCT_HI - T_OCT_LO);
constexpr int N_R_SEG = N_LO_SEG + N_HI_SEG;
constexpr int INV_PATCH = INV_NR * INV_NC;

constexpr int RAD_SIZE = N_CHI_SEG * RATE_DEG;
constexpr int PAIR_SIZE = N_PAIR_SEG * RATE_DEG;
constexpr int KA_SIZE = N_KA * 2 * KA_DEG;
constexpr int KB_SIZE = (KB_OCT_HI - KB_OCT_LO) * 2 * KB_DEG;
constexpr int PHINV_SIZE = N_INV_CHI * N_R_SEG * INV_PATCH;
constexpr int PPINV_SIZE = N_PAIR_INV_CHI * N_R_SEG * INV_PATCH;

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
// chi and gamma.  With E_par = p.E/|p|, E_perp = E - (p.E/|p|^2) p and d = gamma - |p| =
// m^2/(gamma + |p|) (m = 1 leptons, 0 photons):
//   (gamma E + p x B)^2 - (p.E)^2 = | |p| E_perp + p x B + d E_perp |^2 + m^2 E_par^2,
// a sum of squares with gamma - |p| never formed by subtraction, so co-propagating particles
// (where gamma E + p x B -> E/(gamma+|p|)) keep their accuracy.
// ---------------------------------------------------------------------------------------------
// 1/x for normal x > 0: the hardware estimate refined by two Newton steps (error below 2 ulp;
// about half the instructions of a correctly rounded division).
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// sqrt(x) for x >= 0: the hardware reciprocal-square-root estimate refined by a Goldschmidt
// step and a residual correction (about 1 ulp); arguments below 2^-1000 (where the estimate
// would lose range) give 0.  No scaling path for subnormal input, which the step never needs.
__device__ __forceinline__ double sqrt_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double s = x * y, h = 0.5 * y;
    const double r = fma(-s, h, 0.5);
    s = fma(s, r, s);
    h = fma(h, r, h);
    const double d = fma(-s, s, x);
    s = fma(d, h, s);
    return x > 0x1p-1000 ? s : 0.0;
}

__device__ __forceinline__ void gamma_chi(bool photon, double px, double py, double pz, double ex,
                                          double ey, double ez, double bx, double by, double bz,
                                          double lc_over_lr, double& gamma, double& chi)
{
    const double p2 = fma(px, px, fma(py, py, pz * pz));
    const double pn = sqrt_nr(p2);
    gamma = photon ? pn : sqrt_nr(1.0 + p2);
    // A particle at rest (|p|^2 below 1e-300) takes the p -> 0 limit of the expressions below
    // (E_perp = E, u = 0): chi = lc |E| for a lepton, 0 for a photon.  No branch, so the loads
    // feeding this function are issued together.
    const bool moving = p2 > 1e-300;
    const double pe = fma(px, ex, fma(py, ey, pz * ez));
    const double q = moving ? pe * rcp_nr(p2) : 0.0;  // E_par^2 = q pe, E_perp = E - q p
    const double eqx = fma(-q, px, ex), eqy = fma(-q, py, ey), eqz = fma(-q, pz, ez);
    double ux, uy, uz;
    {
        // |p| E_perp + p x B, each product rounded on its own: for an exactly co-propagating
        // particle (|p| == p_x) the two terms cancel exactly
#pragma clang fp contract(off)
        ux = pn * eqx + (py * bz - pz * by);
        uy = pn * eqy + (pz * bx - px * bz);
        uz = pn * eqz + (px * by - py * bx);
    }
    const double d = photon ? 0.0 : rcp_nr(gamma + pn);  // gamma - |p| without cancellation
    const double vx = fma(d, eqx, ux), vy = fma(d, eqy, uy), vz = fma(d, eqz, uz);
    double rad = fma(vx, vx, fma(vy, vy, vz * vz));
    if (!photon) rad = fma(q, pe, rad);
    chi = lc_over_lr * sqrt_nr(rad);
}

// ---------------------------------------------------------------------------------------------
// cos(x) for |x| < 2^20 pi/2 (about 1.6e6), register-light: x = k pi/2 + r with k = rint(2x/pi),
// where pi/2 is split into parts of 33, 33 and 53 significant bits so that k times each of the
// first two is exact (Cody and Waite's argument reduction) and r keeps a few-ulp relative
// accuracy even where cos x is near zero; then the Taylor series of cos r (to r^16) or sin r
// (to r^17) on |r| <= pi/4, whose truncation is below 1e-17 of the result.  Coefficients are
// 1/n! rounded to double.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double cos_cw(double x)
{
    constexpr double TWO_OVER_PI = 0.6366197723675814;
    constexpr double P1 = 1.5707963267341256;     // pi/2 to 33 bits
    constexpr double P2 = 6.077100506303966e-11;  // next 33 bits
    constexpr double P3 = 2.0222662487959506e-21; // the rest
    const double k = rint(x * TWO_OVER_PI);
    double r = fma(-k, P1, x);
    r = fma(-k, P2, r);
    r = fma(-k, P3, r);
    const double z = r * r;
    // cos r = sum_j (-1)^j z^j / (2j)!,  sin r = r sum_j (-1)^j z^j / (2j+1)!,  j = 0..8
    double c = 4.779477332387385e-14;             // 1/16!
    c = fma(c, z, -1.1470745597729725e-11);       // 1/14!
    c = fma(c, z, 2.08767569878681e-09);          // 1/12!
    c = fma(c, z, -2.755731922398589e-07);        // 1/10!
    c = fma(c, z, 2.48015873015873e-05);          // 1/8!
    c = fma(c, z, -0.001388888888888889);         // 1/6!
    c = fma(c, z, 0.041666666666666664);          // 1/4!
    c = fma(c, z, -0.5);                          // 1/2!
    c = fma(c, z, 1.0);
    double s = 2.8114572543455206e-15;            // 1/17!
    s = fma(s, z, -7.647163731819816e-13);        // 1/15!
    s = fma(s, z, 1.6059043836821613e-10);        // 1/13!
    s = fma(s, z, -2.505210838544172e-08);        // 1/11!
    s = fma(s, z, 2.7557319223985893e-06);        // 1/9!
    s = fma(s, z, -0.0001984126984126984);        // 1/7!
    s = fma(s, z, 0.008333333333333333);          // 1/5!
    s = fma(s, z, -0.16666666666666666);          // 1/3!
    s = fma(s * z, r, r);
    // cos(k pi/2 + r) = cos r, -sin r, -cos r, sin r for k = 0, 1, 2, 3 (mod 4)
    const int q = (int)((long long)k & 3);
    const double v = (q & 1) ? s : c;
    return ((q + 1) & 2) ? -v : v;
}

// ---------------------------------------------------------------------------------------------
// Boris push (the leapfrog momentum update of the PIC cycle the step sits in, paper Fig. 7):
// half an electric kick, a rotation about B by the angle 2 atan(|hq B| / gamma^-) evaluated at
// the half-kicked momentum, and the second half kick; hq = q dt / 2 in the step's units (p in
// m c, t in 1/omega_r, E and B in m c omega_r / e).  p is updated in place.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void boris_push(double hq, double ex, double ey, double ez, double bx,
                                           double by, double bz, double& px, double& py,
                                           double& pz)
{
    const double mx = fma(hq, ex, px), my = fma(hq, ey, py), mz = fma(hq, ez, pz);
    const double gm = sqrt_nr(1.0 + fma(mx, mx, fma(my, my, mz * mz)));
    const double f = hq * rcp_nr(gm);
    const double tx = f * bx, ty = f * by, tz = f * bz;
    const double sf = 2.0 * rcp_nr(1.0 + fma(tx, tx, fma(ty, ty, tz * tz)));
    const double sx = sf * tx, sy = sf * ty, sz = sf * tz;
    // u' = u- + u- x t, then u+ = u- + u' x s
    const double rx = mx + (my * tz - mz * ty), ry = my + (mz * tx - mx * tz),
                 rz = mz + (mx * ty - my * tx);
    const double ux = mx + (ry * sz - rz * sy), uy = my + (rz * sx - rx * sz),
                 uz = mz + (rx * sy - ry * sx);
    px = fma(hq, ex, ux);
    py = fma(hq, ey, uy);
    pz = fma(hq, ez, uz);
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
#ifdef SFQ_CLENSHAW_GROUP
        if (k % SFQ_CLENSHAW_GROUP == 0) __builtin_amdgcn_sched_barrier(0);
#endif
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

// e^x for -708 < x <= 0: argument reduction x = n ln2 + r with |r| <= ln2/2 (Cody and Waite,
// with ln2 split into two doubles) and the Taylor series of e^r to degree 13 by Horner's rule
// (truncation below 1e-17); a few ulp.  Written out so that it needs few live registers.
__device__ __forceinline__ double exp_nonpos(double x)
{
    constexpr double LOG2E = 1.4426950408889634;
    constexpr double LN2_HI = 0.6931471805599453;
    constexpr double LN2_LO = 2.3190468138462996e-17;
    const double n = rint(x * LOG2E);
    const double r = fma(-n, LN2_LO, fma(-n, LN2_HI, x));
    double p = 1.0 / 6227020800.0;  // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)n);
}

__device__ __forceinline__ float exp_nonpos(float x) { return expf(x); }

// chi^a in single precision, for the two-term asymptotic rates beyond the tables (chi > 2^16),
// whose own truncation error there (~1e-6) is far above single-precision rounding
template <typename T>
__device__ __forceinline__ T pow_asym(T chi, float a)
{
    return T(exp2f(a * log2f((float)chi)));
}

// ---------------------------------------------------------------------------------------------
// Rates.  `rad` and `pair` point to the (LDS-staged) coefficient tables.
// ---------------------------------------------------------------------------------------------
// W~_rad(chi) (Sec. 4.1, Eq. (wtilde)); sets *ood when chi is beyond the tables.  trunc (the
// same in every lane): the leading RATE_DEG_TRUNC terms only.
template <typename T, typename P>
__device__ __forceinline__ T wtilde_rad(const P* rad, T chi, bool* ood, bool trunc)
{
    int seg;
    T X;
    if (chi_segment(chi, seg, X)) {
        *ood = true;
        return T(WRAD_ASYM_C1) * pow_asym(chi, -1.0f / 3.0f) - T(WRAD_ASYM_C2) / chi;
    }
    const P* c = rad + seg * RATE_DEG;
    return trunc ? clenshaw<RATE_DEG_TRUNC>(c, X) : clenshaw<RATE_DEG>(c, X);
}

// W~_pair(chi) (Sec. 4.2, Eq. (wtilde_pair)) for chi >= 2^PAIR_OCT_LO
template <typename T, typename P>
__device__ __forceinline__ T wtilde_pair(const P* pair, T chi, bool* ood, bool trunc)
{
    int seg;
    T X;
    if (pair_segment(chi, seg, X)) {
        *ood = true;
        return T(WPAIR_ASYM_C) * pow_asym(chi, 2.0f / 3.0f);
    }
    const P* c = pair + seg * RATE_DEG;
    const T P_ = trunc ? clenshaw<RATE_DEG_TRUNC>(c, X) : clenshaw<RATE_DEG>(c, X);
    return chi * P_ * exp_nonpos(T(-8.0 / 3.0) / chi);
}

// ---------------------------------------------------------------------------------------------
// Inverse-CDF tables: patches of 8 x 8 Chebyshev coefficients, row-major [r index][chi index],
// on quarter-octave segments of chi and of t = -ln(1 - r).  The local variable of a
// quarter-octave [2^o q_k, 2^o q_{k+1}) (q_k = 2^{k/4}) is X = (2m - q_k - q_{k+1})/(q_{k+1} - q_k)
// with m the mantissa in [1, 2): the segment is the exponent plus three comparisons.
// Lower region r <= 1/2 (or |r'| <= 1/2): N_LO_SEG equal segments, linear in r.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double subq(int k)
{
    return k == 0 ? 1.0 : k == 1 ? 1.189207115002721 : k == 2 ? 1.4142135623730951
         : k == 3 ? 1.681792830507429 : 2.0;
}

// octave o, quarter k and local variable X of x > 0
__device__ __forceinline__ void quarter_locate(double x, int& o, int& k, double& X)
{
    int e;
    const double m = 2.0 * frexp(x, &e);   // x = m 2^(e-1), m in [1, 2)
    o = e - 1;
    k = (m >= 1.189207115002721 ? 1 : 0) + (m >= 1.4142135623730951 ? 1 : 0) +
        (m >= 1.681792830507429 ? 1 : 0);
    const double a = subq(k), b = subq(k + 1);
    X = (2.0 * m - a - b) / (b - a);
}

// a request for one inverse-table evaluation: patch offset (same in the FP64 and FP32 tables)
// and local variables along r and chi
struct InvReq {
    int patch;     // index of the patch in its table
    double Xr, Xc;
    bool upper;    // upper region: the table holds a logarithm
    bool ood;      // chi beyond the table
};

__device__ __forceinline__ void r_locate(double r, int& seg, double& X, bool& upper)
{
    if (r <= 0.5) {
        int k = (int)(r * (2 * N_LO_SEG));
        k = k > N_LO_SEG - 1 ? N_LO_SEG - 1 : (k < 0 ? 0 : k);
        seg = k;
        X = fma(r, 4.0 * N_LO_SEG, -(2.0 * k + 1.0));
        upper = false;
        return;
    }
    const double t = -log(1.0 - r);  // 1 - r is exact for r >= 1/2
    int o, k;
    quarter_locate(t, o, k, X);
    if (o < T_OCT_LO) { o = T_OCT_LO; k = 0; X = -1.0; }          // not reached: t >= ln 2
    if (o > T_OCT_HI - 1) { o = T_OCT_HI - 1; k = SUB - 1; X = 1.0; }
    seg = N_LO_SEG + SUB * (o - T_OCT_LO) + k;
    upper = true;
}

// photon emission (inverse of Eq. (again)); u = r
__device__ __forceinline__ InvReq photon_req(double chi, double r)
{
    InvReq q;
    int cs;
    q.ood = false;
    if (chi < 0x1p-10) {
        cs = 0;
        q.Xc = fma(chi, 0x1p11, -1.0);
    } else {
        int o, k;
        quarter_locate(chi, o, k, q.Xc);
        cs = 1 + SUB * (o - INV_CHI_OCT_LO) + k;
        if (cs > N_INV_CHI - 1) { cs = N_INV_CHI - 1; q.Xc = 1.0; q.ood = true; }
    }
    int rs;
    r_locate(r, rs, q.Xr, q.upper);
    q.patch = cs * N_R_SEG + rs;
    return q;
}

// pair creation (inverse of Eq. (again_pp)); u = |r'| = |2r - 1|
__device__ __forceinline__ InvReq pair_req(double chi, double u)
{
    InvReq q;
    int o, k;
    quarter_locate(chi, o, k, q.Xc);
    int cs = SUB * (o - PAIR_OCT_LO) + k;
    q.ood = false;
    if (!(cs >= 0)) { cs = 0; q.Xc = -1.0; }
    if (cs > N_PAIR_INV_CHI - 1) { cs = N_PAIR_INV_CHI - 1; q.Xc = 1.0; q.ood = true; }
    int rs;
    r_locate(u, rs, q.Xr, q.upper);
    q.patch = cs * N_R_SEG + rs;
    return q;
}

// Chebyshev polynomial T_m(x) for 0 <= m < 8 by the three-term recurrence
template <typename T>
__device__ __forceinline__ T cheb_T(int m, T x)
{
    T t0 = T(1), t1 = x, out = m == 0 ? t0 : t1;
#pragma unroll
    for (int k = 2; k < 8; ++k) {
        const T t2 = fma(x + x, t1, -t0);
        out = (m == k) ? t2 : out;
        t0 = t1;
        t1 = t2;
    }
    return out;
}

// Position of the k-th set bit (k from 0) of mask, by binary search on popcounts.
__device__ __forceinline__ int kth_set_bit(unsigned long long mask, int k)
{
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const int c = __popcll(mask & ((1ull << w) - 1ull));
        if (k >= c) {
            k -= c;
            mask >>= w;
            pos += w;
        }
    }
    return pos;
}

// Cooperative evaluation of an 8 x 8 patch for every lane with `active` set.  In round b the
// eight lane groups of eight take the next eight active lanes (in lane order): lane m of a
// group loads column m of that lane's patch (eight lanes read a 64-byte row at once), runs
// Clenshaw along the r variable and weights by T_m(Xc), and the group sums its columns with
// xor shuffles.  A wave runs ceil(active lanes / 8) rounds (rounded up to even), so partly
// filled waves and rare re-evaluations cost only what they use.  Every lane of the wave must
// call it.
// With trunc (the same in every lane), the leading INV_TRUNC x INV_TRUNC coefficients: lanes
// m >= INV_TRUNC of a group load nothing and add zero.
template <typename T>
__device__ __forceinline__ T coop_patch_eval(const T* table, int patch, T Xr, T Xc, bool active,
                                             bool trunc)
{
    const int L = __lane_id();
    const int g = L >> 3, m = L & 7;
    const unsigned long long mask = __ballot(active);
    const int cnt = __popcll(mask);
    const int rank = __popcll(mask & ((1ull << L) - 1ull));
    const int first = cnt ? kth_set_bit(mask, 0) : 0;
    T result = T(0);
    // two rounds per trip, so that two column loads are in flight together
#pragma unroll 1
    for (int b = 0; 8 * b < cnt; b += 2) {
        const int k0 = 8 * b + g, k1 = k0 + 8;
        const int s0 = k0 < cnt ? kth_set_bit(mask, k0) : first;  // spare groups redo a lane
        const int s1 = k1 < cnt ? kth_set_bit(mask, k1) : first;
        const int p0 = __shfl(patch, s0), p1 = __shfl(patch, s1);
        const T xr0 = __shfl(Xr, s0), xc0 = __shfl(Xc, s0);
        const T xr1 = __shfl(Xr, s1), xc1 = __shfl(Xc, s1);
        const T* c0 = table + (size_t)p0 * INV_PATCH + m;
        const T* c1 = table + (size_t)p1 * INV_PATCH + m;
        T v0 = T(0), v1 = T(0);
        if (!trunc) {
            T col0[INV_NR], col1[INV_NR];
#pragma unroll
            for (int i = 0; i < INV_NR; ++i) {
                col0[i] = c0[i * INV_NC];
                col1[i] = c1[i * INV_NC];
            }
            v0 = clenshaw<INV_NR>(col0, xr0) * cheb_T(m, xc0);
            v1 = clenshaw<INV_NR>(col1, xr1) * cheb_T(m, xc1);
        } else if (m < INV_TRUNC) {
            T col0[INV_TRUNC], col1[INV_TRUNC];
#pragma unroll
            for (int i = 0; i < INV_TRUNC; ++i) {
                col0[i] = c0[i * INV_NC];
                col1[i] = c1[i * INV_NC];
            }
            v0 = clenshaw<INV_TRUNC>(col0, xr0) * cheb_T(m, xc0);
            v1 = clenshaw<INV_TRUNC>(col1, xr1) * cheb_T(m, xc1);
        }
        v0 += __shfl_xor(v0, 1);
        v1 += __shfl_xor(v1, 1);
        v0 += __shfl_xor(v0, 2);
        v1 += __shfl_xor(v1, 2);
        v0 += __shfl_xor(v0, 4);
        v1 += __shfl_xor(v1, 4);
        const T got0 = __shfl(v0, (rank & 7) << 3), got1 = __shfl(v1, (rank & 7) << 3);
        if (active && (rank >> 3) == b) result = got0;
        if (active && (rank >> 3) == b + 1) result = got1;
    }
    return result;
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
