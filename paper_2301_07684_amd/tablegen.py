"""Offline generator of the approximation tables used by the HIP kernels.

The kernels never evaluate Bessel functions or integrals: they evaluate piecewise Chebyshev
expansions (Clenshaw's recurrence, the paper's App. B) of smooth functions obtained by variable
and function transformations (the paper's Sec. 3), fitted here once at build time, in the
spirit of the paper's own coefficient generator (Sec. 3, item 1 of the Chebyshev properties).
The layout is MI355X-first and differs from the paper's: segments are octaves of chi (and of
the other variables) so that the segment index is the floating-point exponent, the functions
are chosen so that a fixed degree reaches ~1e-13 relative accuracy in every segment, and the
tails of the inverse distributions are expressed in t = -ln(1 - r) instead of exponential
closures.

Functions tabulated (all in normalised units; s = 3 chi w^3 / 2, eta0 = 8/(3 chi)):
  RAD   W~_rad(chi)                                   Sec. 4.1, Eq. (wtilde)
  PAIR  P(chi) = e^{eta0} W~_pair(chi) / chi          Sec. 4.2, Eq. (wtilde_pair)
  KA    w^2 K_{2/3}(w^3), Ki_{1/3}(w^3) for w^3 < 2   (Bessel pieces of Eq. (pe_dp))
  KB    e^x sqrt(x) K_{2/3}(x), e^x sqrt(x) Ki_{1/3}(x) for x >= 2
  PHL   wbar / r for r <= 1/2                         inverse of Eq. (again)
  PHU   ln(wbar^3), t = -ln(1-r), for r > 1/2         inverse of Eq. (again), upper tail
  PPL   sqrt(y) / q for q = |2r-1| <= 1/2              inverse of Eq. (again_pp),
  PPU   y - t, t = -ln(1-q), for q > 1/2              y = eta0 v^2/(1 - v^2)

Bessel values come from scipy.special.kve (AMOS); the tail integral Ki_{1/3} and every CDF are
integrated here with composite Gauss-Legendre rules.  This module is independent of the test
oracle: it shares no code with it and is never used at run time.
"""
from __future__ import annotations

import hashlib
import math
import os
import struct
import sys
import time

import numpy as np
from scipy import special as sp

# ------------------------------------------------------------------------------------------------
# Table geometry.  Must match the constants compiled into the HIP library (sfq_tables.h).
# ------------------------------------------------------------------------------------------------
RATE_DEG = 16          # Chebyshev terms per rate segment
CHI_OCT_LO = -6        # first chi octave [2^-6, 2^-5); chi < 2^-6 is the linear segment 0
CHI_OCT_HI = 16        # last octave ends at 2^16
N_CHI_SEG = 1 + (CHI_OCT_HI - CHI_OCT_LO)   # 23 segments
PAIR_OCT_LO = -7       # pair rate table starts at chi = 2^-7 (< 0.01 cutoff)
N_PAIR_SEG = CHI_OCT_HI - PAIR_OCT_LO       # 23 octaves

KA_DEG = 20            # w in [0, 2^{1/3}): N_KA segments of equal width in w
N_KA = 4
KB_DEG = 18            # x in [2^1, 2^18): one segment per octave
KB_OCT_LO, KB_OCT_HI = 1, 18

# 2D inverse-CDF tables: [chi segment][r segment][N_R][N_C] patches of 8 x 8 coefficients
# (512 bytes, one patch = four 128-byte cache lines).  Segments are quarter-octaves of chi and
# of t = -ln(1 - r): the segment index is the floating-point exponent plus three comparisons
# of the mantissa with 2^{1/4}, 2^{1/2}, 2^{3/4}.
INV_NC = 8             # Chebyshev terms along chi (per chi segment)
INV_NR = 8             # Chebyshev terms along the r variable (per r segment)
SUB = 4                # sub-segments per octave
SUBQ = (1.0, 1.189207115002721, 1.4142135623730951, 1.681792830507429, 2.0)  # 2^{k/4}
INV_CHI_OCT_LO = -10   # photon inverse: chi < 2^-10 is the linear segment 0
N_INV_CHI = 1 + SUB * (CHI_OCT_HI - INV_CHI_OCT_LO)
N_PAIR_INV_CHI = SUB * (CHI_OCT_HI - PAIR_OCT_LO)   # pair inverse: quarter-octaves from 2^-7
N_LO_SEG = 8           # lower region r (or q) in (0, 1/2]: 8 equal segments in r
T_OCT_LO, T_OCT_HI = -1, 6   # upper region t in [2^-1, 2^6): quarter-octaves of t
N_HI_SEG = SUB * (T_OCT_HI - T_OCT_LO)
N_R_SEG = N_LO_SEG + N_HI_SEG
T_MAX = 2.0 ** T_OCT_HI

MAGIC = b"SFQTAB03"

# The truncated evaluation form (the accuracy/speed dial, the analogue of the paper's choice of
# coefficient counts, Sec. 4.5): the kernels may evaluate only the leading RATE_DEG_TRUNC terms
# of every rate segment and the leading INV_TRUNC x INV_TRUNC coefficients of every inverse
# patch.  The same tables serve both forms; the errors of each form are measured below.
RATE_DEG_TRUNC = 10
INV_TRUNC = 5


# ------------------------------------------------------------------------------------------------
# Chebyshev utilities (first-kind nodes; coefficients with c_0 already halved, so that
# f(x) = sum_k c_k T_k(X) with X = (2x - a - b)/(b - a), as in the paper's Eq. (f_approx)).
# ------------------------------------------------------------------------------------------------
def cheb_nodes(n):
    k = np.arange(n)
    return np.cos(np.pi * (k + 0.5) / n)


def cheb_coeffs_from_values(vals, axis=-1):
    """vals sampled at cheb_nodes(n) along `axis` -> coefficients along that axis."""
    vals = np.moveaxis(np.asarray(vals, dtype=np.float64), axis, -1)
    n = vals.shape[-1]
    k = np.arange(n)
    T = np.cos(np.outer(k, np.pi * (k + 0.5) / n))  # T[j, node]
    c = (2.0 / n) * vals @ T.T
    c[..., 0] *= 0.5
    return np.moveaxis(c, -1, axis)


def cheb_eval(c, X):
    """Clenshaw's recurrence (paper App. B) for coefficient vectors c[..., n] at X (broadcast),
    in the floating-point type of c and X (float64, or float32 to measure the FP32 form)."""
    dt = np.result_type(c, X)
    X = np.asarray(X, dtype=dt)
    b1 = np.zeros(np.broadcast(X, c[..., 0]).shape, dtype=dt)
    b2 = np.zeros_like(b1)
    two = dt.type(2.0)
    for k in range(c.shape[-1] - 1, 0, -1):
        b1, b2 = two * X * b1 - b2 + c[..., k], b1
    return X * b1 - b2 + c[..., 0]


def truncate_rates(tab):
    """A rate table with only its leading RATE_DEG_TRUNC terms per segment (the rest zero: the
    same values as a recurrence over the leading terms)."""
    t = np.array(tab, dtype=np.float64)
    t[..., RATE_DEG_TRUNC:] = 0.0
    return t


def truncate_patches(tab):
    """An inverse table with only the leading INV_TRUNC x INV_TRUNC coefficients per patch."""
    t = np.array(tab, dtype=np.float64)
    t[..., INV_TRUNC:, :] = 0.0
    t[..., :, INV_TRUNC:] = 0.0
    return t


def to_unit(x, a, b):
    return (2.0 * x - a - b) / (b - a)


# ------------------------------------------------------------------------------------------------
# Gauss-Legendre rules
# ------------------------------------------------------------------------------------------------
_GL = {}


def gl(n):
    if n not in _GL:
        _GL[n] = np.polynomial.legendre.leggauss(n)
    return _GL[n]


def gl_panels(edges, n):
    """Nodes and weights of composite GL over consecutive edges; returns (x, w) flat arrays."""
    x0, w0 = gl(n)
    a, b = edges[:-1, None], edges[1:, None]
    x = 0.5 * (a + b) + 0.5 * (b - a) * x0[None, :]
    w = 0.5 * (b - a) * w0[None, :]
    return x, w


# ------------------------------------------------------------------------------------------------
# Bessel pieces: K_{2/3} from AMOS; Ki_{1/3}(x) = int_x^inf K_{1/3} by composite GL.
# ------------------------------------------------------------------------------------------------
def ki13_exact(x):
    """int_x^inf K_{1/3}(t) dt for an array of x >= 0 (absolute values, not scaled)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    big = x >= 2.0
    # x >= 2: t = x + s, e^{-s} kve(x+s) panels on s in [0, 60]
    if np.any(big):
        xb = x[big]
        edges = np.array([0, 0.25, 0.5, 1, 1.5, 2, 3, 4, 6, 8, 11, 15, 20, 28, 38, 50, 65.0])
        s, w = gl_panels(edges, 24)
        s, w = s.ravel(), w.ravel()
        vals = sp.kve(1.0 / 3.0, xb[:, None] + s[None, :]) * np.exp(-s)[None, :]
        out[big] = np.exp(-xb) * (vals @ w)
    if np.any(~big):
        # Ki(x) = Ki(2) + int_{x^{1/3}}^{2^{1/3}} 3u^2 K_{1/3}(u^3) du   (analytic integrand in u)
        xs = x[~big]
        ki2 = ki13_exact(np.array([2.0]))[0]
        u0 = np.cbrt(xs)
        u1 = 2.0 ** (1.0 / 3.0)
        xg, wg = gl(40)
        # split [u0, u1] in 4 pieces for safety
        tot = np.zeros_like(xs)
        for p in range(4):
            a = u0 + (u1 - u0) * p / 4.0
            b = u0 + (u1 - u0) * (p + 1) / 4.0
            u = 0.5 * (a + b)[:, None] + 0.5 * (b - a)[:, None] * xg[None, :]
            f = 3.0 * u * u * sp.kv(1.0 / 3.0, u ** 3)
            tot += 0.5 * (b - a) * (f @ wg)
        out[~big] = ki2 + tot
    return out


def ki13_scaled_exact(x):
    """e^x int_x^inf K_{1/3}(t) dt for an array of x >= 2."""
    x = np.asarray(x, dtype=np.float64)
    edges = np.array([0, 0.25, 0.5, 1, 1.5, 2, 3, 4, 6, 8, 11, 15, 20, 28, 38, 50, 65.0])
    s, w = gl_panels(edges, 24)
    s, w = s.ravel(), w.ravel()
    vals = sp.kve(1.0 / 3.0, x[:, None] + s[None, :]) * np.exp(-s)[None, :]
    return vals @ w


def k23_exact(x):
    return sp.kv(2.0 / 3.0, np.asarray(x, dtype=np.float64))


class BesselTables:
    """Piecewise Chebyshev representations of K_{2/3} and Ki_{1/3} (see module docstring)."""

    WS = 2.0 ** (1.0 / 3.0)

    def __init__(self):
        nd = cheb_nodes(KA_DEG)
        self.ka = np.zeros((N_KA, 2, KA_DEG))
        for s in range(N_KA):
            a, b = self.WS * s / N_KA, self.WS * (s + 1) / N_KA
            w = 0.5 * (a + b) + 0.5 * (b - a) * nd
            x = w ** 3
            self.ka[s, 0] = cheb_coeffs_from_values(w * w * k23_exact(x))
            self.ka[s, 1] = cheb_coeffs_from_values(ki13_exact(x))
        nb = cheb_nodes(KB_DEG)
        self.kb = np.zeros((KB_OCT_HI - KB_OCT_LO, 2, KB_DEG))
        for o in range(KB_OCT_LO, KB_OCT_HI):
            a, b = 2.0 ** o, 2.0 ** (o + 1)
            x = 0.5 * (a + b) + 0.5 * (b - a) * nb
            sq = np.sqrt(x)
            self.kb[o - KB_OCT_LO, 0] = cheb_coeffs_from_values(sq * sp.kve(2.0 / 3.0, x))
            self.kb[o - KB_OCT_LO, 1] = cheb_coeffs_from_values(sq * ki13_scaled_exact(x))

    def eval_scaled(self, x):
        """(e^x K_{2/3}(x), e^x Ki_{1/3}(x)) for an array 0 < x < 2^KB_OCT_HI."""
        x = np.asarray(x, dtype=np.float64)
        k, ki = np.zeros_like(x), np.zeros_like(x)
        small = x < 2.0
        if np.any(small):
            k0, ki0 = self.eval(x[small])
            e = np.exp(x[small])
            k[small], ki[small] = k0 * e, ki0 * e
        big = ~small
        if np.any(big):
            xm = x[big]
            o = np.clip(np.floor(np.log2(xm)).astype(int), KB_OCT_LO, KB_OCT_HI - 1)
            a = 2.0 ** o
            X = to_unit(xm, a, 2 * a)
            c = self.kb[o - KB_OCT_LO]
            sq = 1.0 / np.sqrt(xm)
            k[big] = sq * cheb_eval(c[:, 0], X)
            ki[big] = sq * cheb_eval(c[:, 1], X)
        return k, ki

    def eval(self, x):
        """(K_{2/3}(x), Ki_{1/3}(x)) for an array x > 0 via the tables."""
        x = np.asarray(x, dtype=np.float64)
        k, ki = np.zeros_like(x), np.zeros_like(x)
        small = x < 2.0
        if np.any(small):
            w = np.cbrt(x[small])
            seg = np.minimum((w / self.WS * N_KA).astype(int), N_KA - 1)
            a = self.WS * seg / N_KA
            X = to_unit(w, a, a + self.WS / N_KA)
            c = self.ka[seg]
            k[small] = cheb_eval(c[:, 0], X) / (w * w)
            ki[small] = cheb_eval(c[:, 1], X)
        mid = (~small) & (x < 2.0 ** KB_OCT_HI)
        if np.any(mid):
            xm = x[mid]
            o = np.floor(np.log2(xm)).astype(int)
            o = np.clip(o, KB_OCT_LO, KB_OCT_HI - 1)
            a = 2.0 ** o
            X = to_unit(xm, a, 2 * a)
            c = self.kb[o - KB_OCT_LO]
            sc = np.exp(-xm) / np.sqrt(xm)
            k[mid] = sc * cheb_eval(c[:, 0], X)
            ki[mid] = sc * cheb_eval(c[:, 1], X)
        return k, ki


# ------------------------------------------------------------------------------------------------
# Rates
# ------------------------------------------------------------------------------------------------
def wrad_exact(chi):
    """W~_rad(chi) = int_0^inf R(v chi) K_{2/3}(v) dv, v = t^3, composite GL in t."""
    chi = np.atleast_1d(np.asarray(chi, dtype=np.float64))
    out = np.empty_like(chi)
    tmax = 700.0 ** (1.0 / 3.0)
    for i, c in enumerate(chi):
        # the rational factor changes at v ~ 1/chi, i.e. t ~ chi^{-1/3}: geometric panels there
        tc = min(1.0, (1.0 / max(c, 1e-12)) ** (1.0 / 3.0))
        e1 = tc * np.geomspace(1e-3, 1.0, 25)
        edges = np.unique(np.concatenate([[0.0], e1, np.linspace(tc, 2.0, 20),
                                          np.linspace(2.0, tmax, 30)]))
        t, w = gl_panels(edges, 16)
        v = t ** 3
        vc = v * c
        rat = (45.0 * vc * vc + 42.0 * vc + 20.0) / (2.0 + 3.0 * vc) ** 3
        f = rat * k23_exact(v) * 3.0 * t * t
        out[i] = np.sum(f * w)
    return out


def pair_scaled_exact(chi):
    """e^{eta0} W~_pair(chi), eta0 = 8/(3chi):  int_0^1 (9-v^2)/(3(1-v^2)) e^{-(eta-eta0)} kve(eta)."""
    chi = np.atleast_1d(np.asarray(chi, dtype=np.float64))
    out = np.empty_like(chi)
    for i, c in enumerate(chi):
        eta0 = 8.0 / (3.0 * c)
        wd = min(1.0, 1.0 / math.sqrt(eta0))  # width of the distribution in v
        e = np.concatenate([np.linspace(0, min(1.0, 12 * wd), 40), [1.0]])
        if 12 * wd < 1:
            e = np.concatenate([e[:-1], np.linspace(12 * wd, 1.0, 10)])
        e = np.unique(np.concatenate([e, 1 - np.geomspace(1e-9, 0.3, 20)]))
        e = e[(e >= 0) & (e <= 1)]
        v, w = gl_panels(e, 16)
        om = 1.0 - v * v
        d = eta0 * v * v / om                       # eta - eta0
        ok = d < 700.0                              # beyond: the integrand underflows
        eta = np.where(ok, eta0 / om, 1.0)
        f = np.where(ok, (9.0 - v * v) / (3.0 * om) * np.exp(-np.where(ok, d, 0.0)) *
                     sp.kve(2.0 / 3.0, eta), 0.0)
        out[i] = np.sum(f * w)
    return out


def _chi_segment_bounds(seg):
    if seg == 0:
        return 0.0, 2.0 ** CHI_OCT_LO
    o = CHI_OCT_LO + seg - 1
    return 2.0 ** o, 2.0 ** (o + 1)


def build_rate_tables():
    nd = cheb_nodes(RATE_DEG)
    rad = np.zeros((N_CHI_SEG, RATE_DEG))
    for s in range(N_CHI_SEG):
        a, b = _chi_segment_bounds(s)
        chi = 0.5 * (a + b) + 0.5 * (b - a) * nd
        rad[s] = cheb_coeffs_from_values(wrad_exact(chi))
    pair = np.zeros((N_PAIR_SEG, RATE_DEG))
    for s in range(N_PAIR_SEG):
        a = 2.0 ** (PAIR_OCT_LO + s)
        chi = 1.5 * a + 0.5 * a * nd
        pair[s] = cheb_coeffs_from_values(pair_scaled_exact(chi) / chi)
    return rad, pair


def eval_rad(rad, chi, dtype=np.float64):
    chi = np.asarray(chi, dtype=np.float64)
    seg = np.where(chi < 2.0 ** CHI_OCT_LO, 0,
                   np.floor(np.log2(np.maximum(chi, 1e-300))).astype(int) - CHI_OCT_LO + 1)
    seg = np.clip(seg, 0, N_CHI_SEG - 1)
    a = np.where(seg == 0, 0.0, 2.0 ** (seg - 1 + CHI_OCT_LO))
    b = np.where(seg == 0, 2.0 ** CHI_OCT_LO, 2 * a)
    return cheb_eval(rad[seg].astype(dtype), to_unit(chi, a, b).astype(dtype))


def eval_pair_scaled(pair, chi, dtype=np.float64):
    chi = np.asarray(chi, dtype=np.float64)
    o = np.clip(np.floor(np.log2(chi)).astype(int), PAIR_OCT_LO, CHI_OCT_HI - 1)
    a = 2.0 ** o
    return chi.astype(dtype) * cheb_eval(pair[o - PAIR_OCT_LO].astype(dtype),
                                         to_unit(chi, a, 2 * a).astype(dtype))


# ------------------------------------------------------------------------------------------------
# Photon spectrum in w and its inverse
# ------------------------------------------------------------------------------------------------
class PhotonSpectrum:
    """dI~_pe/dw (paper Eq. (pe_eff_int_2)) for one chi, with a panel CDF and its inverse."""

    EDGES = np.unique(np.concatenate([[0.0], np.geomspace(1e-6, 0.05, 30),
                                      np.linspace(0.05, 3.0, 120), np.linspace(3.0, 4.4, 30)]))

    def __init__(self, bt: BesselTables, chi: float):
        self.bt, self.chi = bt, float(chi)
        x, w = gl_panels(self.EDGES, 16)
        f = self.pdf(x)
        pan = np.sum(f * w, axis=1)
        self.lower = np.concatenate([[0.0], np.cumsum(pan)])              # CDF at edges
        self.upper = np.concatenate([np.cumsum(pan[::-1])[::-1], [0.0]])  # tail at edges
        self.total = self.upper[0]

    def pdf(self, w):
        w = np.asarray(w, dtype=np.float64)
        x = w ** 3
        s = 1.5 * self.chi * x
        op = 1.0 + s
        k, ki = self.bt.eval(np.maximum(x, 1e-300))
        return 9.0 * w * w / (2.0 * op ** 3) * ((1.0 + op * op) * k - op * ki)

    def _partial(self, a, b, n=24):
        xg, wg = gl(n)
        m, h = 0.5 * (a + b), 0.5 * (b - a)
        pts = m[:, None] + h[:, None] * xg[None, :]
        return h * (self.pdf(pts) @ wg)

    def inverse(self, r, upper_form):
        """wbar solving CDF = r W~ (lower form) or tail = (1-r) W~ (upper form).
        For the upper form pass omr = 1 - r instead of r."""
        r = np.asarray(r, dtype=np.float64)
        E = self.EDGES
        if not upper_form:
            L = r * self.total
            j = np.clip(np.searchsorted(self.lower, L, side="right") - 1, 0, E.size - 2)
            base = L - self.lower[j]
            a = E[j]
            wv = a + (E[j + 1] - a) * np.clip(base / (self.lower[j + 1] - self.lower[j]), 0, 1)
            for _ in range(40):
                g = self._partial(a, wv) - base
                step = g / self.pdf(wv)
                wv = np.clip(wv - step, a, E[j + 1])
                if np.all(np.abs(step) <= 1e-16 * wv):
                    break
            return wv
        U = r * self.total
        j = np.clip(np.searchsorted(-self.upper, -U, side="left") - 1, 0, E.size - 2)
        # upper[j] >= U > upper[j+1]
        base = U - self.upper[j + 1]
        b = E[j + 1]
        wv = E[j] + (b - E[j]) * np.clip(1 - base / (self.upper[j] - self.upper[j + 1]), 0, 1)
        for _ in range(40):
            g = self._partial(wv, b) - base
            step = -g / self.pdf(wv)
            wv = np.clip(wv - step, E[j], b)
            if np.all(np.abs(step) <= 1e-16 * wv):
                break
        return wv


def photon_xbar(bt, chi, rvar, region):
    """Exact inverse for one chi: region 'L' -> rvar = r, returns wbar/r;
    region 'U' -> rvar = t = -ln(1-r), returns wbar^3 - t."""
    ps = PhotonSpectrum(bt, chi)
    if region == "L":
        return ps.inverse(rvar, False) / rvar
    omr = np.exp(-rvar)
    wb = ps.inverse(omr, True)
    return wb ** 3 - rvar


def _quarter(o, k):
    """[2^o 2^{k/4}, 2^o 2^{(k+1)/4})"""
    return math.ldexp(SUBQ[k], o), math.ldexp(SUBQ[k + 1], o)


def _r_segment_bounds(seg):
    """Lower segments: r in [seg/16, (seg+1)/16); upper: quarter-octaves of t = -ln(1-r)."""
    if seg < N_LO_SEG:
        return "L", 0.5 * seg / N_LO_SEG, 0.5 * (seg + 1) / N_LO_SEG
    h = seg - N_LO_SEG
    a, b = _quarter(T_OCT_LO + h // SUB, h % SUB)
    return "U", a, b


def _inv_chi_segment_bounds(seg):
    if seg == 0:
        return 0.0, 2.0 ** INV_CHI_OCT_LO
    h = seg - 1
    return _quarter(INV_CHI_OCT_LO + h // SUB, h % SUB)


def _pair_inv_chi_segment_bounds(seg):
    return _quarter(PAIR_OCT_LO + seg // SUB, seg % SUB)


def _sub_of_mantissa(m):
    """index of the quarter-octave of a mantissa m in [1, 2)"""
    return ((m >= SUBQ[1]).astype(int) + (m >= SUBQ[2]).astype(int) + (m >= SUBQ[3]).astype(int))


def _quarter_locate(x):
    """(octave, sub-segment, X) of positive x, X the local variable of the quarter-octave."""
    m2, e = np.frexp(x)
    o = e - 1
    m = 2.0 * m2
    k = _sub_of_mantissa(m)
    a = np.array(SUBQ)[k]
    b = np.array(SUBQ)[k + 1]
    return o, k, (2.0 * m - a - b) / (b - a)


def build_photon_inverse(bt, verbose=False):
    ndc, ndr = cheb_nodes(INV_NC), cheb_nodes(INV_NR)
    tab = np.zeros((N_INV_CHI, N_R_SEG, INV_NR, INV_NC))
    for cs in range(N_INV_CHI):
        ca, cb = _inv_chi_segment_bounds(cs)
        chis = 0.5 * (ca + cb) + 0.5 * (cb - ca) * ndc
        vals = np.zeros((N_R_SEG, INV_NR, INV_NC))
        for j, chi in enumerate(chis):
            ps = PhotonSpectrum(bt, max(chi, 1e-300))
            for rs in range(N_R_SEG):
                reg, a, b = _r_segment_bounds(rs)
                xv = 0.5 * (a + b) + 0.5 * (b - a) * ndr
                if reg == "L":
                    vals[rs, :, j] = ps.inverse(xv, False) / xv
                else:
                    wb = ps.inverse(np.exp(-xv), True)
                    vals[rs, :, j] = 3.0 * np.log(wb)
        c = cheb_coeffs_from_values(vals, axis=1)
        tab[cs] = cheb_coeffs_from_values(c, axis=2)
        if verbose:
            print(f"  photon inverse: chi segment {cs + 1}/{N_INV_CHI}", flush=True)
    return tab


def chi_segment(chi):
    """segment and local variable of chi in the photon inverse table"""
    chi = np.asarray(chi, dtype=np.float64)
    low = chi < 2.0 ** INV_CHI_OCT_LO
    o, k, X = _quarter_locate(np.where(low, 1.0, chi))
    seg = 1 + SUB * (o - INV_CHI_OCT_LO) + k
    over = seg > N_INV_CHI - 1
    seg = np.where(over, N_INV_CHI - 1, seg)
    X = np.where(over, 1.0, X)
    Xl = chi * 2.0 ** (1 - INV_CHI_OCT_LO) - 1.0
    return np.where(low, 0, seg), np.where(low, Xl, X)


def r_segment(r):
    """(segment, local variable X, is_upper, t) for an array of r in (0, 1)."""
    r = np.asarray(r, dtype=np.float64)
    upper = r > 0.5
    t = -np.log1p(-np.where(upper, r, 0.0))
    segl = np.minimum((r * 2 * N_LO_SEG).astype(int), N_LO_SEG - 1)
    al = 0.5 * segl / N_LO_SEG
    Xl = to_unit(r, al, al + 0.5 / N_LO_SEG)
    o, k, Xu = _quarter_locate(np.where(upper, t, 1.0))
    o = np.clip(o, T_OCT_LO, T_OCT_HI - 1)
    seg = np.where(upper, N_LO_SEG + SUB * (o - T_OCT_LO) + k, segl)
    X = np.where(upper, Xu, Xl)
    return seg, X, upper, t


def eval_inverse_2d(tab, chi, r, dtype=np.float64):
    """Evaluate a [chi seg][r seg][NR][NC] table: returns the tabulated function value."""
    cs, Xc = chi_segment(chi)
    rs, Xr, up, t = r_segment(r)
    c = tab[cs, rs].astype(dtype)                     # (n, NR, NC)
    d = cheb_eval(c, Xc[:, None].astype(dtype))       # inner along chi -> (n, NR)
    return cheb_eval(d, Xr.astype(dtype)), up, t


def eval_photon_xbar(tab, chi, r, dtype=np.float64):
    """wbar^3 from the photon table."""
    f, up, t = eval_inverse_2d(tab, chi, r, dtype)
    r = np.asarray(r, dtype=np.float64).astype(dtype)
    return np.where(up, np.exp(f), (f * r) ** 3)


# ------------------------------------------------------------------------------------------------
# Pair spectrum in u = sqrt(y), y = eta0 v^2/(1 - v^2) = eta_v - eta0, and its inverse.
# With v^2 = u^2/(u^2 + eta0) and dv/du = eta0/(u^2 + eta0)^{3/2}, the scaled integrand of
# Eq. (tilde_I_pp) times dv/du is
#   g(u) = e^{-u^2} (u^2 + eta0)^{-3/2} [2 (2u^2 + eta0) Ks(eta) + eta0 Kis(eta)],
# eta = eta0 + u^2, Ks = e^x K_{2/3}, Kis = e^x Ki_{1/3}: smooth on [0, inf).
# ------------------------------------------------------------------------------------------------
class PairSpectrum:
    def __init__(self, bt: BesselTables, chi: float):
        self.bt, self.chi = bt, float(chi)
        self.eta0 = 8.0 / (3.0 * self.chi)
        s0 = math.sqrt(self.eta0)
        e = [np.array([0.0]), s0 * np.geomspace(1e-4, 1.0, 30), np.linspace(0.0, 9.5, 160)]
        if s0 < 9.0:
            e.append(np.geomspace(s0, 9.5, 40))
        e = np.concatenate(e)
        e = e[e <= 9.5]
        self.edges = np.unique(e)
        x, w = gl_panels(self.edges, 16)
        pan = np.sum(self.pdf(x) * w, axis=1)
        self.lower = np.concatenate([[0.0], np.cumsum(pan)])
        self.upper = np.concatenate([np.cumsum(pan[::-1])[::-1], [0.0]])
        self.total = self.upper[0]

    def pdf(self, u):
        u = np.asarray(u, dtype=np.float64)
        y = u * u
        eta = self.eta0 + y
        ks, kis = self.bt.eval_scaled(np.minimum(eta, 2.0 ** KB_OCT_HI * 0.999))
        g = np.exp(-y) * (2.0 * (2.0 * y + self.eta0) * ks + self.eta0 * kis) / (y + self.eta0) ** 1.5
        return np.where(y < 700.0, g, 0.0)

    def _partial(self, a, b, n=24):
        xg, wg = gl(n)
        m, h = 0.5 * (a + b), 0.5 * (b - a)
        pts = m[:, None] + h[:, None] * xg[None, :]
        return h * (self.pdf(pts) @ wg)

    def inverse(self, q, upper_form):
        """ubar with CDF = q * total (lower form) or tail = q * total (upper form, q = 1 - |r'|)."""
        q = np.asarray(q, dtype=np.float64)
        E = self.edges
        if not upper_form:
            L = q * self.total
            j = np.clip(np.searchsorted(self.lower, L, side="right") - 1, 0, E.size - 2)
            base = L - self.lower[j]
            a = E[j]
            u = a + (E[j + 1] - a) * np.clip(base / (self.lower[j + 1] - self.lower[j]), 0, 1)
            for _ in range(50):
                step = (self._partial(a, u) - base) / self.pdf(u)
                u = np.clip(u - step, a, E[j + 1])
                if np.all(np.abs(step) <= 1e-16 * u):
                    break
            return u
        U = q * self.total
        j = np.clip(np.searchsorted(-self.upper, -U, side="left") - 1, 0, E.size - 2)
        base = U - self.upper[j + 1]
        b = E[j + 1]
        u = E[j] + (b - E[j]) * np.clip(1 - base / (self.upper[j] - self.upper[j + 1]), 0, 1)
        for _ in range(50):
            step = -(self._partial(u, b) - base) / self.pdf(u)
            u = np.clip(u - step, E[j], b)
            if np.all(np.abs(step) <= 1e-16 * u):
                break
        return u


def build_pair_inverse(bt, verbose=False):
    ndc, ndr = cheb_nodes(INV_NC), cheb_nodes(INV_NR)
    tab = np.zeros((N_PAIR_INV_CHI, N_R_SEG, INV_NR, INV_NC))
    for cs in range(N_PAIR_INV_CHI):
        ca, cb = _pair_inv_chi_segment_bounds(cs)
        chis = 0.5 * (ca + cb) + 0.5 * (cb - ca) * ndc
        vals = np.zeros((N_R_SEG, INV_NR, INV_NC))
        for j, chi in enumerate(chis):
            ps = PairSpectrum(bt, chi)
            for rs in range(N_R_SEG):
                reg, a, b = _r_segment_bounds(rs)
                xv = 0.5 * (a + b) + 0.5 * (b - a) * ndr
                if reg == "L":
                    vals[rs, :, j] = ps.inverse(xv, False) / xv
                else:
                    vals[rs, :, j] = 2.0 * np.log(ps.inverse(np.exp(-xv), True))
        c = cheb_coeffs_from_values(vals, axis=1)
        tab[cs] = cheb_coeffs_from_values(c, axis=2)
        if verbose:
            print(f"  pair inverse: chi segment {cs + 1}/{N_PAIR_INV_CHI}", flush=True)
    return tab


def pair_chi_segment(chi):
    chi = np.asarray(chi, dtype=np.float64)
    o, k, X = _quarter_locate(chi)
    seg = SUB * (o - PAIR_OCT_LO) + k
    lo, hi = seg < 0, seg > N_PAIR_INV_CHI - 1
    seg = np.clip(seg, 0, N_PAIR_INV_CHI - 1)
    X = np.where(lo, -1.0, np.where(hi, 1.0, X))
    return seg, X


def eval_pair_y(tab, chi, r, dtype=np.float64):
    """y = eta_v - eta0 for the pair sample with uniform r (r' = 2r - 1, q = |r'|)."""
    chi, r = np.asarray(chi, dtype=np.float64), np.asarray(r, dtype=np.float64)
    q = np.abs(2.0 * r - 1.0)
    cs, Xc = pair_chi_segment(chi)
    rs, Xr, up, t = r_segment(q)
    d = cheb_eval(tab[cs, rs].astype(dtype), Xc[:, None].astype(dtype))
    f = cheb_eval(d, Xr.astype(dtype))
    qd = q.astype(dtype)
    return np.where(up, np.exp(f), (f * qd) ** 2)


def photon_sample_forms(tab, chi, r):
    """wbar^3 as each evaluation form gives it: FP64 or FP32 arithmetic (the FP32 form re-
    evaluating in FP64 where the energy fraction exceeds 0.999, s = 3 chi wbar^3/2 > 999, as
    the kernels do), full or truncated patches."""
    out = {}
    for trunc in (False, True):
        t = truncate_patches(tab) if trunc else tab
        x64 = eval_photon_xbar(t, chi, r)
        x32 = eval_photon_xbar(t, chi, r, np.float32).astype(np.float64)
        s32 = 1.5 * np.asarray(chi) * x32
        out[("fp64", trunc)] = x64
        out[("mixed", trunc)] = np.where(s32 > 999.0, x64, x32)
    return out


def pair_sample_forms(tab, chi, r):
    """y as each evaluation form gives it (the FP32 form re-evaluating in FP64 where
    v = sqrt(y/(y + eta0)) exceeds 0.998)."""
    out = {}
    eta0 = 8.0 / (3.0 * np.asarray(chi, dtype=np.float64))
    for trunc in (False, True):
        t = truncate_patches(tab) if trunc else tab
        y64 = eval_pair_y(t, chi, r)
        y32 = eval_pair_y(t, chi, r, np.float32).astype(np.float64)
        v32 = np.sqrt(y32 / (y32 + eta0))
        out[("fp64", trunc)] = y64
        out[("mixed", trunc)] = np.where(v32 > 0.998, y64, y32)
    return out


# ------------------------------------------------------------------------------------------------
# Build, self-check and write the table blob
# ------------------------------------------------------------------------------------------------
GEOMETRY = ("RATE_DEG", "CHI_OCT_LO", "CHI_OCT_HI", "N_CHI_SEG", "PAIR_OCT_LO", "N_PAIR_SEG",
            "KA_DEG", "N_KA", "KB_DEG", "KB_OCT_LO", "KB_OCT_HI", "INV_NC", "INV_NR", "N_LO_SEG",
            "T_OCT_LO", "T_OCT_HI", "N_HI_SEG", "N_R_SEG", "SUB", "INV_CHI_OCT_LO", "N_INV_CHI",
            "N_PAIR_INV_CHI", "RATE_DEG_TRUNC", "INV_TRUNC")


def source_hash() -> int:
    with open(os.path.abspath(__file__), "rb") as f:
        return int.from_bytes(hashlib.sha256(f.read()).digest()[:8], "little")


def _photon_segment(cs):
    bt = BesselTables()
    ndc, ndr = cheb_nodes(INV_NC), cheb_nodes(INV_NR)
    ca, cb = _inv_chi_segment_bounds(cs)
    chis = 0.5 * (ca + cb) + 0.5 * (cb - ca) * ndc
    vals = np.zeros((N_R_SEG, INV_NR, INV_NC))
    for j, chi in enumerate(chis):
        ps = PhotonSpectrum(bt, chi)
        for rs in range(N_R_SEG):
            reg, a, b = _r_segment_bounds(rs)
            xv = 0.5 * (a + b) + 0.5 * (b - a) * ndr
            if reg == "L":
                vals[rs, :, j] = ps.inverse(xv, False) / xv
            else:
                vals[rs, :, j] = 3.0 * np.log(ps.inverse(np.exp(-xv), True))
    c = cheb_coeffs_from_values(vals, axis=1)
    return cheb_coeffs_from_values(c, axis=2)


def _pair_segment(cs):
    bt = BesselTables()
    ndc, ndr = cheb_nodes(INV_NC), cheb_nodes(INV_NR)
    ca, cb = _pair_inv_chi_segment_bounds(cs)
    chis = 0.5 * (ca + cb) + 0.5 * (cb - ca) * ndc
    vals = np.zeros((N_R_SEG, INV_NR, INV_NC))
    for j, chi in enumerate(chis):
        ps = PairSpectrum(bt, chi)
        for rs in range(N_R_SEG):
            reg, a, b = _r_segment_bounds(rs)
            xv = 0.5 * (a + b) + 0.5 * (b - a) * ndr
            if reg == "L":
                vals[rs, :, j] = ps.inverse(xv, False) / xv
            else:
                vals[rs, :, j] = 2.0 * np.log(ps.inverse(np.exp(-xv), True))
    c = cheb_coeffs_from_values(vals, axis=1)
    return cheb_coeffs_from_values(c, axis=2)


FORMS = (("fp64", False), ("fp64", True), ("mixed", False), ("mixed", True))


def form_name(prec, trunc):
    return prec + ("_trunc" if trunc else "")


def _check_segment(args):
    """Max relative error of the inverse tables against fresh exact inversions in one segment,
    for every evaluation form (the full-table FP64 value is the tables' own error)."""
    kind, cs, tab, seed = args
    bt = BesselTables()
    rng = np.random.default_rng(seed)
    worst = {form_name(*f): 0.0 for f in FORMS}
    if kind == "photon":
        ca, cb = _inv_chi_segment_bounds(cs)
    else:
        ca, cb = _pair_inv_chi_segment_bounds(cs)
    for chi in rng.uniform(ca, cb, 3):
        chi = max(chi, 1e-12)
        omr = np.exp(rng.uniform(np.log(2.0 ** -52), np.log(0.5), 40))
        r_hi = 1.0 - omr
        omr = 1.0 - r_hi
        r_lo = rng.uniform(1e-6, 0.5, 40)
        if kind == "photon":
            ps = PhotonSpectrum(bt, chi)
            ex = np.concatenate([ps.inverse(r_lo, False), ps.inverse(omr, True)]) ** 3
            forms = photon_sample_forms(tab, np.full(80, chi), np.concatenate([r_lo, r_hi]))
        else:
            ps = PairSpectrum(bt, chi)
            r = np.concatenate([0.5 + 0.5 * r_lo, 0.5 + 0.5 * r_hi])
            q = np.abs(2.0 * r - 1.0)          # the level the sampler sees (exact in double)
            ex = np.concatenate([ps.inverse(q[:40], False), ps.inverse(1.0 - q[40:], True)]) ** 2
            forms = pair_sample_forms(tab, np.full(80, chi), r)
        for f, ap in forms.items():
            name = form_name(*f)
            worst[name] = max(worst[name], float(np.max(np.abs(ap / ex - 1))))
    return kind, cs, worst


def build_all(jobs=8, verbose=True):
    from concurrent.futures import ProcessPoolExecutor

    t0 = time.time()
    bt = BesselTables()
    rad, pair = build_rate_tables()
    with ProcessPoolExecutor(max_workers=jobs) as ex:
        ph = list(ex.map(_photon_segment, range(N_INV_CHI)))
        pp = list(ex.map(_pair_segment, range(N_PAIR_INV_CHI)))
        phinv, ppinv = np.stack(ph), np.stack(pp)
        if verbose:
            print(f"tables fitted in {time.time() - t0:.1f} s", flush=True)
        checks = [("photon", cs, phinv, 100 + cs) for cs in range(N_INV_CHI)]
        checks += [("pair", cs, ppinv, 1000 + cs) for cs in range(N_PAIR_INV_CHI)]
        errs = list(ex.map(_check_segment, checks))
    chi_r = np.concatenate([np.geomspace(1e-9, 2.0 ** CHI_OCT_HI * 0.999, 500),
                            np.linspace(0, 2.0 ** CHI_OCT_LO, 60)[1:]])
    chi_p = np.geomspace(0.01, 2.0 ** CHI_OCT_HI * 0.999, 500)
    ex_r = wrad_exact(chi_r)
    ex_p = np.exp(-8.0 / (3.0 * chi_p)) * pair_scaled_exact(chi_p)   # W~_pair itself
    forms = {}
    for prec, trunc in FORMS:
        dt = np.float32 if prec == "mixed" else np.float64
        rt, pt = (truncate_rates(rad), truncate_rates(pair)) if trunc else (rad, pair)
        e_r = float(np.max(np.abs(eval_rad(rt, chi_r, dt).astype(np.float64) / ex_r - 1)))
        # W~_pair as the kernels form it, e^{-8/(3 chi)} included, in the form's precision: the
        # rounding of the exponent's argument costs |8/(3 chi)| units in the last place; where
        # the single-precision value underflows (chi below about 0.03, W~_pair < 1e-38) the
        # kernels' result is compared with an absolute tolerance instead
        cp = chi_p.astype(dt)
        wp = (eval_pair_scaled(pt, chi_p, dt) * np.exp(dt(-8.0 / 3.0) / cp)).astype(np.float64)
        keep = ex_p > np.finfo(dt).tiny * 16
        e_p = float(np.max(np.abs(wp[keep] / ex_p[keep] - 1)))
        name = form_name(prec, trunc)
        e_ph = max(w[name] for k, cs, w in errs if k == "photon")
        e_pp = max(w[name] for k, cs, w in errs if k == "pair")
        forms[name] = {"rate": max(e_r, e_p), "photon_rate": e_r, "pair_rate": e_p,
                       "sample": max(e_ph, e_pp), "photon_sample": e_ph, "pair_sample": e_pp,
                       "rate_terms": RATE_DEG_TRUNC if trunc else RATE_DEG,
                       "patch_terms": INV_TRUNC if trunc else INV_NR}
    report = {
        "rate_rel_err": forms["fp64"]["photon_rate"], "pair_rate_rel_err": forms["fp64"]["pair_rate"],
        "photon_inverse_rel_err_by_segment": {cs: w["fp64"] for k, cs, w in errs if k == "photon"},
        "pair_inverse_rel_err_by_segment": {cs: w["fp64"] for k, cs, w in errs if k == "pair"},
        # measured relative errors of each evaluation form: rates against the quadrature of
        # Eqs. (wtilde), (wtilde_pair); samples (wbar^3 and y, which bound the errors of the
        # energy fractions and their complements) against exact inversions; FP32 forms
        # evaluated in single precision as the kernels do (without their fused multiply-adds)
        "forms": forms,
        "build_seconds": time.time() - t0,
    }
    return dict(rad=rad, pair=pair, ka=bt.ka, kb=bt.kb, phinv=phinv, ppinv=ppinv), report


ARRAY_ORDER = ("rad", "pair", "ka", "kb", "phinv", "ppinv")


def write_blob(path, tables):
    g = globals()
    with open(path + ".tmp", "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<IIQ", 3, len(ARRAY_ORDER), source_hash()))
        f.write(struct.pack("<%di" % len(GEOMETRY), *[int(g[k]) for k in GEOMETRY]))
        for name in ARRAY_ORDER:
            a = np.ascontiguousarray(tables[name], dtype="<f8")
            f.write(struct.pack("<Q", a.size))
            f.write(a.tobytes())
    os.replace(path + ".tmp", path)


def read_blob_hash(path):
    try:
        with open(path, "rb") as f:
            if f.read(8) != MAGIC:
                return None
            _, _, h = struct.unpack("<IIQ", f.read(16))
            return h
    except OSError:
        return None


def default_path():
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "sfq_tables.bin")


def main(argv=None):
    import json

    argv = sys.argv[1:] if argv is None else argv
    paths = [a for a in argv if not a.startswith("--")]
    out = paths[0] if paths else default_path()
    force = "--force" in argv
    if not force and read_blob_hash(out) == source_hash():
        print(f"tables up to date: {out}")
        return 0
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tables, report = build_all()
    write_blob(out, tables)
    with open(os.path.splitext(out)[0] + "_report.json", "w") as f:
        json.dump(report, f, indent=1)
    worst_ph = max(report["photon_inverse_rel_err_by_segment"].values())
    worst_pp = max(report["pair_inverse_rel_err_by_segment"].values())
    print(f"wrote {out}: rate err {report['rate_rel_err']:.2e}, pair-rate err "
          f"{report['pair_rate_rel_err']:.2e}, photon inverse err {worst_ph:.2e}, "
          f"pair inverse err {worst_pp:.2e}, {report['build_seconds']:.1f} s")
    return 0


if __name__ == "__main__":
    sys.exit(main())
