"""Python access to the CPU oracle (``oracle/sfq_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use this module; the product library never imports it.  The oracle computes the
plain definitions of the strong-field QED step of Montefiori & Tamburini (arXiv:2301.07684):
Bessel functions from their integral representations, the rates of Sec. 4.1-4.2 by adaptive
quadrature, the energy samples of Sec. 4.3-4.4 by inverse transform sampling with Brent's root
finder, the decisions of Sec. 2, the beyond-LCFA steps of Sec. 5 and the Boris momentum push of
the PIC cycle (Fig. 7).  See the C source for the equation each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sfq_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

ELECTRON, POSITRON, PHOTON = 0, 1, 2
OPTICAL_DEPTH, LOCAL = 0, 1
P_INIT, P_EMIT, P_CHILD, P_CHILD2, P_LOCAL = 0, 1, 2, 3, 4


def build(force: bool = False) -> str:
    """Compile the oracle with gcc + OpenMP (plain C, -O2, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class StepCfg(C.Structure):
    _fields_ = [("dt", C.c_double), ("lc_over_lr", C.c_double), ("seed", C.c_uint64),
                ("step", C.c_uint32), ("decision", C.c_int32), ("bw_fast", C.c_int32),
                ("pad", C.c_int32)]


class Product(C.Structure):
    _fields_ = [("px", C.c_double), ("py", C.c_double), ("pz", C.c_double), ("tau", C.c_double),
                ("uid", C.c_uint64), ("parent", C.c_uint64), ("gamma", C.c_double),
                ("species", C.c_int32), ("valid", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("chi", C.c_double), ("gamma", C.c_double), ("rate", C.c_double),
                ("tau_out", C.c_double), ("px", C.c_double), ("py", C.c_double),
                ("pz", C.c_double), ("emitted", C.c_int32), ("alive_out", C.c_int32),
                ("clamped", C.c_int32), ("pad", C.c_int32), ("r_energy", C.c_double),
                ("xi_or_v", C.c_double), ("prod", Product * 2)]


_lib = None
_dp = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        d, i, l, u64 = C.c_double, C.c_int, C.c_long, C.c_uint64
        sig = {
            "orc_alpha": (d, []), "orc_lambda_compton": (d, []), "orc_speed_of_light": (d, []),
            "orc_gl_order": (i, []), "orc_gl_rule": (None, [_dp, _dp]),
            "orc_bessel_k": (d, [d, d]), "orc_bessel_ki": (d, [d, d]),
            "orc_bessel_k_scaled": (d, [d, d]), "orc_bessel_ki_scaled": (d, [d, d]),
            "orc_wtilde_rad": (d, [d]), "orc_wtilde_pair": (d, [d]),
            "orc_wtilde_pair_scaled": (d, [d]),
            "orc_rate_compton": (d, [d, d, d]), "orc_rate_breit_wheeler": (d, [d, d, d, i]),
            "orc_photon_spectrum_w": (d, [d, d]), "orc_photon_spectrum_w_k53": (d, [d, d]),
            "orc_photon_cdf": (d, [d, d]), "orc_photon_ccdf": (d, [d, d]),
            "orc_pair_spectrum_v_scaled": (d, [d, d]),
            "orc_pair_cdf_scaled": (d, [d, d]), "orc_pair_ccdf_scaled": (d, [d, d]),
            "orc_photon_wbar": (d, [d, d]), "orc_pair_vbar": (d, [d, d]),
            "orc_sample_photon": (None, [d, d, d, _dp, _dp, _dp]),
            "orc_sample_pair": (None, [d, d, d, _dp, _dp, _dp]),
            "orc_chi": (d, [i, _dp, _dp, _dp, d]), "orc_gamma": (d, [i, _dp]),
            "orc_philox4x32_10": (None, [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                         C.POINTER(C.c_uint32)]),
            "orc_draw": (None, [u64, u64, C.c_uint32, C.c_uint32, C.POINTER(u64),
                                C.POINTER(u64)]),
            "orc_uniform": (d, [u64]), "orc_optical_depth": (d, [u64]),
            "orc_blcfa_update": (i, [_dp, _dp, d, d, _dp, _dp, C.POINTER(i), _dp, _dp, _dp,
                                     C.POINTER(i)]),
            "orc_blcfa_threshold": (d, [_dp, d, d, d]),
            "orc_photon_pdf_energy": (d, [d, d, d]),
            "orc_blcfa_accept": (i, [d, d, d, d, d]),
            "orc_num_threads": (i, []),
            "orc_wtilde_rad_batch": (None, [l, _dp, _dp]),
            "orc_wtilde_pair_scaled_batch": (None, [l, _dp, _dp]),
            "orc_rates_batch": (None, [l, i, _dp, _dp, d, i, _dp]),
            "orc_chi_batch": (None, [l, i] + [_dp] * 9 + [d, _dp, _dp]),
            "orc_sample_photon_batch": (None, [l, _dp, _dp, _dp, _dp, _dp, _dp]),
            "orc_sample_pair_batch": (None, [l, _dp, _dp, _dp, _dp, _dp, _dp]),
            "orc_step_batch": (None, [C.POINTER(StepCfg), i, l] + [_dp] * 10 +
                               [C.POINTER(u64), C.POINTER(C.c_uint8), C.POINTER(Result)]),
            "orc_result_size": (l, []), "orc_product_size": (l, []),
            "orc_decide_batch": (None, [C.POINTER(StepCfg), l, _dp, _dp, C.POINTER(u64),
                                        C.POINTER(C.c_int32)]),
            "orc_step_blcfa_batch": (None, [C.POINTER(StepCfg), l] + [_dp] * 8 +
                                     [C.POINTER(C.c_uint8), C.POINTER(u64), C.POINTER(Result)]),
            "orc_boris_push": (None, [d, _dp, _dp, _dp, d, _dp]),
            "orc_boris_push_batch": (None, [d, l] + [_dp] * 9 + [d, _dp, _dp, _dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        assert L.orc_result_size() == C.sizeof(Result), "oracle Result layout mismatch"
        assert L.orc_product_size() == C.sizeof(Product), "oracle Product layout mismatch"
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---- constants -------------------------------------------------------------------------------
def alpha() -> float:
    return lib().orc_alpha()


def lambda_compton() -> float:
    return lib().orc_lambda_compton()


def speed_of_light() -> float:
    return lib().orc_speed_of_light()


def gl_rule():
    n = lib().orc_gl_order()
    x, w = np.zeros(n), np.zeros(n)
    lib().orc_gl_rule(_ptr(x), _ptr(w))
    return x, w


# ---- special functions (scalar) ---------------------------------------------------------------
def bessel_k(nu, x):
    return lib().orc_bessel_k(float(nu), float(x))


def bessel_ki(nu, x):
    return lib().orc_bessel_ki(float(nu), float(x))


def bessel_k_scaled(nu, x):
    return lib().orc_bessel_k_scaled(float(nu), float(x))


def bessel_ki_scaled(nu, x):
    return lib().orc_bessel_ki_scaled(float(nu), float(x))


# ---- rates --------------------------------------------------------------------------------------
def wtilde_rad(chi):
    chi = _f64(np.atleast_1d(chi))
    out = np.empty_like(chi)
    lib().orc_wtilde_rad_batch(chi.size, _ptr(chi), _ptr(out))
    return out


def wtilde_pair_scaled(chi):
    """exp(8/(3 chi)) * W~_pair(chi)."""
    chi = _f64(np.atleast_1d(chi))
    out = np.empty_like(chi)
    lib().orc_wtilde_pair_scaled_batch(chi.size, _ptr(chi), _ptr(out))
    return out


def wtilde_pair(chi):
    chi = _f64(np.atleast_1d(chi))
    return np.exp(-8.0 / (3.0 * chi)) * wtilde_pair_scaled(chi)


def rates(species, gamma, chi, lr_over_lc, bw_fast=False):
    gamma, chi = _f64(gamma), _f64(chi)
    out = np.empty_like(chi)
    lib().orc_rates_batch(chi.size, int(species == PHOTON), _ptr(gamma), _ptr(chi),
                          float(lr_over_lc), int(bw_fast), _ptr(out))
    return out


# ---- spectra ------------------------------------------------------------------------------------
def photon_spectrum_w(w, chi):
    return lib().orc_photon_spectrum_w(float(w), float(chi))


def photon_spectrum_w_k53(w, chi):
    return lib().orc_photon_spectrum_w_k53(float(w), float(chi))


def photon_cdf(w, chi):
    return lib().orc_photon_cdf(float(w), float(chi))


def photon_ccdf(w, chi):
    return lib().orc_photon_ccdf(float(w), float(chi))


def pair_spectrum_v_scaled(v, chi):
    return lib().orc_pair_spectrum_v_scaled(float(v), float(chi))


def pair_cdf_scaled(v, chi):
    return lib().orc_pair_cdf_scaled(float(v), float(chi))


def pair_ccdf_scaled(v, chi):
    return lib().orc_pair_ccdf_scaled(float(v), float(chi))


def photon_pdf_energy(g_ph, gamma, chi):
    return lib().orc_photon_pdf_energy(float(g_ph), float(gamma), float(chi))


# ---- sampling -----------------------------------------------------------------------------------
def sample_photon(gamma, chi, r):
    """Returns (gamma_photon, gamma_emitter_after, wbar)."""
    gamma, chi, r = _f64(gamma), _f64(chi), _f64(r)
    n = chi.size
    gph, gem, wb = np.empty(n), np.empty(n), np.empty(n)
    lib().orc_sample_photon_batch(n, _ptr(gamma), _ptr(chi), _ptr(r), _ptr(gph), _ptr(gem),
                                  _ptr(wb))
    return gph, gem, wb


def sample_pair(gamma, chi, r):
    """Returns (gamma_electron, gamma_positron, vbar)."""
    gamma, chi, r = _f64(gamma), _f64(chi), _f64(r)
    n = chi.size
    ge, gp, vb = np.empty(n), np.empty(n), np.empty(n)
    lib().orc_sample_pair_batch(n, _ptr(gamma), _ptr(chi), _ptr(r), _ptr(ge), _ptr(gp), _ptr(vb))
    return ge, gp, vb


# ---- chi ----------------------------------------------------------------------------------------
def chi(species, p, E, B, lc_over_lr):
    """p, E, B: arrays of shape (3, n).  Returns (gamma, chi)."""
    p, E, B = (_f64(a) for a in (p, E, B))
    n = p.shape[1]
    g, c = np.empty(n), np.empty(n)
    args = [_ptr(np.ascontiguousarray(a[k])) for a in (p, E, B) for k in range(3)]
    lib().orc_chi_batch(n, int(species == PHOTON), *args, float(lc_over_lr), _ptr(g), _ptr(c))
    return g, c


# ---- random numbers -----------------------------------------------------------------------------
def boris_push(species, p, E, B, dt):
    """Boris push of n particles ((3, n) arrays) over dt: charge -1 for electrons, +1 for
    positrons; photons are returned unchanged (they feel no force)."""
    p = _f64(p)
    if species == PHOTON:
        return p.copy()
    q = -1.0 if species == ELECTRON else 1.0
    E, B = _f64(E), _f64(B)
    n = p.shape[1]
    out = np.empty_like(p)
    cols = [np.ascontiguousarray(a[k]) for a in (p, E, B) for k in range(3)]
    outs = [np.empty(n) for _ in range(3)]
    lib().orc_boris_push_batch(q, n, *[_ptr(c) for c in cols], float(dt), *[_ptr(o) for o in outs])
    for k in range(3):
        out[k] = outs[k]
    return out


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(int(v) for v in o)


def draw(seed, uid, step, purpose):
    a, b = C.c_uint64(), C.c_uint64()
    lib().orc_draw(int(seed), int(uid), int(step), int(purpose), C.byref(a), C.byref(b))
    return a.value, b.value


def uniform(a):
    return lib().orc_uniform(int(a))


def optical_depth(a):
    return lib().orc_optical_depth(int(a))


def init_optical_depth(seed, uid):
    """tau_0 = -ln(1 - r) with r from draw purpose P_INIT at step 0."""
    return np.array([optical_depth(draw(seed, int(u), 0, P_INIT)[0]) for u in np.asarray(uid)])


# ---- the step -----------------------------------------------------------------------------------
def step(species, p, E, B, tau, uid, *, dt, lc_over_lr, seed, step, decision=OPTICAL_DEPTH,
         bw_fast=False, alive=None):
    """One Monte Carlo step for n particles of one species.

    p, E, B: (3, n) float64; tau: (n,); uid: (n,) uint64.  Returns a dict of numpy arrays:
    chi, gamma, rate, tau, p (3, n), emitted, alive, clamped, r_energy, xi_or_v and
    ``products``: a list of dicts (species, px, py, pz, tau, uid, parent, gamma)."""
    p, E, B = (_f64(a) for a in (p, E, B))
    tau = _f64(tau)
    uid = np.ascontiguousarray(np.asarray(uid, dtype=np.uint64))
    n = tau.size
    al = None if alive is None else np.ascontiguousarray(np.asarray(alive, dtype=np.uint8))
    cfg = StepCfg(dt=float(dt), lc_over_lr=float(lc_over_lr), seed=int(seed), step=int(step),
                  decision=int(decision), bw_fast=int(bw_fast), pad=0)
    out = (Result * max(n, 1))()
    cols = [np.ascontiguousarray(a[k]) for a in (p, E, B) for k in range(3)]
    lib().orc_step_batch(C.byref(cfg), int(species), n, *[_ptr(c) for c in cols], _ptr(tau),
                         uid.ctypes.data_as(C.POINTER(C.c_uint64)),
                         None if al is None else al.ctypes.data_as(C.POINTER(C.c_uint8)), out)
    res = np.ctypeslib.as_array(out)[:n] if n else None
    d = {}
    names = ["chi", "gamma", "rate", "tau_out", "px", "py", "pz", "emitted", "alive_out",
             "clamped", "r_energy", "xi_or_v"]
    for nm in names:
        d[nm] = np.array([getattr(r, nm) for r in out[:n]])
    d["tau"] = d.pop("tau_out")
    d["alive"] = d.pop("alive_out")
    d["p"] = np.stack([d.pop("px"), d.pop("py"), d.pop("pz")])
    prods = []
    for r in out[:n]:
        for q in r.prod:
            if q.valid:
                prods.append(dict(species=q.species, px=q.px, py=q.py, pz=q.pz, tau=q.tau,
                                  uid=q.uid, parent=q.parent, gamma=q.gamma))
    d["products"] = prods
    del res
    return d


def decide(W, tau, uid, *, dt, seed, step, decision=OPTICAL_DEPTH):
    """Decision of one step for given rates W (no chi, no sampling).  Returns (tau, emitted)."""
    W, tau = _f64(W), _f64(tau).copy()
    uid = np.ascontiguousarray(np.asarray(uid, dtype=np.uint64))
    em = np.zeros(tau.size, dtype=np.int32)
    cfg = StepCfg(dt=float(dt), lc_over_lr=1.0, seed=int(seed), step=int(step),
                  decision=int(decision), bw_fast=0, pad=0)
    lib().orc_decide_batch(C.byref(cfg), tau.size, _ptr(W), _ptr(tau),
                           uid.ctypes.data_as(C.POINTER(C.c_uint64)),
                           em.ctypes.data_as(C.POINTER(C.c_int32)))
    return tau, em.astype(bool)


# ---- beyond LCFA --------------------------------------------------------------------------------
def blcfa_update(p_prev, p_push, dt, tau_c, Fperp, dF, just_created):
    """Returns (flag, gamma, chi, delta, first_step, Fperp_new, dF_new, just_created_new)."""
    pp = (C.c_double * 3)(*p_prev)
    pu = (C.c_double * 3)(*p_push)
    F = (C.c_double * 3)(*Fperp)
    D = (C.c_double * 3)(*dF)
    jc = C.c_int(int(just_created))
    g, c, de = C.c_double(), C.c_double(), C.c_double()
    fs = C.c_int()
    flag = lib().orc_blcfa_update(pp, pu, float(dt), float(tau_c), F, D, C.byref(jc),
                                  C.byref(g), C.byref(c), C.byref(de), C.byref(fs))
    return (bool(flag), g.value, c.value, de.value, bool(fs.value), list(F), list(D),
            bool(jc.value))


def step_blcfa(p_prev, p_push, fperp, dfperp, just_created, uid, *, dt, lc_over_lr, seed, step):
    """One beyond-LCFA step (local decision) for n leptons.  p_prev, p_push: (3, n); fperp,
    dfperp: (3n,) component-major state (updated copies are returned); just_created: (n,) uint8.
    Returns a dict like step() plus the new state and a `rejected` flag array."""
    pp, pu = _f64(p_prev), _f64(p_push)
    n = pu.shape[1]
    F, D = _f64(fperp).copy(), _f64(dfperp).copy()
    jc = np.ascontiguousarray(np.asarray(just_created, dtype=np.uint8)).copy()
    uid = np.ascontiguousarray(np.asarray(uid, dtype=np.uint64))
    cfg = StepCfg(dt=float(dt), lc_over_lr=float(lc_over_lr), seed=int(seed), step=int(step),
                  decision=LOCAL, bw_fast=0, pad=0)
    out = (Result * max(n, 1))()
    cols = [np.ascontiguousarray(a[k]) for a in (pp, pu) for k in range(3)]
    lib().orc_step_blcfa_batch(C.byref(cfg), n, *[_ptr(c) for c in cols], _ptr(F), _ptr(D),
                               jc.ctypes.data_as(C.POINTER(C.c_uint8)),
                               uid.ctypes.data_as(C.POINTER(C.c_uint64)), out)
    d = {nm: np.array([getattr(r, nm) for r in out[:n]]) for nm in
         ("chi", "gamma", "rate", "emitted", "clamped", "r_energy", "xi_or_v")}
    d["rejected"] = d["clamped"] < 0
    d["clamped"] = np.maximum(d["clamped"], 0)
    d["p"] = np.stack([np.array([r.px for r in out[:n]]), np.array([r.py for r in out[:n]]),
                       np.array([r.pz for r in out[:n]])])
    d["products"] = [dict(species=q.species, px=q.px, py=q.py, pz=q.pz, tau=q.tau, uid=q.uid,
                          parent=q.parent, gamma=q.gamma)
                     for r in out[:n] for q in r.prod if q.valid]
    d["fperp"], d["dfperp"], d["just_created"] = F, D, jc
    return d


def blcfa_threshold(Fperp, delta, gamma, chi):
    F = (C.c_double * 3)(*Fperp)
    return lib().orc_blcfa_threshold(F, float(delta), float(gamma), float(chi))


def blcfa_accept(gbar, limit, gamma, chi, r2):
    return bool(lib().orc_blcfa_accept(float(gbar), float(limit), float(gamma), float(chi),
                                       float(r2)))


def num_threads() -> int:
    return lib().orc_num_threads()
