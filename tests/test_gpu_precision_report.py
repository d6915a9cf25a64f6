"""Per-output error of the MIXED form (FP32 evaluation; FP64 chi, optical depth and the
re-evaluated tails) against the FP64 oracle, by decade of chi over [1e-4, 1e3): thousands of
rates and samples per decade.

Outputs: the rates W of Eqs. (pe_rate_3) and (pp_tot_real), the photon energy fraction xi and
1 - xi (Sec. 4.3), the electron and positron shares of a pair (Sec. 4.4), and on their own the
photon samples with xi > 0.999 (r drawn near 1), which the kernels re-evaluate in FP64.  Every
output must stay within the MIXED form's reported bound (autotune.form_errors) plus the
oracle's own accuracy; the table is printed (pytest -s or -rP).

The oracle's values at these points are in tests/golden/mixed_precision_oracle.npz, written by
tests/golden/make_mixed_precision_fixture.py, which calls only the oracle (its inversions take
about a fifth of a CPU-second each).
"""
import os

import numpy as np
import pytest
import torch

from paper_2301_07684_amd import autotune, inputs, sfq

pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "mixed_precision_oracle.npz")
ORACLE_RATE = 1e-12    # the oracle's outer quadratures
ORACLE_SAMPLE = 1e-11  # its inversions of those quadratures


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.abs(a - b) / np.abs(b)
    r[a == b] = 0
    return r


def test_mixed_precision_error_by_chi_decade():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda", 0)
    f = np.load(FIXTURE)
    decades = [int(d) for d in f["decades"]]
    n_rate, n_samp, n_tail = (int(v) for v in f["sizes"])
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=sfq.MIXED)
    b = autotune.form_errors()[(sfq.MIXED, sfq.APPROX_FULL)]
    tiny = np.finfo(np.float32).tiny * h.lr_over_lc
    gam_r, chi_r = f["gam_r"], f["chi_r"]
    o_e = h.rates(sfq.ELECTRON, T(gam_r, dev), T(chi_r, dev)).cpu().numpy()
    o_p = h.rates(sfq.PHOTON, T(gam_r, dev), T(chi_r, dev)).cpu().numpy()
    w_e, w_p = f["w_compton"] * h.lr_over_lc, f["w_pair"] * h.lr_over_lc   # stored for 1
    g_s = np.full(f["chi_s"].size, float(f["gamma"][0]))
    g_t = np.full(f["chi_t"].size, float(f["gamma"][0]))
    a, bb = (x.cpu().numpy() for x in h.sample_photon(T(g_s, dev), T(f["chi_s"], dev),
                                                      T(f["r_s"], dev)))
    ea, eb = (x.cpu().numpy() for x in h.sample_pair(T(g_s, dev), T(f["chi_p"], dev),
                                                     T(f["r_s"], dev)))
    ta, tb = (x.cpu().numpy() for x in h.sample_photon(T(g_t, dev), T(f["chi_t"], dev),
                                                       T(f["r_t"], dev)))
    err_e = np.where(np.abs(o_e - w_e) <= tiny, 0.0, rel(o_e, w_e))
    err_p = np.where(np.abs(o_p - w_p) <= tiny, 0.0, rel(o_p, w_p))
    e_xi, e_om = rel(a, f["ph_gamma"]), rel(bb, f["ph_emitter"])
    e_pair = np.maximum(rel(ea, f["pp_electron"]), rel(eb, f["pp_positron"]))
    hi = f["tail_gamma"] / g_t > 0.999
    e_txi, e_tom = rel(ta, f["tail_gamma"]), rel(tb, f["tail_emitter"])
    rows = []
    for k, d in enumerate(decades):
        sr = slice(k * n_rate, (k + 1) * n_rate)
        ss = slice(k * n_samp, (k + 1) * n_samp)
        st = slice(k * n_tail, (k + 1) * n_tail)
        h_k = hi[st]
        rows.append((f"[1e{d}, 1e{d + 1})", err_e[sr].max(), err_p[sr].max(), e_xi[ss].max(),
                     e_om[ss].max(), e_pair[ss].max(), int(h_k.sum()),
                     e_txi[st][h_k].max() if h_k.any() else float("nan"),
                     e_tom[st][h_k].max() if h_k.any() else float("nan")))
    print(f"\nMIXED vs the FP64 oracle: largest relative error per chi decade ({n_rate} rates of "
          f"each process, {n_samp} photon and {n_samp} pair samples, {n_tail} photon samples "
          "with r near 1, of which n have xi > 0.999)")
    print("| chi | W_compton | W_pair | xi | 1 - xi | pair shares | n | xi (xi > 0.999) | "
          "1 - xi (xi > 0.999) |")
    print("|---|---|---|---|---|---|---|---|---|")
    for r_ in rows:
        print(f"| {r_[0]} | {r_[1]:.2e} | {r_[2]:.2e} | {r_[3]:.2e} | {r_[4]:.2e} | {r_[5]:.2e} "
              f"| {r_[6]} | {r_[7]:.2e} | {r_[8]:.2e} |")
    assert np.all(err_e <= b["emission_rate"] + ORACLE_RATE)
    assert np.all(err_p <= b["pair_rate"] + ORACLE_RATE)
    sb = b["sample"] + ORACLE_SAMPLE
    assert max(e_xi.max(), e_om.max(), e_pair.max()) <= sb
    assert hi.sum() > 200 and max(e_txi[hi].max(), e_tom[hi].max()) <= sb
    h.close()
