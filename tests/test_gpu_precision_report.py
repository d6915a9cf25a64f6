"""Per-output error of the MIXED (FP32 evaluation, FP64 chi / optical depth / tails) form
against the FP64 oracle, by decade of chi, on the skewed-chi ensemble (chi log-uniform
[1e-4, 1e3]).  Prints the table (pytest -s) and asserts the 2e-5 bound for every output:
rates W, photon energy fraction xi and 1 - xi, pair split v-shares, and separately the samples
whose energy fraction exceeds 0.999 (evaluated in FP64 by construction)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2301_07684_amd import inputs, sfq

pytestmark = pytest.mark.gpu


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
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=sfq.MIXED)
    rng = np.random.default_rng(21)
    rows = []
    worst = 0.0
    for d in range(-4, 3):
        n_rate, n_samp = 48, 12
        chi = 10.0 ** rng.uniform(d, d + 1, n_rate)
        gam = 10.0 ** rng.uniform(2, 5, n_rate)
        e_rate = {}
        for sp, name in ((sfq.ELECTRON, "W_compton"), (sfq.PHOTON, "W_pair")):
            out = h.rates(sp, T(gam, dev), T(chi, dev)).cpu().numpy()
            ref = O.rates(sp, gam, chi, h.lr_over_lc)
            tiny = np.finfo(np.float32).tiny * h.lr_over_lc
            err = np.where(np.abs(out - ref) <= tiny, 0.0, rel(out, ref))
            e_rate[name] = float(np.max(err))
        cs = chi[:n_samp]
        r = np.concatenate([rng.uniform(0, 1, n_samp - 3), [1 - 1e-6, 1 - 2.0 ** -40, 1e-7]])
        g = np.full(n_samp, 1e4)
        a, b = h.sample_photon(T(g, dev), T(cs, dev), T(r, dev))
        gph, gem, _ = O.sample_photon(g, cs, r)
        e_xi = float(np.max(rel(a.cpu().numpy(), gph)))
        e_omxi = float(np.max(rel(b.cpu().numpy(), gem)))
        hi = gph / g > 0.999
        e_hi = float(np.max(rel(b.cpu().numpy()[hi], gem[hi]))) if hi.any() else float("nan")
        cp = np.maximum(cs, 0.011)
        ea, eb = h.sample_pair(T(g, dev), T(cp, dev), T(r, dev))
        ge, gp, _ = O.sample_pair(g, cp, r)
        e_pair = float(max(np.max(rel(ea.cpu().numpy(), ge)), np.max(rel(eb.cpu().numpy(), gp))))
        row = dict(decade=f"[1e{d}, 1e{d + 1})", **e_rate, xi=e_xi, one_minus_xi=e_omxi,
                   xi_gt_0999=e_hi, pair_shares=e_pair)
        rows.append(row)
        worst = max(worst, *[v for k, v in row.items() if k != "decade" and v == v])
    print("\nMIXED vs FP64 oracle, max relative error per chi decade")
    print(f"{'decade':>14} {'W_compton':>10} {'W_pair':>10} {'xi':>10} {'1-xi':>10} {'xi>0.999':>10} {'pair':>10}")
    for r_ in rows:
        print(f"{r_['decade']:>14} {r_['W_compton']:10.2e} {r_['W_pair']:10.2e} {r_['xi']:10.2e} "
              f"{r_['one_minus_xi']:10.2e} {r_['xi_gt_0999']:10.2e} {r_['pair_shares']:10.2e}")
    assert worst < 2e-5
