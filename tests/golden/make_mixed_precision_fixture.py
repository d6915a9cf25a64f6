"""Writes tests/golden/mixed_precision_oracle.npz: the oracle's rates and energy samples at the
points tests/test_gpu_precision_report.py checks the MIXED form on (by decade of chi over
[1e-4, 1e3)).  It calls only oracle/: the rates of Eqs. (pe_rate_3) and (pp_tot_real) by
quadrature, the photon and pair samples by exact inversion of Eqs. (again) and (again_pp).

    python tests/golden/make_mixed_precision_fixture.py

The oracle's inversions take about a fifth of a CPU-second each, which is why they are stored
rather than recomputed in the GPU test.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402

DECADES = list(range(-4, 3))
N_RATE = 2000      # per decade, for each process
N_SAMPLE = 1000    # photon and pair samples per decade
N_TAIL = 300       # photon samples per decade with r in [1 - 1e-3, 1)
LR_OVER_LC = 1.0   # the rates are stored as W gamma / (lambda_r / lambda_C)
GAMMA = 1e4        # the emitting particle's energy of the samples
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mixed_precision_oracle.npz")


def points(seed=21):
    rng = np.random.default_rng(seed)
    c = {k: [] for k in ("chi_r", "gam_r", "chi_s", "r_s", "chi_p", "chi_t", "r_t")}
    for d in DECADES:
        c["chi_r"].append(10.0 ** rng.uniform(d, d + 1, N_RATE))
        c["gam_r"].append(10.0 ** rng.uniform(1, 6, N_RATE))
        c["chi_s"].append(10.0 ** rng.uniform(d, d + 1, N_SAMPLE))
        c["r_s"].append(rng.uniform(0, 1, N_SAMPLE))
        # pair creation is neglected below chi = 0.01 (Sec. 4.2)
        c["chi_p"].append(10.0 ** rng.uniform(max(d, -2), max(d + 1, -1), N_SAMPLE))
        c["chi_t"].append(10.0 ** rng.uniform(d, d + 1, N_TAIL))
        c["r_t"].append(1.0 - 10.0 ** rng.uniform(-16, -3, N_TAIL))
    return {k: np.concatenate(v) for k, v in c.items()}


def main():
    c = points()
    g_s = np.full(c["chi_s"].size, GAMMA)
    g_t = np.full(c["chi_t"].size, GAMMA)
    out = dict(c)
    out["decades"] = np.array(DECADES)
    out["sizes"] = np.array([N_RATE, N_SAMPLE, N_TAIL])
    out["gamma"] = np.array([GAMMA])
    out["w_compton"] = O.rates(O.ELECTRON, c["gam_r"], c["chi_r"], LR_OVER_LC)
    out["w_pair"] = O.rates(O.PHOTON, c["gam_r"], c["chi_r"], LR_OVER_LC)
    out["ph_gamma"], out["ph_emitter"], _ = O.sample_photon(g_s, c["chi_s"], c["r_s"])
    out["pp_electron"], out["pp_positron"], _ = O.sample_pair(g_s, c["chi_p"], c["r_s"])
    out["tail_gamma"], out["tail_emitter"], _ = O.sample_photon(g_t, c["chi_t"], c["r_t"])
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
