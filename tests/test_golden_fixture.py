"""The stored oracle values of tests/golden/mixed_precision_oracle.npz are the oracle's own:
a sample of its points recomputed now gives the same numbers bit for bit (the fixture is
written by tests/golden/make_mixed_precision_fixture.py, which calls only the oracle)."""
import os

import numpy as np

from oracle import oracle as O

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "mixed_precision_oracle.npz")


def test_fixture_is_the_oracles_output():
    f = np.load(FIXTURE)
    rng = np.random.default_rng(3)
    k = rng.choice(f["chi_r"].size, 24, replace=False)
    assert np.array_equal(O.rates(O.ELECTRON, f["gam_r"][k], f["chi_r"][k], 1.0),
                          f["w_compton"][k])
    assert np.array_equal(O.rates(O.PHOTON, f["gam_r"][k], f["chi_r"][k], 1.0), f["w_pair"][k])
    g = float(f["gamma"][0])
    j = rng.choice(f["chi_s"].size, 6, replace=False)
    a, b, _ = O.sample_photon(np.full(j.size, g), f["chi_s"][j], f["r_s"][j])
    assert np.array_equal(a, f["ph_gamma"][j]) and np.array_equal(b, f["ph_emitter"][j])
    a, b, _ = O.sample_pair(np.full(j.size, g), f["chi_p"][j], f["r_s"][j])
    assert np.array_equal(a, f["pp_electron"][j]) and np.array_equal(b, f["pp_positron"][j])
    t = rng.choice(f["chi_t"].size, 4, replace=False)
    a, b, _ = O.sample_photon(np.full(t.size, g), f["chi_t"][t], f["r_t"][t])
    assert np.array_equal(a, f["tail_gamma"][t]) and np.array_equal(b, f["tail_emitter"][t])
    # the shapes the GPU test reads: decades x per-decade counts
    n_rate, n_samp, n_tail = (int(v) for v in f["sizes"])
    nd = f["decades"].size
    assert f["chi_r"].size == nd * n_rate and f["chi_s"].size == nd * n_samp
    assert f["chi_t"].size == nd * n_tail
