"""End-to-end statistical checks of the GPU step at scale, in the spirit of the paper's
constant-field validation (Sec. 4.1: photon number against N_e T R, and the emitted spectrum).

Particles sit in a constant magnetic field perpendicular to their momentum, and their momenta
are restored after every step (converted photons are revived with a fresh exponential depth),
so chi and gamma stay fixed.  With
optical-depth decisions and a fresh exponential depth after each event, the remaining depth at
every step boundary is exponential (memorylessness), so every particle-step is an independent
Bernoulli trial with probability 1 - exp(-W dt): the total number of events over K steps is
exactly Binomial(N K, 1 - exp(-W dt)), with W from the oracle's quadrature.  The energy
fractions of the products are histogrammed in bins of equal probability under the oracle's own
spectrum (bin edges from the oracle's inverse CDF) and compared by a chi-square test.  This
exercises the whole GPU pipeline (chi, rate tables, decisions, Philox uniforms, inverse-CDF
tables, recoil and products) against distributions the oracle fixes.
"""
import numpy as np
import pytest
import torch
from scipy import stats

from oracle import oracle as O
from paper_2301_07684_amd import inputs, sfq

pytestmark = pytest.mark.gpu

N = 1 << 20
K = 40
BINS = 40


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def constant_field_tile(dev, h, species, gamma, chi, seed):
    pm = gamma if species == sfq.PHOTON else np.sqrt((gamma - 1.0) * (gamma + 1.0))
    b = chi / (pm * h.lc_over_lr)
    f = lambda v: torch.full((N,), v, dtype=torch.float64, device=dev)
    uid = torch.from_numpy(inputs.ids(seed, np.arange(N))).to(dev)
    tile = sfq.TileArrays(species, f(pm), f(0.0), f(0.0), f(0.0), f(0.0), f(0.0), f(0.0), f(0.0),
                          f(b), tau=h.init_optical_depth(uid, seed=seed), uid=uid,
                          alive=torch.ones(N, dtype=torch.uint8, device=dev))
    return tile, pm


def run_steps(h, tile, pm, products, counters, seed):
    for s in range(K):
        h.step([tile], seed=seed, step=s, products=products, counters=counters)
        tile.px.fill_(pm)  # restore: no recoil, no conversion between steps
        tile.py.zero_()
        tile.pz.zero_()
        # a converted photon is dead and keeps its spent depth: revive it with a fresh,
        # independent exponential depth (leptons get theirs from the step itself)
        dead = tile.alive == 0
        fresh = h.init_optical_depth(tile.uid, seed=seed + 1000 + s)
        tile.tau.copy_(torch.where(dead, fresh, tile.tau))
        tile.alive.fill_(1)
    torch.cuda.synchronize()


def binomial_check(events, W, dt, label):
    p = -np.expm1(-W * dt)
    mean, sd = N * K * p, np.sqrt(N * K * p * (1 - p))
    print(f"\n{label}: {events} events, binomial mean {mean:.1f} sd {sd:.1f}, "
          f"z = {(events - mean) / sd:+.2f}")
    assert abs(events - mean) < 5 * sd, (events, mean, sd)
    return mean, sd


def chi_square_pvalue(x, edges, label):
    counts = np.histogram(x, bins=edges)[0]
    expected = len(x) / (len(edges) - 1)
    stat = np.sum((counts - expected) ** 2 / expected)
    pv = stats.chi2.sf(stat, len(edges) - 2)
    print(f"{label}: chi-square {stat:.1f} on {len(edges) - 2} degrees of freedom, p = {pv:.3f}")
    return pv


@pytest.mark.parametrize("precision", [sfq.FP64, sfq.MIXED])
def test_photon_count_and_spectrum_in_a_constant_field(dev, precision):
    gamma, chi, seed = 19569.5, 1.0, 2024  # 10 GeV electrons at chi = 1 (Sec. 4.1)
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=precision)
    tile, pm = constant_field_tile(dev, h, sfq.ELECTRON, gamma, chi, seed)
    W = float(O.rates(O.ELECTRON, np.array([gamma]), np.array([chi]), h.lr_over_lc)[0])
    prods = sfq.ProductBuffers.empty(int(N * K * W * h.dt * 1.2) + 1000, 1, dev)
    cnt = sfq.Counters(dev)
    run_steps(h, tile, pm, prods, cnt, seed)
    c = cnt.as_dict()
    assert c["overflow"] == 0 and c["processed"] == N * K
    binomial_check(c["emitted"], W, h.dt, f"photon emissions ({'MIXED' if precision else 'FP64'})")
    k = prods.host_counts()[0]
    ph = prods.photons
    xi = torch.sqrt(ph.px[:k] ** 2 + ph.py[:k] ** 2 + ph.pz[:k] ** 2).cpu().numpy() / gamma
    r = np.arange(1, BINS) / BINS
    g = np.full(BINS - 1, gamma)
    edges = np.concatenate([[0.0], O.sample_photon(g, np.full(BINS - 1, chi), r)[0] / gamma,
                            [1.0]])
    assert chi_square_pvalue(xi, edges, "photon energy fractions") > 1e-4


@pytest.mark.parametrize("precision", [sfq.FP64, sfq.MIXED])
def test_pair_count_and_split_in_a_constant_field(dev, precision):
    gamma, chi, seed = 2.0e4, 3.0, 2025
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=precision)
    tile, pm = constant_field_tile(dev, h, sfq.PHOTON, gamma, chi, seed)
    W = float(O.rates(O.PHOTON, np.array([gamma]), np.array([chi]), h.lr_over_lc)[0])
    cap = int(N * K * W * h.dt * 1.2) + 1000
    prods = sfq.ProductBuffers.empty(1, cap, dev)
    cnt = sfq.Counters(dev)
    run_steps(h, tile, pm, prods, cnt, seed)
    c = cnt.as_dict()
    assert c["overflow"] == 0 and c["processed"] == N * K
    binomial_check(c["converted"], W, h.dt, f"pair creations ({'MIXED' if precision else 'FP64'})")
    k = prods.host_counts()[1]
    e = prods.electrons
    ge = torch.sqrt(1.0 + e.px[:k] ** 2 + e.py[:k] ** 2 + e.pz[:k] ** 2).cpu().numpy()
    f = ge / gamma  # electron share of the photon energy
    r = np.arange(1, BINS) / BINS
    edges = np.concatenate([[0.0], O.sample_pair(np.full(BINS - 1, gamma),
                                                 np.full(BINS - 1, chi), r)[0] / gamma, [1.0]])
    assert chi_square_pvalue(f, edges, "electron shares") > 1e-4
