"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances (FP64 form): Philox words and all integer/index results bit-exact; chi <= 1e-13 and
rates <= 1e-12 relative; sampled energy fractions xi and 1 - xi (electron and positron shares
for pairs) <= 1e-9 relative; emission decisions identical outside a relative band of 1e-9 around
the threshold.  MIXED form: rates and samples <= 2e-5 relative, decisions identical outside a
2e-5 band.  Paper: Montefiori & Tamburini, arXiv:2301.07684.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2301_07684_amd import inputs, sfq

pytestmark = pytest.mark.gpu

TOL_CHI = 1e-13
TOL_RATE = 1e-12
TOL_SAMPLE = 1e-9
TOL_MIXED = 2e-5
BAND = 1e-9


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def handle(**kw):
    kw.setdefault("ref_length", inputs.LAMBDA_R)
    kw.setdefault("dt", inputs.DT)
    return sfq.Handle(**kw)


@pytest.fixture(scope="module")
def h64(dev):
    return handle()


@pytest.fixture(scope="module")
def h32(dev):
    return handle(precision=sfq.MIXED)


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.abs(a - b) / np.abs(b)
    r[(a == b)] = 0.0
    return r


def vrel(a, b):
    """|a - b| / |b| of momentum vectors (the columns of (3, n) arrays, or one 3-vector): every
    component counts, so a wrong sign, a swapped axis or an electron and positron in each other's
    buffers fail.  Two zero vectors (a lepton put at rest on both sides) compare equal."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(a - b, axis=0)
    m = np.linalg.norm(b, axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(d == 0, 0.0, d / m)


# ----------------------------------------------------------------------------------------------
# random numbers
# ----------------------------------------------------------------------------------------------
def test_philox_bit_exact(h64, dev):
    rng = np.random.default_rng(1)
    uid = rng.integers(0, 2 ** 63, 400, dtype=np.int64)
    for seed in (0, 123456789123, 2 ** 64 - 1):
        for step in (0, 1, 2 ** 31 + 5):
            for purpose in range(5):
                a, b = h64.philox(T(uid, dev), seed, step, purpose)
                a, b = a.cpu().numpy().view(np.uint64), b.cpu().numpy().view(np.uint64)
                for k in range(0, uid.size, 37):
                    ra, rb = O.draw(seed, int(uid.view(np.uint64)[k]), step, purpose)
                    assert int(a[k]) == ra and int(b[k]) == rb


def test_init_optical_depth(h64, dev):
    uid = inputs.ids(5, np.arange(5000))
    tau = h64.init_optical_depth(T(uid, dev), seed=42).cpu().numpy()
    ref = O.init_optical_depth(42, uid.view(np.uint64)[:5000])
    assert np.max(rel(tau, ref)) < 1e-15


# ----------------------------------------------------------------------------------------------
# chi
# ----------------------------------------------------------------------------------------------
def test_chi_plain_compton_full(h64, dev):
    w = inputs.plain_compton(65536)
    g, c = h64.chi(sfq.ELECTRON, *[[T(w[k][i], dev) for i in range(3)] for k in "pEB"])
    og, oc = O.chi(O.ELECTRON, w["p"], w["E"], w["B"], h64.lc_over_lr)
    assert np.max(rel(c.cpu().numpy(), oc)) < TOL_CHI
    assert np.max(rel(g.cpu().numpy(), og)) < 1e-15


@pytest.mark.parametrize("species", [sfq.ELECTRON, sfq.PHOTON])
def test_chi_plane_wave(h64, dev, species):
    w = inputs.plane_wave(4096, species=species)
    g, c = h64.chi(species, *[[T(w[k][i], dev) for i in range(3)] for k in "pEB"])
    og, oc = O.chi(species, w["p"], w["E"], w["B"], h64.lc_over_lr)
    assert np.max(rel(c.cpu().numpy(), oc)) < TOL_CHI


def test_chi_co_propagating_stress(h64, dev):
    # particles along +x with the wave: chi = |a cos phi| lc / (gamma + |p|) exactly; the naive
    # formula loses ~log10(gamma^2) digits here
    w = inputs.plane_wave(4096, species=sfq.ELECTRON)
    p = w["p"].copy()
    p[0] = -p[0]
    g, c = h64.chi(sfq.ELECTRON, [T(p[i], dev) for i in range(3)],
                   *[[T(w[k][i], dev) for i in range(3)] for k in "EB"])
    pm = np.abs(p[0])
    gam = np.sqrt(1 + pm * pm)
    exact = np.abs(w["E"][1]) * h64.lc_over_lr / (gam + pm)
    assert np.max(rel(c.cpu().numpy(), exact)) < 1e-13


# ----------------------------------------------------------------------------------------------
# rates
# ----------------------------------------------------------------------------------------------
def _rate_grid(species):
    lo = -5 if species != sfq.PHOTON else -2
    chi = np.concatenate([10.0 ** np.linspace(lo, math.log10(3000), 70), [0.0099, 0.01, 0.2999, 0.3]])
    gamma = 10.0 ** np.linspace(1, 6, chi.size)
    return gamma, chi


@pytest.mark.parametrize("species", [sfq.ELECTRON, sfq.POSITRON, sfq.PHOTON])
def test_rates_fp64(h64, dev, species):
    gamma, chi = _rate_grid(species)
    out = h64.rates(species, T(gamma, dev), T(chi, dev)).cpu().numpy()
    ref = O.rates(species, gamma, chi, h64.lr_over_lc)
    assert np.array_equal(out == 0, ref == 0)
    assert np.max(rel(out[ref > 0], ref[ref > 0])) < TOL_RATE


def test_rates_bw_fast(dev):
    h = handle(bw_fast=True)
    gamma, chi = _rate_grid(sfq.PHOTON)
    out = h.rates(sfq.PHOTON, T(gamma, dev), T(chi, dev)).cpu().numpy()
    ref = O.rates(O.PHOTON, gamma, chi, h.lr_over_lc, bw_fast=True)
    assert np.array_equal(out == 0, ref == 0) and np.all(out[chi < 0.3] == 0)
    assert np.max(rel(out[ref > 0], ref[ref > 0])) < TOL_RATE


@pytest.mark.parametrize("species", [sfq.ELECTRON, sfq.PHOTON])
def test_rates_mixed(h32, dev, species):
    gamma, chi = _rate_grid(species)
    out = h32.rates(species, T(gamma, dev), T(chi, dev)).cpu().numpy()
    ref = O.rates(species, gamma, chi, h32.lr_over_lc)
    # where the FP32 exponential of the pair rate underflows, an absolute tolerance applies
    tiny = np.finfo(np.float32).tiny * h32.lr_over_lc
    ok = (np.abs(out - ref) <= TOL_MIXED * np.abs(ref)) | (np.abs(out - ref) <= tiny)
    assert np.all(ok), (chi[~ok], out[~ok], ref[~ok])


# ----------------------------------------------------------------------------------------------
# energy sampling
# ----------------------------------------------------------------------------------------------
PH_CHI = [1e-5, 1e-3, 0.02, 0.3, 1.0, 7.0, 60.0, 500.0, 1900.0]
PH_R = [1e-9, 1e-4, 0.01, 0.2, 0.4999, 0.5001, 0.8, 0.99, 0.9999, 1 - 2.0 ** -40, 1 - 2.0 ** -52]
PP_CHI = [0.01, 0.05, 0.3, 1.0, 10.0, 100.0, 1000.0]
PP_R = [1e-12, 1e-5, 0.1, 0.3, 0.4999, 0.5001, 0.7, 0.9, 0.99999, 1 - 2.0 ** -40]


@pytest.fixture(scope="module")
def photon_grid():
    chi, r = np.meshgrid(PH_CHI, PH_R, indexing="ij")
    chi, r = chi.ravel(), r.ravel()
    gamma = np.full(chi.size, 1e4)
    gph, gem, _ = O.sample_photon(gamma, chi, r)
    return gamma, chi, r, gph, gem


@pytest.fixture(scope="module")
def pair_grid():
    chi, r = np.meshgrid(PP_CHI, PP_R, indexing="ij")
    chi, r = chi.ravel(), r.ravel()
    gamma = np.full(chi.size, 1e4)
    ge, gp, _ = O.sample_pair(gamma, chi, r)
    return gamma, chi, r, ge, gp


@pytest.mark.parametrize("mixed", [False, True])
def test_sample_photon(h64, h32, dev, photon_grid, mixed):
    gamma, chi, r, gph, gem = photon_grid
    h = h32 if mixed else h64
    a, b = h.sample_photon(T(gamma, dev), T(chi, dev), T(r, dev))
    tol = TOL_MIXED if mixed else TOL_SAMPLE
    assert np.max(rel(a.cpu().numpy(), gph)) < tol  # xi
    assert np.max(rel(b.cpu().numpy(), gem)) < tol  # 1 - xi


@pytest.mark.parametrize("mixed", [False, True])
def test_sample_pair(h64, h32, dev, pair_grid, mixed):
    gamma, chi, r, ge, gp = pair_grid
    h = h32 if mixed else h64
    a, b = h.sample_pair(T(gamma, dev), T(chi, dev), T(r, dev))
    tol = TOL_MIXED if mixed else TOL_SAMPLE
    assert np.max(rel(a.cpu().numpy(), ge)) < tol
    assert np.max(rel(b.cpu().numpy(), gp)) < tol


# ----------------------------------------------------------------------------------------------
# the full step
# ----------------------------------------------------------------------------------------------
def make_tile(w, dev, tau, *, alive=True, diag=True):
    n = w["p"].shape[1]
    p = [T(w["p"][i], dev) for i in range(3)]
    E = [T(w["E"][i], dev) for i in range(3)]
    B = [T(w["B"][i], dev) for i in range(3)]
    ta = sfq.TileArrays(w["species"], *p, *E, *B, tau=T(tau, dev), uid=T(w["uid"], dev),
                        alive=torch.ones(n, dtype=torch.uint8, device=dev) if alive else None,
                        chi_out=torch.zeros(n, dtype=torch.float64, device=dev) if diag else None,
                        rate_out=torch.zeros(n, dtype=torch.float64, device=dev) if diag else None)
    return ta


def products_by_parent(pb, which):
    ps = getattr(pb, which)
    k = min(pb.host_counts()[{"photons": 0, "electrons": 1, "positrons": 2}[which]], ps.capacity)
    d = {}
    par = ps.parent[:k].cpu().numpy().view(np.uint64)
    arr = [a[:k].cpu().numpy() for a in (ps.px, ps.py, ps.pz, ps.tau)]
    uid = ps.uid[:k].cpu().numpy().view(np.uint64)
    for j in range(k):
        d[int(par[j])] = (np.array([arr[0][j], arr[1][j], arr[2][j]]), arr[3][j], int(uid[j]))
    return d


def check_step_against_oracle(w, tile, tau0, prods, h, *, seed, step, tol_rate, tol_sample, band,
                              n_sample=200, rng_seed=0):
    """Compare one GPU step (already run) with the oracle on every particle's rate/decision and
    on a subsample of particles for the full sampled outcome."""
    n = tau0.size
    photon = w["species"] == sfq.PHOTON
    og, oc = O.chi(w["species"], w["p"], w["E"], w["B"], h.lc_over_lr)
    W = O.rates(w["species"], og, oc, h.lr_over_lc)
    chi = tile.chi_out.cpu().numpy()
    rate = tile.rate_out.cpu().numpy()
    assert np.max(rel(chi, oc)) < (TOL_CHI if tol_rate == TOL_RATE else tol_rate)
    if tol_rate == TOL_RATE:
        pos = W > 0
        assert np.array_equal(rate == 0, W == 0)
        assert np.max(rel(rate[pos], W[pos])) < tol_rate
    else:
        # FP32: where e^{-8/(3chi)} of the pair rate underflows, an absolute tolerance applies
        tiny = np.finfo(np.float32).tiny * h.lr_over_lc
        ok = (np.abs(rate - W) <= tol_rate * np.abs(W)) | (np.abs(rate - W) <= tiny)
        assert np.all(ok)
    # decisions: the oracle's emitter set, outside the band
    thr = W * h.dt
    emit_or = tau0 - thr < 0
    in_band = np.abs(tau0 - thr) <= band * np.maximum(tau0, thr)
    key = "electrons" if photon else "photons"
    pmap = products_by_parent(prods, key)
    uids = w["uid"].view(np.uint64)
    emit_gpu = np.array([int(u) in pmap for u in uids])
    mism = (emit_gpu != emit_or) & ~in_band
    assert not mism.any(), f"{mism.sum()} decision mismatches outside the band"
    # full outcome on a subsample (emitters and non-emitters)
    rng = np.random.default_rng(rng_seed)
    em_idx = np.flatnonzero(emit_or & ~in_band)
    ne_idx = np.flatnonzero(~emit_or & ~in_band)
    pick = np.concatenate([rng.choice(em_idx, min(n_sample, em_idx.size), replace=False),
                           rng.choice(ne_idx, min(n_sample // 4, ne_idx.size), replace=False)])
    sub = {k: w[k][:, pick] for k in ("p", "E", "B")}
    ref = O.step(w["species"], sub["p"], sub["E"], sub["B"], tau0[pick], uids[pick],
                 dt=h.dt, lc_over_lr=h.lc_over_lr, seed=seed, step=step)
    p_gpu = np.stack([tile.px.cpu().numpy(), tile.py.cpu().numpy(), tile.pz.cpu().numpy()])[:, pick]
    tau_gpu = tile.tau.cpu().numpy()[pick]
    if not photon:
        em = ref["emitted"].astype(bool)
        # the recoiled momentum component by component; non-emitters keep theirs bit for bit
        assert np.max(vrel(p_gpu[:, em], ref["p"][:, em])) < tol_sample
        assert np.array_equal(p_gpu[:, ~em], sub["p"][:, ~em])
        # emitters: a fresh depth -ln(1 - r) from the same Philox word
        assert np.max(rel(tau_gpu[em], ref["tau"][em])) < 1e-15
        # others: tau0 - W dt, whose error is the rate error times W dt
        err = np.abs(tau_gpu[~em] - ref["tau"][~em])
        assert np.all(err <= tol_rate * W[pick][~em] * h.dt + 4e-16 * np.abs(tau0[pick][~em]))
    else:
        alive = tile.alive.cpu().numpy()[pick]
        assert np.array_equal(alive, ref["alive"])
        # every photon, converted or not, holds tau0 - W dt
        err = np.abs(tau_gpu - ref["tau"])
        assert np.all(err <= tol_rate * W[pick] * h.dt + 4e-16 * np.abs(tau0[pick]))
    prods_ref = {}
    for q in ref["products"]:
        prods_ref.setdefault(q["species"], {})[q["parent"]] = q
    for sp, name in ((O.PHOTON, "photons"), (O.ELECTRON, "electrons"), (O.POSITRON, "positrons")):
        got = products_by_parent(prods, name)
        for parent, q in prods_ref.get(sp, {}).items():
            assert parent in got, (name, parent)
            pv, tau_q, uid_q = got[parent]
            assert uid_q == q["uid"]
            assert abs(tau_q / q["tau"] - 1) < 1e-15
            assert vrel(pv, [q["px"], q["py"], q["pz"]]) < tol_sample, (name, parent)
    return emit_or, in_band


def test_step_plain_compton_full(h64, dev):
    n = 65536
    w = inputs.plain_compton(n)
    uid = T(w["uid"], dev)
    tau0 = h64.init_optical_depth(uid, seed=0).cpu().numpy()
    tile = make_tile(w, dev, tau0)
    prods = sfq.ProductBuffers.empty(n, 1, dev)
    cnt = sfq.Counters(dev)
    h64.step([tile], seed=0, step=1, products=prods, counters=cnt)
    torch.cuda.synchronize()
    c = cnt.as_dict()
    assert c["processed"] == n and c["overflow"] == 0
    emit_or, band = check_step_against_oracle(w, tile, tau0, prods, h64, seed=0, step=1,
                                              tol_rate=TOL_RATE, tol_sample=TOL_SAMPLE, band=BAND)
    assert abs(c["emitted"] - emit_or.sum()) <= band.sum()
    assert prods.host_counts()[0] == c["emitted"]
    # the expected emitter fraction of this workload is about 11.6 %
    assert 0.09 < c["emitted"] / n < 0.14


def test_step_plane_wave_two_species(h64, dev):
    n = 8192
    we = inputs.plane_wave(1 << 24, idx=np.arange(n) * 2048, species=sfq.ELECTRON)
    wg = inputs.plane_wave(1 << 24, idx=np.arange(n) * 2048, species=sfq.PHOTON)
    tiles, taus = [], []
    for w in (we, wg):
        tau0 = h64.init_optical_depth(T(w["uid"], dev), seed=7).cpu().numpy()
        # shrink optical depths so that a large share of particles acts in this one step
        tau0 = tau0 * 1e-3
        taus.append(tau0)
        tiles.append(make_tile(w, dev, tau0))
    prods = sfq.ProductBuffers.empty(n, n, dev)
    cnt = sfq.Counters(dev)
    h64.step(tiles, seed=7, step=3, products=prods, counters=cnt)
    torch.cuda.synchronize()
    for w, tile, tau0 in zip((we, wg), tiles, taus):
        check_step_against_oracle(w, tile, tau0, prods, h64, seed=7, step=3, tol_rate=TOL_RATE,
                                  tol_sample=TOL_SAMPLE, band=BAND, n_sample=150)
    c = cnt.as_dict()
    assert c["converted"] > 0 and c["emitted"] > 0
    assert prods.host_counts()[1] == prods.host_counts()[2] == c["converted"]


def test_step_mixed_precision_skewed_chi(h32, dev):
    n = 4096
    for species in (sfq.ELECTRON, sfq.PHOTON):
        w = inputs.plane_wave(1 << 24, idx=np.arange(n) * 4096, seed=inputs.SEED_SKEW,
                              species=species, chi_range=(1e-4, 1e3))
        tau0 = h32.init_optical_depth(T(w["uid"], dev), seed=3).cpu().numpy() * 1e-2
        tile = make_tile(w, dev, tau0)
        prods = sfq.ProductBuffers.empty(n, n, dev)
        cnt = sfq.Counters(dev)
        h32.step([tile], seed=3, step=9, products=prods, counters=cnt)
        torch.cuda.synchronize()
        check_step_against_oracle(w, tile, tau0, prods, h32, seed=3, step=9, tol_rate=TOL_MIXED,
                                  tol_sample=TOL_MIXED, band=TOL_MIXED, n_sample=100)


def test_step_tiling_invariance_and_ragged_tiles(h64, dev):
    n = 9000
    w = inputs.plain_compton(n, seed=77)
    tau0 = h64.init_optical_depth(T(w["uid"], dev), seed=1).cpu().numpy() * 0.1

    def run(cuts):
        tiles = []
        for a, b in zip(cuts[:-1], cuts[1:]):
            sub = dict(species=w["species"], p=w["p"][:, a:b], E=w["E"][:, a:b], B=w["B"][:, a:b],
                       uid=w["uid"][a:b])
            tiles.append(make_tile(sub, dev, tau0[a:b]))
        prods = sfq.ProductBuffers.empty(n, 1, dev)
        cnt = sfq.Counters(dev)
        h64.step(tiles, seed=5, step=2, products=prods, counters=cnt)
        torch.cuda.synchronize()
        p = np.concatenate([np.stack([t.px.cpu().numpy(), t.py.cpu().numpy(), t.pz.cpu().numpy()])
                            for t in tiles], axis=1)
        tau = np.concatenate([t.tau.cpu().numpy() for t in tiles])
        # the counters of the results (`deferred` depends on how the work was scheduled)
        return p, tau, products_by_parent(prods, "photons"), cnt.results()

    p1, t1, m1, c1 = run([0, n])
    p2, t2, m2, c2 = run([0, 1, 256, 513, 4610, 4610, n])  # includes an empty tile
    assert np.array_equal(p1, p2) and np.array_equal(t1, t2)
    assert m1.keys() == m2.keys()
    for k in m1:
        assert np.array_equal(m1[k][0], m2[k][0]) and m1[k][1] == m2[k][1] and m1[k][2] == m2[k][2]
    assert c1 == c2


@pytest.mark.parametrize("form", ["fp64", "mixed", "fp64_push"])
@pytest.mark.parametrize("shifted", ["all", "tau", "alive"])
def test_step_same_on_unaligned_views(dev, form, shifted):
    """Array tiles whose arrays all start on 16-byte boundaries (and whose alive flags start on
    an even byte) are streamed two adjacent particles per lane with 16-byte accesses; a tile
    with any array one element off such a boundary takes the one-particle-per-lane loop.  Both
    give the same bits for the same particles: momenta, depths, flags, diagnostics, products
    and counters."""
    h = handle(precision=sfq.MIXED if form == "mixed" else sfq.FP64)
    h.set_launch(2, 1024)   # 1024-particle chunks: two full 2 x 256 iterations each, ragged tail
    push = form.endswith("push")
    n = 5000

    def run(shift_names):
        tiles = []
        for species in (sfq.ELECTRON, sfq.PHOTON):
            w = inputs.plane_wave(1 << 24, idx=np.arange(n) * 1024, species=species, seed=21)
            tau0 = h.init_optical_depth(T(w["uid"], dev), seed=4).cpu().numpy() * 1e-3
            alive = (np.arange(n) % 7 != 5).astype(np.uint8)

            def put(name, a):
                t = torch.from_numpy(np.ascontiguousarray(a))
                s = 1 if (shift_names == "all" or shift_names == name) else 0
                buf = torch.zeros(n + 2, dtype=t.dtype, device=dev)
                buf[s:s + n] = t.to(dev)
                return buf[s:s + n]

            p = [put("p", w["p"][i]) for i in range(3)]
            E = [put("E", w["E"][i]) for i in range(3)]
            B = [put("B", w["B"][i]) for i in range(3)]
            tiles.append(sfq.TileArrays(
                species, *p, *E, *B, tau=put("tau", tau0), uid=put("uid", w["uid"]),
                alive=put("alive", alive),
                chi_out=torch.zeros(n, dtype=torch.float64, device=dev),
                rate_out=torch.zeros(n, dtype=torch.float64, device=dev)))
        prods = sfq.ProductBuffers.empty(2 * n, n, dev)
        cnt = sfq.Counters(dev)
        h.step(tiles, seed=6, step=2, products=prods, counters=cnt, push=push)
        torch.cuda.synchronize()
        out = [torch.stack([t.px, t.py, t.pz, t.tau, t.chi_out, t.rate_out]).cpu().numpy()
               for t in tiles]
        flags = [t.alive.cpu().numpy() for t in tiles]
        ptrs = [t.tau.data_ptr() % 16 for t in tiles]
        maps = {k: products_by_parent(prods, k) for k in ("photons", "electrons", "positrons")}
        return out, flags, maps, cnt.results(), ptrs

    o1, f1, m1, c1, a1 = run(None)
    o2, f2, m2, c2, a2 = run(shifted)
    assert a1 == [0, 0] and a2 == ([8, 8] if shifted in ("all", "tau") else [0, 0])
    assert c1["emitted"] > 0 and c1["converted"] > 0 and c1 == c2
    for x, y in zip(o1, o2):
        assert np.array_equal(x.view(np.uint64), y.view(np.uint64))
    for x, y in zip(f1, f2):
        assert np.array_equal(x, y)
    for k in m1:
        assert m1[k].keys() == m2[k].keys()
        for parent in m1[k]:
            assert np.array_equal(m1[k][parent][0], m2[k][parent][0])
            assert m1[k][parent][1:] == m2[k][parent][1:]


def test_step_edge_cases(h64, dev):
    n = 3000
    w = inputs.plain_compton(n, seed=91)
    tau0 = np.full(n, 1e-30)                  # every particle with a positive rate emits
    tile = make_tile(w, dev, tau0)
    tile.alive[::3] = 0                        # dead particles are skipped and untouched
    px0 = tile.px.clone()
    prods = sfq.ProductBuffers.empty(1, 1, dev)  # capacity 1: all but one photon overflow
    cnt = sfq.Counters(dev)
    h64.step([tile], seed=2, step=4, products=prods, counters=cnt)
    torch.cuda.synchronize()
    c = cnt.as_dict()
    n_alive = n - len(range(0, n, 3))
    assert c["processed"] == n_alive
    assert c["emitted"] == n_alive
    assert prods.host_counts()[0] == n_alive and c["overflow"] == n_alive - 1
    dead = np.arange(0, n, 3)
    assert torch.equal(tile.px[dead], px0[dead])
    assert np.all(tile.tau.cpu().numpy()[dead] == 1e-30)
    # photons below chi = 0.01 never convert; an empty step is a no-op
    wg = inputs.plain_compton(1000, seed=92, species=sfq.PHOTON, chi_range=(1e-4, 0.0099))
    tg = make_tile(wg, dev, np.full(1000, 1e-30))
    prods = sfq.ProductBuffers.empty(1, 1000, dev)
    cnt = sfq.Counters(dev)
    empty = make_tile(dict(species=sfq.ELECTRON, p=np.zeros((3, 0)), E=np.zeros((3, 0)),
                           B=np.zeros((3, 0)), uid=np.zeros(0, dtype=np.int64)), dev, np.zeros(0))
    h64.step([empty, tg], seed=2, step=4, products=prods, counters=cnt)
    torch.cuda.synchronize()
    assert cnt.as_dict()["converted"] == 0 and torch.all(tg.alive == 1)
    assert torch.all(tg.rate_out == 0)
    # a step whose tiles are all empty still zeroes the product counts when asked, for one set
    # of buffers and for per-owner sets
    prods.counts.copy_(torch.tensor([5, 6, 7], device=dev))
    h64.step([empty], seed=2, step=5, products=prods, counters=cnt)
    torch.cuda.synchronize()
    assert prods.host_counts() == [5, 6, 7]
    h64.step([empty, empty], seed=2, step=5, products=prods, counters=cnt,
             zero_product_counts=True)
    torch.cuda.synchronize()
    assert prods.host_counts() == [0, 0, 0]
    sets = [sfq.ProductBuffers.empty(4, 4, dev) for _ in range(2)]
    for k, pb in enumerate(sets):
        pb.counts.copy_(torch.tensor([1 + k, 2, 3], device=dev))
    h64.step([empty], seed=2, step=5, counters=cnt, product_sets=sets, zero_product_counts=True)
    torch.cuda.synchronize()
    assert all(pb.host_counts() == [0, 0, 0] for pb in sets)
    assert cnt.as_dict()["processed"] == 1000 + 0  # the empty steps processed nothing


def test_step_refused_inside_a_stream_capture(h64, dev):
    # a captured sfq_step would keep pointers to the handle's recycled scratch: it is refused
    # with SFQ_E_STATE and enqueues nothing (graphs of steps come from plans)
    n = 256
    w = inputs.plain_compton(n, seed=93)
    tile = make_tile(w, dev, np.full(n, 0.5))
    prods = sfq.ProductBuffers.empty(n, 1, dev)
    cnt = sfq.Counters(dev)
    x = torch.zeros(4, device=dev)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        x.add_(1.0)
        with pytest.raises(sfq.SFQError, match="capturing"):
            h64.step([tile], seed=1, step=1, products=prods, counters=cnt)
    torch.cuda.synchronize()
    assert cnt.as_dict()["processed"] == 0
    # the handle still steps outside the capture
    h64.step([tile], seed=1, step=1, products=prods, counters=cnt)
    torch.cuda.synchronize()
    assert cnt.as_dict()["processed"] == n


@pytest.mark.parametrize("precision", [sfq.FP64, sfq.MIXED])
def test_step_full_size_plane_wave(dev, precision):
    """The benchmark workload at full size (2^24 electrons + 2^24 photons) in the benchmark's
    launch configuration (2 blocks per compute unit x 4096 particles per chunk): energy
    conservation over every emitter, and the full outcome (rate, decision, recoil, products)
    against the oracle on sampled particles, random ones and emitters."""
    mixed = precision == sfq.MIXED
    tol_rate, tol_sample, band = (TOL_MIXED, TOL_MIXED, TOL_MIXED) if mixed else \
        (TOL_RATE, TOL_SAMPLE, BAND)
    h = handle(precision=precision)
    h.set_launch(2, 4096)
    n = 1 << 24
    rng = np.random.default_rng(11)
    tiles, ws, taus = [], [], []
    for species in (sfq.ELECTRON, sfq.PHOTON):
        w = inputs.plane_wave(n, species=species)
        tau0 = h.init_optical_depth(T(w["uid"], dev), seed=0)
        tiles.append(make_tile(w, dev, tau0.cpu().numpy()))
        ws.append(w)
        taus.append(tau0.cpu().numpy())
    prods = sfq.ProductBuffers.empty(n // 8, n // 32, dev)
    cnt = sfq.Counters(dev)
    h.step(tiles, seed=0, step=1, products=prods, counters=cnt)
    torch.cuda.synchronize()
    c = cnt.as_dict()
    assert c["processed"] == 2 * n and c["overflow"] == 0
    # energy conservation for every Compton emitter: |p'| of the emitter and the photon energy
    k = prods.host_counts()[0]
    par = prods.photons.parent[:k].cpu().numpy().view(np.uint64)
    idx = (par - (np.uint64(inputs.SEED_WAVE) << np.uint64(40))).astype(np.int64)
    e = tiles[0]
    pnew = torch.stack([e.px, e.py, e.pz])[:, torch.from_numpy(idx).to(dev)].cpu().numpy()
    g_after = np.sqrt(1 + np.sum(pnew ** 2, axis=0))
    g_ph = np.linalg.norm(np.stack([prods.photons.px[:k].cpu().numpy(),
                                    prods.photons.py[:k].cpu().numpy(),
                                    prods.photons.pz[:k].cpu().numpy()]), axis=0)
    g_before = ws[0]["gamma"][idx]
    ok = g_after > 1.0 + 1e-6  # clamped recoils excluded
    assert np.max(rel(g_after[ok] + g_ph[ok], g_before[ok])) < 1e-9
    # sampled particles (random ones and emitters): the oracle's full step on each
    maps = {name: products_by_parent(prods, name) for name in ("photons", "electrons",
                                                              "positrons")}
    for w, tile, tau0, key in zip(ws, tiles, taus, ("photons", "electrons")):
        photon = w["species"] == sfq.PHOTON
        got = maps[key]
        base = np.uint64(w["uid"].view(np.uint64)[0])
        emitters = np.array([int(np.uint64(u) - base) for u in list(got)[:4000]], dtype=np.int64)
        assert emitters.size >= 60
        pick = np.unique(np.concatenate([rng.choice(n, 80, replace=False),
                                         rng.choice(emitters, 60, replace=False)]))
        uids = w["uid"].view(np.uint64)[pick]
        sub = {kk: w[kk][:, pick] for kk in ("p", "E", "B")}
        ref = O.step(w["species"], sub["p"], sub["E"], sub["B"], tau0[pick], uids, dt=h.dt,
                     lc_over_lr=h.lc_over_lr, seed=0, step=1)
        W = ref["rate"]
        rate = tile.rate_out.cpu().numpy()[pick]
        if mixed:
            # where e^{-8/(3chi)} of the pair rate underflows in FP32 (to zero, too), an
            # absolute tolerance
            tiny = np.finfo(np.float32).tiny * h.lr_over_lc
            assert np.all((np.abs(rate - W) <= tol_rate * W) | (np.abs(rate - W) <= tiny))
        else:
            assert np.array_equal(rate == 0, W == 0)
            assert np.max(rel(rate[W > 0], W[W > 0])) < tol_rate
        thr = W * h.dt
        in_band = np.abs(tau0[pick] - thr) <= band * np.maximum(tau0[pick], thr)
        emit_gpu = np.array([int(u) in got for u in uids])
        emitted = ref["emitted"].astype(bool)
        assert not ((emit_gpu != emitted) & ~in_band).any()
        assert (emitted & ~in_band).sum() >= 50
        # outcomes of the sampled emitters: recoil (leptons) and every product
        em = emitted & ~in_band
        if not photon:
            p_gpu = np.stack([tile.px.cpu().numpy()[pick], tile.py.cpu().numpy()[pick],
                              tile.pz.cpu().numpy()[pick]])
            assert np.max(vrel(p_gpu[:, em], ref["p"][:, em])) < tol_sample
            keep = ~emitted & ~in_band
            assert np.array_equal(p_gpu[:, keep], sub["p"][:, keep])
        band_uids = {int(u) for u in uids[in_band]}
        checked = 0
        for q in ref["products"]:
            if q["parent"] in band_uids:
                continue
            name = {O.PHOTON: "photons", O.ELECTRON: "electrons", O.POSITRON: "positrons"}[
                q["species"]]
            pv, tau_q, uid_q = maps[name][q["parent"]]
            assert uid_q == q["uid"] and abs(tau_q / q["tau"] - 1) < 1e-15
            assert vrel(pv, [q["px"], q["py"], q["pz"]]) < tol_sample, (name, q["parent"])
            checked += 1
        assert checked >= 50
