"""Host-side logic of the serving layer (no GPU): admission by HBM budget, batch formation,
percentiles and the job mix."""
import numpy as np
import pytest

from paper_2301_07684_amd import serve
from paper_2301_07684_amd.serve import JobSpec, Scheduler


def spec(j, n, steps=3, t=0.0):
    return JobSpec(j, n // 2, n - n // 2, steps, arrival=t)


def test_admission_is_fifo_under_the_budget():
    a, b, c = spec(0, 100000), spec(1, 400000), spec(2, 10000)
    budget = a.footprint + b.footprint - 1  # a and b do not fit together
    s = Scheduler(budget, 10 ** 9, 64)
    for x in (a, b, c):
        s.arrive(x)
    assert [x.job_id for x in s.admit()] == [0]
    # c would fit, but b arrived first and waits: no overtaking
    assert s.admit() == [] and s.used == a.footprint
    assert s.deferred == {1, 2}
    s.release(a)
    assert [x.job_id for x in s.admit()] == [1, 2]
    assert s.used == b.footprint + c.footprint <= budget
    s.release(b)
    s.release(c)
    assert s.used == 0


def test_a_job_larger_than_the_budget_is_refused():
    s = Scheduler(1000, 10 ** 9, 64)
    with pytest.raises(ValueError):
        s.arrive(spec(0, 100000))


def test_footprint_counts_state_and_products():
    j = spec(0, 2_000_000)
    per = (j.n_leptons * serve.LEPTON_BYTES + j.n_photons * serve.PHOTON_BYTES)
    assert j.footprint > per
    assert j.footprint - per == serve.PRODUCT_BYTES * (j.photon_capacity + 2 * j.pair_capacity) + 4096


def test_batches_take_ready_requests_in_order_up_to_the_limits():
    s = Scheduler(10 ** 12, 1000, 6)
    for n in (400, 300, 500, 100, 2000, 50):
        s.submit(n)
    size = lambda r: r
    tiles = lambda r: 2
    assert s.next_batch(size, tiles) == [400, 300]     # 400 + 300 + 500 > 1000
    assert s.next_batch(size, tiles) == [500, 100]     # + 2000 exceeds
    assert s.next_batch(size, tiles) == [2000]         # alone, even above the limit
    assert s.next_batch(size, tiles) == [50]
    assert s.next_batch(size, tiles) == []
    s2 = Scheduler(10 ** 12, 10 ** 9, 4)               # tile limit: 2 requests of 2 tiles
    for n in range(5):
        s2.submit(n)
    assert s2.next_batch(size, tiles) == [0, 1]


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert serve.percentile(v, 50) == 50 and serve.percentile(v, 99) == 99
    assert serve.percentile(v, 100) == 100 and serve.percentile([7.0], 99) == 7.0
    assert np.isnan(serve.percentile([], 50))


def test_workload_mix():
    w = serve.workload(clients=8, jobs_per_client=50, steps=5)
    n = np.array([j.n_leptons + j.n_photons for j in w])
    assert len(w) == 400 and len({j.job_id for j in w}) == 400
    assert n.min() >= 10_000 and n.max() <= 20_000_000
    assert 1.4e6 < n.mean() < 2.6e6            # Exp(2e6) clamped
    assert {j.client for j in w} == set(range(8))
    seeds = {j.seed for j in w}
    assert len(seeds) == 400 and all((s + 2) not in seeds for s in seeds)  # distinct uids
    assert w == serve.workload(clients=8, jobs_per_client=50, steps=5)     # seeded


def test_device_generator_matches_numpy_draws():
    torch = pytest.importorskip("torch")
    from paper_2301_07684_amd import inputs

    idx = np.arange(20000)
    for seed, st in ((102, 10), (serve.JobSpec(7, 1, 1, 1).seed, 3), (2 ** 40 + 5, 91)):
        a = inputs.uniforms(seed, st, idx)
        b = inputs.uniforms_t(seed, st, torch.from_numpy(idx.astype(np.int64))).numpy()
        assert np.array_equal(a, b)
    for sp in (0, 2):
        w, wt = inputs.plane_wave(3000, species=sp), inputs.plane_wave_t(3000, "cpu", species=sp)
        assert np.array_equal(wt["uid"].numpy(), w["uid"])
        assert np.allclose(wt["p"].numpy(), w["p"], rtol=1e-14, atol=0)
        assert np.allclose(wt["E"].numpy(), w["E"], rtol=1e-13, atol=1e-13)
