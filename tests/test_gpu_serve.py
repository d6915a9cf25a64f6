"""Serving on the GPU: per-tile product sets and step offsets, and the served form's
alone-vs-mix equality.

A step over tiles of several owners, each with its own product set and Philox step offset, must
give every owner exactly the particle state and the set of products it gets when stepped alone
(the arithmetic is identical; draws depend only on seed, uid, step and purpose).  The served
simulation's state after every step and its products must be the same whether it runs alone
or batched with other simulations of different sizes.
"""
import numpy as np
import pytest
import torch

from paper_2301_07684_amd import inputs, serve, sfq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def owner_tiles(dev, h, owner, sizes):
    tiles = []
    for k, (sp, n) in enumerate(sizes):
        w = inputs.plane_wave(n, seed=300 + 10 * owner + k, species=sp, chi_range=(1e-2, 50.0))
        uid = T(w["uid"], dev)
        tiles.append(sfq.TileArrays(sp, *[T(w["p"][i], dev) for i in range(3)],
                                    *[T(w["E"][i], dev) for i in range(3)],
                                    *[T(w["B"][i], dev) for i in range(3)],
                                    tau=h.init_optical_depth(uid, seed=2) * 0.05, uid=uid,
                                    alive=torch.ones(n, dtype=torch.uint8, device=dev)))
    return tiles


def clone(tiles, product_set=0, step_offset=0):
    out = []
    for t in tiles:
        out.append(sfq.TileArrays(t.species, t.px.clone(), t.py.clone(), t.pz.clone(), t.ex, t.ey,
                                  t.ez, t.bx, t.by, t.bz, tau=t.tau.clone(), uid=t.uid,
                                  alive=t.alive.clone(), product_set=product_set,
                                  step_offset=step_offset))
    return out


def state(tiles):
    return [torch.cat([t.px, t.py, t.pz, t.tau]).cpu().numpy() for t in tiles] + \
           [t.alive.cpu().numpy() for t in tiles]


def product_set(pb):
    c = pb.host_counts()
    out = []
    for k, name in enumerate(("photons", "electrons", "positrons")):
        ps = getattr(pb, name)
        n = min(c[k], ps.capacity)
        uid, parent = ps.uid[:n].cpu().numpy(), ps.parent[:n].cpu().numpy()
        order = np.lexsort((uid, parent))
        out.append(np.stack([uid, parent])[:, order])
        out.append(np.stack([getattr(ps, f)[:n].cpu().numpy() for f in ("px", "py", "pz", "tau")])
                   [:, order])
    return c, out


def same(a, b):
    return len(a) == len(b) and all(np.array_equal(x, y) for x, y in zip(a, b))


OWNERS = [[(sfq.ELECTRON, 3000), (sfq.PHOTON, 2000)],
          [(sfq.POSITRON, 700)],
          [(sfq.PHOTON, 5000), (sfq.ELECTRON, 1), (sfq.ELECTRON, 4100)]]
OFFSETS = [0, 17, 5]


@pytest.mark.parametrize("precision", [sfq.FP64, sfq.MIXED])
def test_product_sets_and_step_offsets_match_separate_steps(dev, precision):
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=precision)
    base = [owner_tiles(dev, h, o, sz) for o, sz in enumerate(OWNERS)]
    mixed, sets = [], []
    for o, tiles in enumerate(base):
        mixed += clone(tiles, product_set=o, step_offset=OFFSETS[o])
        sets.append(sfq.ProductBuffers.empty(6000, 6000, dev))
    cnt = sfq.Counters(dev)
    h.step(mixed, seed=11, step=100, counters=cnt, product_sets=sets)
    alone_c = sfq.Counters(dev)
    k = 0
    for o, tiles in enumerate(base):
        a = clone(tiles)
        pb = sfq.ProductBuffers.empty(6000, 6000, dev)
        h.step(a, seed=11, step=100 + OFFSETS[o], products=pb, counters=alone_c)
        torch.cuda.synchronize()
        assert same(state(a), state(mixed[k:k + len(a)])), o
        ca, pa = product_set(pb)
        cm, pm = product_set(sets[o])
        assert ca == cm and same(pa, pm), o
        k += len(a)
    assert cnt.results() == alone_c.results()
    assert cnt.as_dict()["emitted"] > 100 and cnt.as_dict()["converted"] > 10


def test_plan_with_product_sets_zeroes_every_set(dev):
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT)
    base = [owner_tiles(dev, h, o, sz) for o, sz in enumerate(OWNERS)]
    eager, planned, sets_e, sets_p = [], [], [], []
    for o, tiles in enumerate(base):
        eager += clone(tiles, product_set=o, step_offset=OFFSETS[o])
        planned += clone(tiles, product_set=o, step_offset=OFFSETS[o])
        sets_e.append(sfq.ProductBuffers.empty(6000, 6000, dev))
        sets_p.append(sfq.ProductBuffers.empty(6000, 6000, dev))
    ce, cp = sfq.Counters(dev), sfq.Counters(dev)
    plan = h.plan(planned, seed=3, step=40, counters=cp, product_sets=sets_p)
    plan.capture(1)
    for s in range(3):
        for pb in sets_e:
            pb.reset()
        h.step(eager, seed=3, step=40 + s, counters=ce, product_sets=sets_e)
        plan.replay()
        torch.cuda.synchronize()
        assert same(state(eager), state(planned)), s
        for a, b in zip(sets_e, sets_p):
            ca, pa = product_set(a)
            cb, pb_ = product_set(b)
            assert ca == cb and same(pa, pb_), s
    plan.close()


def test_product_set_validation(dev):
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT)
    tiles = clone(owner_tiles(dev, h, 0, [(sfq.ELECTRON, 100)]), product_set=1)
    with pytest.raises(sfq.SFQError):  # index beyond the sets
        h.step(tiles, seed=0, step=0, counters=sfq.Counters(dev),
               product_sets=[sfq.ProductBuffers.empty(10, 10, dev)])
    with pytest.raises(ValueError):    # a set index without sets
        h.step(tiles, seed=0, step=0, counters=sfq.Counters(dev),
               products=sfq.ProductBuffers.empty(10, 10, dev))


def _recorder(target_id, log):
    def on_step(sim):
        if sim.spec.job_id != target_id:
            return
        torch.cuda.synchronize()
        st = [x.cpu().numpy().copy() for x in (sim.p, sim.fperp, sim.dfperp, sim.just_created,
                                                 sim.k, sim.alive)]
        log.append((sim.step, sim.last_batch, st, product_set(sim.products)))
    return on_step


def test_served_results_are_the_same_alone_and_in_the_mix(dev):
    target = serve.JobSpec(0, 30000, 20000, steps=6)
    others = [serve.JobSpec(1, 120000, 40000, steps=9, client=1),
              serve.JobSpec(2, 5000, 90000, steps=4, arrival=0.001, client=2),
              serve.JobSpec(3, 60000, 1, steps=7, arrival=0.002, client=3),
              serve.JobSpec(4, 20000, 20000, steps=5, arrival=0.003, client=4)]
    logs = {}
    # the lanes' emitter queues are charged to the budget before any simulation
    probe = serve.Server(dev, hbm_budget=1 << 30, lanes=1, max_batch_particles=1 << 22)
    lane_queue = probe.queue_bytes
    assert 0 < lane_queue and probe.sched.budget == (1 << 30) - lane_queue
    probe.close()
    for name, jobs, lanes, budget in (("alone", [target], 1, 1 << 30),
                                      ("mix", [target] + others, 2, 1 << 30),
                                      ("mix_tight", [target] + others, 1,
                                       lane_queue + target.footprint + others[0].footprint
                                       + 4096)):
        log = []
        srv = serve.Server(dev, hbm_budget=budget, lanes=lanes, max_batch_particles=1 << 22,
                           on_step=_recorder(0, log))
        srv.add_jobs(jobs)
        res = srv.run(time_limit=120)
        srv.close()
        assert res["jobs"] == len(jobs) and res["requests"] == sum(j.steps for j in jobs)
        assert res["counters"]["overflow"] == 0
        logs[name] = (log, res)
    alone = logs["alone"][0]
    assert [s for s, *_ in alone] == list(range(1, 7)) and all(b == 1 for _, b, *_ in alone)
    for name in ("mix", "mix_tight"):
        log, res = logs[name]
        assert [s for s, *_ in log] == list(range(1, 7))
        assert max(b for _, b, *_ in log) > 1, name  # the target really was batched with others
        for (s, _, st_a, pr_a), (_, _, st_m, pr_m) in zip(alone, log):
            assert same(st_a, st_m), (name, s)
            assert pr_a[0] == pr_m[0] and same(pr_a[1], pr_m[1]), (name, s)
    # the tight budget made later simulations wait for admission
    assert logs["mix_tight"][1]["waited"] > 0
    tot = logs["mix"][1]["counters"]
    assert tot["emitted"] > 0 and tot["blcfa_rejected"] >= 0


def test_step_zeroes_product_counts(dev):
    """zero_product_counts=True: the buffers (one set, or every set) hold this step's products
    only, exactly as fresh buffers would."""
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT)
    base = [owner_tiles(dev, h, o, sz) for o, sz in enumerate(OWNERS)]
    flat = [t for tiles in base for t in tiles]
    used = sfq.ProductBuffers.empty(20000, 20000, dev)
    h.step(clone(flat), seed=1, step=1, products=used, counters=sfq.Counters(dev))
    assert sum(used.host_counts()) > 0
    fresh = sfq.ProductBuffers.empty(20000, 20000, dev)
    a, b = clone(flat), clone(flat)
    h.step(a, seed=1, step=2, products=used, counters=sfq.Counters(dev), zero_product_counts=True)
    h.step(b, seed=1, step=2, products=fresh, counters=sfq.Counters(dev))
    torch.cuda.synchronize()
    assert same(state(a), state(b))
    ca, pa = product_set(used)
    cb, pb = product_set(fresh)
    assert ca == cb and same(pa, pb)
    # per-owner sets
    sets_used = [sfq.ProductBuffers.empty(6000, 6000, dev) for _ in OWNERS]
    sets_fresh = [sfq.ProductBuffers.empty(6000, 6000, dev) for _ in OWNERS]
    mixed = lambda: [t for o, tiles in enumerate(base) for t in clone(tiles, product_set=o)]
    h.step(mixed(), seed=1, step=1, counters=sfq.Counters(dev), product_sets=sets_used)
    a, b = mixed(), mixed()
    h.step(a, seed=1, step=2, counters=sfq.Counters(dev), product_sets=sets_used,
           zero_product_counts=True)
    h.step(b, seed=1, step=2, counters=sfq.Counters(dev), product_sets=sets_fresh)
    torch.cuda.synchronize()
    assert same(state(a), state(b))
    for x, y in zip(sets_used, sets_fresh):
        cx, px = product_set(x)
        cy, py = product_set(y)
        assert cx == cy and same(px, py)
