"""Plans, graph capture and the autotuner: the same results as plain sfq_step calls.

A plan launch and a graph replay must give bit-identical particle states and the same set of
products as the equivalent sequence of sfq_step calls (the arithmetic is the same; only launch
plumbing differs).  Graph replays are checked after every replay, with eager work and
synchronisations in between.
"""
import numpy as np
import pytest
import torch

from paper_2301_07684_amd import autotune, inputs, sfq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def make_tiles(dev, h, sizes=(5000, 1, 3000, 700)):
    tiles = []
    for k, n in enumerate(sizes):
        sp = [sfq.ELECTRON, sfq.PHOTON, sfq.POSITRON, sfq.PHOTON][k % 4]
        w = inputs.plain_compton(n, seed=500 + k, species=sp)
        uid = T(w["uid"], dev)
        tau = h.init_optical_depth(uid, seed=3) * 0.2
        tiles.append(sfq.TileArrays(sp, *[T(w["p"][i], dev) for i in range(3)],
                                    *[T(w["E"][i], dev) for i in range(3)],
                                    *[T(w["B"][i], dev) for i in range(3)], tau=tau, uid=uid,
                                    alive=torch.ones(n, dtype=torch.uint8, device=dev)))
    return tiles


def clone_tiles(tiles):
    out = []
    for t in tiles:
        kw = {f: (getattr(t, f).clone() if getattr(t, f) is not None else None)
              for f in ("px", "py", "pz", "tau", "alive")}
        out.append(sfq.TileArrays(t.species, kw["px"], kw["py"], kw["pz"], t.ex, t.ey, t.ez, t.bx,
                                  t.by, t.bz, tau=kw["tau"], uid=t.uid, alive=kw["alive"]))
    return out


def state(tiles):
    return [torch.cat([t.px, t.py, t.pz, t.tau]).cpu().numpy() for t in tiles] + \
           [t.alive.cpu().numpy() for t in tiles]


def product_set(pb):
    """Products of the last step per species, sorted by (parent, uid): their order in the
    buffers depends on block scheduling, their contents do not."""
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
    return out


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("precision", [sfq.FP64, sfq.MIXED])
def test_plan_and_graph_match_step(dev, precision):
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=precision)
    base = make_tiles(dev, h)
    eager, planned, graphed = clone_tiles(base), clone_tiles(base), clone_tiles(base)
    pe, pp, pg = (sfq.ProductBuffers.empty(20000, 20000, dev) for _ in range(3))
    ce, cp, cg = sfq.Counters(dev), sfq.Counters(dev), sfq.Counters(dev)
    plan = h.plan(planned, seed=9, step=10, products=pp, counters=cp)
    gplan = h.plan(graphed, seed=9, step=10, products=pg, counters=cg)
    gplan.capture(2)  # one replay = two steps
    for rep in range(3):
        for k in range(2):
            pe.reset()
            h.step(eager, seed=9, step=10 + 2 * rep + k, products=pe, counters=ce)
            plan.launch()
            torch.cuda.synchronize()
            assert same(state(eager), state(planned)), (rep, k)
            assert same(product_set(pe), product_set(pp))
        gplan.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device=dev).sum().item()  # eager work between replays
        assert same(state(eager), state(graphed)), rep
        assert same(product_set(pe), product_set(pg)), rep  # the last step's products
    assert ce.results() == cp.results() == cg.results()
    plan.close()
    gplan.close()


def test_plan_set_step(dev):
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT)
    base = make_tiles(dev, h, sizes=(3000,))
    a, b = clone_tiles(base), clone_tiles(base)
    pa, pb = sfq.ProductBuffers.empty(5000, 1, dev), sfq.ProductBuffers.empty(5000, 1, dev)
    ca, cb = sfq.Counters(dev), sfq.Counters(dev)
    plan = h.plan(a, seed=1, step=0, products=pa, counters=ca)
    plan.set_step(77)
    plan.launch()
    h.step(b, seed=1, step=77, products=pb, counters=cb)
    torch.cuda.synchronize()
    assert same(state(a), state(b))


def test_autotune_restores_state_and_picks_a_candidate(dev, tmp_path):
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=sfq.MIXED)
    base = make_tiles(dev, h, sizes=(40000, 20000, 30000))
    tuned, ref = clone_tiles(base), clone_tiles(base)
    pt, pr = sfq.ProductBuffers.empty(90000, 90000, dev), sfq.ProductBuffers.empty(90000, 90000, dev)
    ct, cr = sfq.Counters(dev), sfq.Counters(dev)
    cache = str(tmp_path / "tune.json")
    res = autotune.tune(h, tuned, pt, ct, cache_path=cache, repeats=2)
    assert tuple(res["shape"]) in autotune.DEFAULT_CANDIDATES and not res["cached"]
    assert h.get_launch() == tuple(res["shape"])
    assert same(state(tuned), state(base))  # tuning left the particles as they were
    assert ct.as_dict()["processed"] == 0 and pt.host_counts() == [0, 0, 0]
    res2 = autotune.tune(h, tuned, pt, ct, cache_path=cache)
    assert res2["cached"] and res2["shape"] == res["shape"]
    h.step(tuned, seed=2, step=5, products=pt, counters=ct)
    h.set_launch(4, 2048)
    h.step(ref, seed=2, step=5, products=pr, counters=cr)
    torch.cuda.synchronize()
    assert same(state(tuned), state(ref))  # launch shapes never change results
    assert same(product_set(pt), product_set(pr))
    # the pushed form is tuned on its own kernels, under its own cache entry, and its
    # momenta (which the timed steps push) come back as they were
    pushed = clone_tiles(base)
    res3 = autotune.tune(h, pushed, pt, ct, cache_path=cache, repeats=2, push=True)
    assert not res3["cached"] and tuple(res3["shape"]) in autotune.DEFAULT_CANDIDATES
    assert same(state(pushed), state(base))
    assert autotune.signature(h, pushed, True) != autotune.signature(h, pushed, False)
    assert len(autotune.load_cache(cache)) == 2


def test_autotune_keeps_products_already_in_the_buffers(dev, tmp_path):
    # the timed launches write their products from slot 0; the caller's products come back
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT)
    tiles = make_tiles(dev, h, sizes=(20000, 6000))
    pb, cnt = sfq.ProductBuffers.empty(60000, 60000, dev), sfq.Counters(dev)
    h.step(clone_tiles(tiles), seed=7, step=1, products=pb, counters=cnt)
    torch.cuda.synchronize()
    before = product_set(pb)
    counts = pb.host_counts()
    assert counts[0] > 100 and counts[1] > 0
    raw = [getattr(getattr(pb, sp), f)[:counts[k]].clone()
           for k, sp in enumerate(("photons", "electrons", "positrons"))
           for f in ("px", "py", "pz", "tau", "uid", "parent")]
    autotune.tune(h, tiles, pb, cnt, cache_path=str(tmp_path / "t.json"), repeats=1,
                  candidates=[(2, 1024), (8, 2048)])
    assert pb.host_counts() == counts
    assert same(product_set(pb), before)
    raw2 = [getattr(getattr(pb, sp), f)[:counts[k]]
            for k, sp in enumerate(("photons", "electrons", "positrons"))
            for f in ("px", "py", "pz", "tau", "uid", "parent")]
    assert all(torch.equal(a, b) for a, b in zip(raw, raw2))  # in place, in the same order


def test_reserve_and_kernel_timing(dev):
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT)
    h.reserve(50000, 4)
    base = make_tiles(dev, h)
    a, b = clone_tiles(base), clone_tiles(base)
    pa, pb = sfq.ProductBuffers.empty(20000, 20000, dev), sfq.ProductBuffers.empty(20000, 20000, dev)
    ca, cb = sfq.Counters(dev), sfq.Counters(dev)
    h.profile(True)
    for s in range(3):
        h.step(a, seed=5, step=s, products=pa, counters=ca)
    plan = h.plan(b, seed=5, step=0, products=pb, counters=cb, zero_product_counts=False)
    for s in range(3):
        plan.launch()
    bulk_ms, emit_ms, n = h.profile_read()
    assert n == 6 and bulk_ms > 0 and emit_ms > 0
    assert h.profile_read() == (0.0, 0.0, 0)  # cleared by the read
    # step by step: one entry per timed step, in order, summing to the totals
    for s in range(3, 6):
        h.step(a, seed=5, step=s, products=pa, counters=ca)
        plan.launch()
    with pytest.raises(sfq.SFQError):
        h.profile_read_steps(5)          # more steps pending than room: nothing cleared
    bulk, emit = h.profile_read_steps(6)
    assert len(bulk) == len(emit) == 6 and np.all(bulk > 0) and np.all(emit > 0)
    assert h.profile_read() == (0.0, 0.0, 0)
    h.profile(False)
    h.step(a, seed=5, step=6, products=pa, counters=ca)
    torch.cuda.synchronize()
    assert h.profile_read()[2] == 0
    plan.launch()
    torch.cuda.synchronize()
    assert same(state(a), state(b)) and same(product_set(pa), product_set(pb))
    # steps timed whole (two events per step): the step's time, and 0 for the emitter pass;
    # a split-timed step beside them keeps its split
    h.profile(True, whole_step=True)
    h.step(a, seed=5, step=7, products=pa, counters=ca)
    plan.launch()
    h.profile(True)
    h.step(a, seed=5, step=8, products=pa, counters=ca)
    whole, zero = h.profile_read_steps(3)
    assert len(whole) == 3 and np.all(whole > 0)
    assert zero[0] == 0 and zero[1] == 0 and zero[2] > 0
    h.profile(False)
    with pytest.raises(sfq.SFQError):
        h._check(h._L.sfq_profile_enable(h._h, 3))    # only 0, 1 and 2
    plan.close()
    with pytest.raises(sfq.SFQError):
        h.reserve(10, 0)


@pytest.mark.parametrize("precision", [sfq.FP64, sfq.MIXED])
def test_extreme_launch_shapes_give_identical_results(dev, precision):
    """16384 blocks of 256-particle chunks (each emitter block sums up to 16384 block totals) and
    1 block per CU with 2^22-particle chunks against the default shape: same state, same
    products."""
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=precision)
    base = make_tiles(dev, h, sizes=(1 << 21, 3, (1 << 21) + 77, 4096))
    results = []
    for shape in ((8, 2048), (64, 256), (1, 1 << 22)):
        h.set_launch(*shape)
        tiles = clone_tiles(base)
        pb = sfq.ProductBuffers.empty(1 << 22, 1 << 20, dev)
        cnt = sfq.Counters(dev)
        for s in range(2):
            h.step(tiles, seed=21, step=s, products=pb, counters=cnt)
        torch.cuda.synchronize()
        results.append((state(tiles), product_set(pb), cnt.results()))
    c0 = results[0][2]
    assert c0["emitted"] > 1000 and c0["overflow"] == 0
    for st, ps, c in results[1:]:
        assert same(st, results[0][0]) and same(ps, results[0][1]) and c == c0


def test_select_form_dial(dev):
    """The accuracy/speed dial times only the forms within the error budget, returns the fastest
    with its error bound, leaves the particle state as it was, and its handle steps exactly like
    a fresh handle of the chosen form."""
    kw = dict(ref_length=inputs.LAMBDA_R, dt=inputs.DT)
    h0 = sfq.Handle(**kw)
    tiles = make_tiles(dev, h0, sizes=(40000, 30000, 20000, 10000))
    before = state(tiles)
    prods = sfq.ProductBuffers.empty(100000, 100000, dev)
    cnt = sfq.Counters(dev)
    cand = [(2, 4096), (8, 1024)]
    errs = autotune.form_errors()
    fp64 = errs[(sfq.FP64, sfq.APPROX_FULL)]
    r = autotune.select_form(kw, tiles, prods, cnt, max_rel_error=1e-8, candidates=cand, repeats=2)
    assert r["precision"] == sfq.FP64 and not r["bw_fast"] and list(r["timings"]) == ["fp64"]
    assert r["approx"] == sfq.APPROX_FULL
    assert r["error_bound"] == {"rate": fp64["rate"], "sample": fp64["sample"]}
    assert all(np.array_equal(a, b) for a, b in zip(before, state(tiles)))
    r["handle"].close()
    # the truncated forms' bounds come from the table generator's measured report
    assert errs[(sfq.FP64, sfq.APPROX_TRUNCATED)]["sample"] > fp64["sample"]
    r = autotune.select_form(kw, tiles, prods, cnt, max_rel_error=1e-4, allow_bw_fast=True,
                             candidates=cand, repeats=2)
    assert set(r["timings"]) == {f + b for f in ("fp64", "mixed", "fp64_trunc", "mixed_trunc")
                                 for b in ("", "+bw_fast")}
    assert r["ms"] == min(r["timings"].values())
    assert ("bw_fast" in r["error_bound"]) == r["bw_fast"]
    assert all(np.array_equal(a, b) for a, b in zip(before, state(tiles)))
    assert prods.host_counts() == [0, 0, 0] and cnt.as_dict()["processed"] == 0
    # the chosen handle is ready to use and gives the results of its form
    a, b = clone_tiles(tiles), clone_tiles(tiles)
    pa, pb = sfq.ProductBuffers.empty(100000, 100000, dev), sfq.ProductBuffers.empty(100000, 100000, dev)
    r["handle"].step(a, seed=4, step=2, products=pa, counters=sfq.Counters(dev))
    ref = sfq.Handle(**kw, precision=r["precision"], bw_fast=r["bw_fast"], approx=r["approx"])
    ref.step(b, seed=4, step=2, products=pb, counters=sfq.Counters(dev))
    torch.cuda.synchronize()
    assert all(np.array_equal(x, y) for x, y in zip(state(a), state(b)))
    assert same(product_set(pa), product_set(pb))
    r["handle"].close()
    ref.close()
    with pytest.raises(ValueError):
        autotune.select_form(kw, tiles, prods, cnt, max_rel_error=1e-13)


def test_one_handle_on_two_streams(dev):
    """sfq_step calls of one handle on two streams, enqueued back to back with no host
    synchronisation, give what sequential steps give (the handle orders its queue use)."""
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT)
    ref_h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT)
    a = make_tiles(dev, h, sizes=(300000, 1000))
    b = make_tiles(dev, h, sizes=(5000, 200000, 7000))
    ra, rb = clone_tiles(a), clone_tiles(b)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    pa, pb = sfq.ProductBuffers.empty(400000, 400000, dev), sfq.ProductBuffers.empty(400000, 400000, dev)
    qa, qb = sfq.ProductBuffers.empty(400000, 400000, dev), sfq.ProductBuffers.empty(400000, 400000, dev)
    ca, cb = sfq.Counters(dev), sfq.Counters(dev)
    torch.cuda.synchronize()
    for step in range(3):
        h.step(a, seed=6, step=step, products=pa, counters=ca, stream=s1)
        h.step(b, seed=6, step=step, products=pb, counters=cb, stream=s2)
    torch.cuda.synchronize()
    rca, rcb = sfq.Counters(dev), sfq.Counters(dev)
    for step in range(3):
        ref_h.step(ra, seed=6, step=step, products=qa, counters=rca)
        ref_h.step(rb, seed=6, step=step, products=qb, counters=rcb)
    torch.cuda.synchronize()
    assert same(state(a), state(ra)) and same(state(b), state(rb))
    assert pa.host_counts() == qa.host_counts() and pb.host_counts() == qb.host_counts()
    assert same(product_set(pa), product_set(qa)) and same(product_set(pb), product_set(qb))
    assert ca.results() == rca.results() and cb.results() == rcb.results()
    assert ca.as_dict()["processed"] > 3 * 300000 and ca.as_dict()["overflow"] == 0
    assert cb.as_dict()["overflow"] == 0


def test_maximum_tile_count_and_overflow_rerun(dev):
    """SFQ_MAX_TILES ragged tiles (sizes 0..40, mixed species) give what the same particles give
    in one tile per species; one tile more is refused.  A step that overflows its product
    buffers, re-run from the restored state with buffers of the size it reported, gives what a
    step with large buffers gives."""
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT)
    sizes = (inputs.uniforms(5, 0, np.arange(sfq.MAX_TILES)) * 41).astype(int)
    species = [sfq.ELECTRON, sfq.POSITRON, sfq.PHOTON]
    tot = [int(sizes[k::3].sum()) for k in range(3)]
    big = []
    for k, sp in enumerate(species):
        w = inputs.plain_compton(tot[k], seed=600 + k, species=sp)
        uid = T(w["uid"], dev)
        big.append(sfq.TileArrays(sp, *[T(w["p"][i], dev) for i in range(3)],
                                  *[T(w["E"][i], dev) for i in range(3)],
                                  *[T(w["B"][i], dev) for i in range(3)],
                                  tau=h.init_optical_depth(uid, seed=4) * 0.3, uid=uid,
                                  alive=torch.ones(tot[k], dtype=torch.uint8, device=dev)))
    ref = clone_tiles(big)
    # the same particles cut into MAX_TILES views, species cycling
    small, pos = [], [0, 0, 0]
    for t in range(sfq.MAX_TILES):
        k, n = t % 3, int(sizes[t])
        b = big[k]
        sl = slice(pos[k], pos[k] + n)
        small.append(sfq.TileArrays(b.species, b.px[sl], b.py[sl], b.pz[sl], b.ex[sl], b.ey[sl],
                                    b.ez[sl], b.bx[sl], b.by[sl], b.bz[sl], tau=b.tau[sl],
                                    uid=b.uid[sl], alive=b.alive[sl]))
        pos[k] += n
    assert pos == tot
    cap = sum(tot)
    pa, pr = sfq.ProductBuffers.empty(cap, cap, dev), sfq.ProductBuffers.empty(cap, cap, dev)
    ca, cr = sfq.Counters(dev), sfq.Counters(dev)
    h.step(small, seed=8, step=6, products=pa, counters=ca)
    h.step(ref, seed=8, step=6, products=pr, counters=cr)
    torch.cuda.synchronize()
    assert same(state(big), state(ref))
    assert same(product_set(pa), product_set(pr)) and ca.results() == cr.results()
    assert ca.as_dict()["emitted"] > 100 and ca.as_dict()["converted"] > 10
    with pytest.raises(ValueError):
        h.step(small + small[:1], seed=8, step=6, products=pa, counters=ca)
    # overflow, then re-run with the reported sizes
    base = clone_tiles(ref)
    a = clone_tiles(base)
    tiny = sfq.ProductBuffers.empty(16, 4, dev)
    ct = sfq.Counters(dev)
    h.step(a, seed=3, step=1, products=tiny, counters=ct)
    torch.cuda.synchronize()
    need = tiny.host_counts()
    assert ct.as_dict()["overflow"] > 0 and need[0] > 16
    b = clone_tiles(base)
    fit = sfq.ProductBuffers.empty(need[0], max(need[1], need[2]), dev)
    cf = sfq.Counters(dev)
    h.step(b, seed=3, step=1, products=fit, counters=cf)
    c = clone_tiles(base)
    large = sfq.ProductBuffers.empty(cap, cap, dev)
    h.step(c, seed=3, step=1, products=large, counters=sfq.Counters(dev))
    torch.cuda.synchronize()
    assert cf.as_dict()["overflow"] == 0 and fit.host_counts() == need
    assert same(state(a), state(c)) and same(state(b), state(c))
    assert same(product_set(fit), product_set(large))


def test_descriptor_reuse_follows_the_tiles(dev):
    """The handle reuses the device copy of the last uploaded tile descriptors when a step
    passes the same ones.  Alternating tile sets (A, A, B, A), new contents in the same arrays,
    and a new launch shape must all give what a fresh handle per step gives."""
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT)
    a = make_tiles(dev, h, sizes=(6000, 2000))
    b = make_tiles(dev, h, sizes=(3000, 500, 4000))
    ra, rb = clone_tiles(a), clone_tiles(b)
    pb_, qb_ = sfq.ProductBuffers.empty(20000, 20000, dev), sfq.ProductBuffers.empty(20000, 20000, dev)
    seq = [("a", 0), ("a", 1), ("b", 0), ("a", 2), ("a", 3)]
    for which, step in seq:
        t, r = (a, ra) if which == "a" else (b, rb)
        if step == 3:
            # new contents in the same arrays: same descriptors, different particles
            for x, y in zip(t, r):
                x.px.mul_(1.5)
                y.px.mul_(1.5)
            h.set_launch(4, 1024)      # and a new launch shape (new chunk offsets)
        h.step(t, seed=8, step=step, products=pb_, counters=sfq.Counters(dev),
               zero_product_counts=True)
        fresh = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT)
        fresh.step(r, seed=8, step=step, products=qb_, counters=sfq.Counters(dev),
                   zero_product_counts=True)
        torch.cuda.synchronize()
        assert same(state(t), state(r)), (which, step)
        assert pb_.host_counts() == qb_.host_counts()
        assert same(product_set(pb_), product_set(qb_)), (which, step)
        fresh.close()
    h.close()
