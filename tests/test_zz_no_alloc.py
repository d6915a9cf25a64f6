"""sfq_step_noalloc (the step that allocates nothing) against sfq_step.

The no-allocation entry point runs the same kernels on scratch in the library's static device
array, so two calls in a row -- the second on a smaller input, over what the first left in the
array -- must give bit for bit the particle state, the same set of products and the same result
counters as sfq_step on the same inputs (the order of products in their buffers may differ).
Called through the C ABI (the binding's step_noalloc marshals the same descriptor as step).
"""
import numpy as np
import pytest
import torch

from paper_2301_07684_amd import inputs, sfq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


STATE = ("px", "py", "pz", "tau", "alive")


def state(tiles):
    return [getattr(t, f).cpu().numpy().copy() for t in tiles for f in STATE
            if getattr(t, f) is not None]


def product_set(pb):
    c = pb.host_counts()
    out = [np.array(c)]
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
    return len(a) == len(b) and all(np.array_equal(x, y) for x, y in zip(a, b))


def make_tiles(dev, h, n_e, n_g, seed, tau_scale=0.3):
    out = []
    for sp, n, s in ((sfq.ELECTRON, n_e, seed), (sfq.PHOTON, n_g, seed + 1)):
        w = inputs.plane_wave(n, seed=s, species=sp)
        uid = T(w["uid"], dev)
        out.append(sfq.TileArrays(sp, *[T(w["p"][i], dev) for i in range(3)],
                                  *[T(w["E"][i], dev) for i in range(3)],
                                  *[T(w["B"][i], dev) for i in range(3)],
                                  tau=h.init_optical_depth(uid, seed=4) * tau_scale, uid=uid,
                                  alive=torch.ones(n, dtype=torch.uint8, device=dev)))
    return out


def clone(tiles):
    return [sfq.TileArrays(t.species, t.px.clone(), t.py.clone(), t.pz.clone(), t.ex, t.ey, t.ez,
                           t.bx, t.by, t.bz, tau=t.tau.clone(), uid=t.uid, alive=t.alive.clone())
            for t in tiles]


@pytest.mark.parametrize("precision", [sfq.FP64, sfq.MIXED])
def test_noalloc_step_matches_step_twice_second_smaller(dev, precision):
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=precision)
    # the first call emits so much (almost every electron, most photons) that the static queue
    # defers shares; the second, smaller one runs over what the first left in the array
    for k, (n_e, n_g, ts) in enumerate(((1 << 22, 1 << 22, 1e-4), (70001, 3333, 0.3))):
        base = make_tiles(dev, h, n_e, n_g, 1300 + 10 * k, tau_scale=ts)
        ref, na = clone(base), clone(base)
        pr = sfq.ProductBuffers.empty(n_e, n_g, dev)
        pn = sfq.ProductBuffers.empty(n_e, n_g, dev)
        cr, cn = sfq.Counters(dev), sfq.Counters(dev)
        h.step(ref, seed=3, step=10 + k, products=pr, counters=cr, zero_product_counts=True)
        h.step_noalloc(na, seed=3, step=10 + k, products=pn, counters=cn,
                       zero_product_counts=True)
        torch.cuda.synchronize()
        assert same(state(ref), state(na)), (k, "state")
        assert same(product_set(pr), product_set(pn)), (k, "products")
        assert cr.results() == cn.results(), (k, cr.as_dict(), cn.as_dict())
        c = cn.as_dict()
        assert c["processed"] == n_e + n_g and c["emitted"] > 100 and c["overflow"] == 0
        if k == 0:
            assert c["deferred"] > 0  # the static queue was too small for some shares


def test_noalloc_step_with_push_and_product_sets(dev):
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, decision=sfq.LOCAL)
    base = make_tiles(dev, h, 200000, 100000, 1400)
    ref, na = clone(base), clone(base)
    for k, t in enumerate(ref + na):
        t.product_set = k % 2
    sr = [sfq.ProductBuffers.empty(200000, 50000, dev) for _ in range(2)]
    sn = [sfq.ProductBuffers.empty(200000, 50000, dev) for _ in range(2)]
    cr, cn = sfq.Counters(dev), sfq.Counters(dev)
    for s in range(2):
        h.step(ref, seed=8, step=s, product_sets=sr, counters=cr, push=True,
               zero_product_counts=True)
        h.step_noalloc(na, seed=8, step=s, product_sets=sn, counters=cn, push=True,
                       zero_product_counts=True)
        torch.cuda.synchronize()
        assert same(state(ref), state(na)), s
        for a, b in zip(sr, sn):
            assert same(product_set(a), product_set(b)), s
    assert cr.results() == cn.results()
