"""Nothing outside a tile is written: tiles are views into larger buffers, with sentinel values
before, between and after them, and every step form (optical-depth and local decisions, FP64 and
MIXED, with and without the fused push, array and plane-wave fields, beyond-LCFA) must leave the
sentinels bit for bit; and a step that zeroes its product counts leaves exactly its own products
in the buffers.  The streaming kernels write every slot of a chunk (whole cache lines),
so the chunk tails of ragged tiles are where a missing bound would show.  Paper: Montefiori &
Tamburini, arXiv:2301.07684 (the step of Sec. 2-4 and Sec. 5 acts on the given particles only).
"""
import numpy as np
import pytest
import torch

from paper_2301_07684_amd import inputs, sfq

pytestmark = pytest.mark.gpu

GAP = 300          # sentinel slots before, between and after the tiles
SIZES = (1000, 4097, 257)   # ragged tiles: chunk tails of every kind
SENT = -12345.678  # a value the step never writes


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


class Padded:
    """One buffer per array, holding every tile at an offset, sentinels elsewhere."""

    def __init__(self, dev, width=1):
        self.offs, pos = [], GAP
        for n in SIZES:
            self.offs.append(pos)
            pos += width * n + GAP
        self.total = pos
        self.dev = dev
        self.width = width

    def make(self, values, dtype, sentinel):
        buf = torch.full((self.total,), sentinel, dtype=dtype, device=self.dev)
        for k, (o, n) in enumerate(zip(self.offs, SIZES)):
            buf[o:o + self.width * n] = values[k]
        return buf

    def views(self, buf):
        return [buf[o:o + self.width * n] for o, n in zip(self.offs, SIZES)]

    def mask(self):
        m = np.ones(self.total, dtype=bool)
        for o, n in zip(self.offs, SIZES):
            m[o:o + self.width * n] = False
        return m


def build(dev, species, *, seed, fields, blcfa, h):
    pad, pad3 = Padded(dev), Padded(dev, 3)
    ws = [inputs.plane_wave(n, idx=np.arange(n) + 7919 * k, seed=seed, species=species)
          for k, n in enumerate(SIZES)]
    f64, u8 = torch.float64, torch.uint8
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    bufs = {}
    for c, name in enumerate(("px", "py", "pz")):
        bufs[name] = pad.make([T(w["p"][c]) for w in ws], f64, SENT)
    if fields == "arrays":
        for c, name in enumerate(("ex", "ey", "ez")):
            bufs[name] = pad.make([T(w["E"][c]) for w in ws], f64, SENT)
        for c, name in enumerate(("bx", "by", "bz")):
            bufs[name] = pad.make([T(w["B"][c]) for w in ws], f64, SENT)
    else:
        bufs["wave_amp"] = pad.make([T(w["wave_a"]) for w in ws], f64, SENT)
        bufs["wave_phase"] = pad.make([T(w["wave_phase"]) for w in ws], f64, SENT)
    bufs["uid"] = pad.make([T(w["uid"]) for w in ws], torch.int64, -7)
    alive = [torch.from_numpy((np.arange(n) % 5 != 3).astype(np.uint8)) for n in SIZES]
    bufs["alive"] = pad.make(alive, u8, 77)
    if not (blcfa and species != sfq.PHOTON):
        tau = [h.init_optical_depth(T(w["uid"]).to(dev), seed=seed).cpu() * 0.02 for w in ws]
        bufs["tau"] = pad.make(tau, f64, SENT)
    if blcfa and species != sfq.PHOTON:
        bufs["fperp"] = pad3.make([torch.full((3 * n,), 0.5, dtype=f64) for n in SIZES], f64,
                                  SENT)
        bufs["dfperp"] = pad3.make([torch.zeros(3 * n, dtype=f64) for n in SIZES], f64, SENT)
        bufs["just_created"] = pad.make([torch.zeros(n, dtype=u8) for n in SIZES], u8, 77)
    tiles = []
    for k in range(len(SIZES)):
        v = {name: (pad3 if name in ("fperp", "dfperp") else pad).views(b)[k]
             for name, b in bufs.items()}
        kw = dict(uid=v["uid"], alive=v["alive"])
        if "tau" in v:
            kw["tau"] = v["tau"]
        if "fperp" in v:
            kw.update(fperp=v["fperp"], dfperp=v["dfperp"], just_created=v["just_created"])
        if fields == "arrays":
            fk = {name: v[name] for name in ("ex", "ey", "ez", "bx", "by", "bz")}
        else:
            fk = dict(field_mode=sfq.FIELDS_PLANE_WAVE, wave_amp=v["wave_amp"],
                      wave_phase=v["wave_phase"], wave_k=(1.0, 0.0, 0.0),
                      wave_pol=(0.0, 1.0, 0.0))
        tiles.append(sfq.TileArrays(species, v["px"], v["py"], v["pz"], **fk, **kw))
    masks = {name: (pad3 if name in ("fperp", "dfperp") else pad).mask() for name in bufs}
    return tiles, bufs, masks


def snapshot(bufs, masks):
    return {name: b.cpu().numpy()[masks[name]].copy() for name, b in bufs.items()}


@pytest.mark.parametrize("form", ["fp64", "mixed", "local", "fp64_push", "wave", "wave_push",
                                  "blcfa_push", "blcfa_wave_push"])
def test_steps_write_nothing_outside_the_tiles(dev, form):
    precision = sfq.MIXED if form == "mixed" else sfq.FP64
    blcfa = form.startswith("blcfa")
    local = form == "local" or blcfa
    push = form.endswith("push")
    fields = "wave" if "wave" in form else "arrays"
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=precision,
                   decision=sfq.LOCAL if local else sfq.OPTICAL_DEPTH, blcfa=blcfa)
    h.set_launch(2, 1024)
    tiles, bufs, masks = [], {}, {}
    for species in (sfq.ELECTRON, sfq.POSITRON, sfq.PHOTON):
        t, b, m = build(dev, species, seed=40 + species, fields=fields, blcfa=blcfa, h=h)
        tiles += t
        bufs.update({f"{species}:{k}": v for k, v in b.items()})
        masks.update({f"{species}:{k}": v for k, v in m.items()})
    before = snapshot(bufs, masks)
    prods = sfq.ProductBuffers.empty(20000, 8000, dev)
    cnt = sfq.Counters(dev)
    for step in range(1, 4):
        h.step(tiles, seed=3, step=step, products=prods, counters=cnt, push=push,
               zero_product_counts=True)
    torch.cuda.synchronize()
    c = cnt.as_dict()
    assert c["processed"] > 0 and c["overflow"] == 0
    assert c["emitted"] > 0, "the check needs emitters (holes in the written lines)"
    after = snapshot(bufs, masks)
    for name in before:
        assert np.array_equal(before[name].view(np.uint8), after[name].view(np.uint8)), name
    # zero_product_counts: the buffers hold exactly the last step's products
    last = sfq.Counters(dev)
    h.step(tiles, seed=3, step=4, products=prods, counters=last, push=push,
           zero_product_counts=True)
    torch.cuda.synchronize()
    c = last.as_dict()
    assert prods.host_counts() == [c["emitted"], c["converted"], c["converted"]]
    h.close()
