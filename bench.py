#!/usr/bin/env python3
"""Benchmark of the QED Monte Carlo step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Headline workload (the plain FP64 form at scale): 2^24 electrons + 2^24 photons
counter-propagating through a linearly polarised plane wave (a ~ U[10, 500], random phase,
gamma log-uniform [1e2, 1e5]), nonlinear Compton and Breit-Wheeler both active, optical-depth
decisions, dt = 0.01 fs, FP64 SoA arrays resident in HBM.  A step is one sfq_step over both
tiles (chi, rates, decisions, sampling, recoil, products).  Then, on the same GPU:
  * the MIXED form on the skewed-chi ensemble (chi log-uniform [1e-4, 1e3]), and on the
    headline workload itself (the FP32 / FP64 comparison on the same inputs);
  * the batched form: 64 uneven tiles of mixed species (sizes log-uniform 1e3..4e6, static-B
    geometry, chi log-uniform [1e-3, 1e2]), MIXED, launch shape from the autotuner, each step
    one replay of a HIP graph captured from a plan;
  * the served form: continuous batching of step requests from 8 clients' simulations with
    beyond-LCFA electrons, admitted under an HBM budget (request latency p50/p99);
  * the fused form: the headline workload with every electron's momentum pushed through its
    fields (Boris) inside the streaming kernel before the QED step;
  * the plane-wave-fields form: the headline workload with its fields given as the plane wave
    they come from (per-particle amplitude and phase; E and B computed in the kernel);
  * the constant-field run: 2^30 electrons of 10 GeV at chi = 1 in a uniform magnetic field
    (one value per tile) for 1.3 fs, fused push, recoil.

Prints ONE JSON line: value = FP64 particle-updates/s over the timed steps (wall clock); p50/p99
step latency (each step's kernels, from before the streaming kernel to the end of the emitter
pass, with the library's timing-only HIP events on the step's stream; graph replays of the
batched form with events around each replay); the roofline of the dominant (streaming) kernel
from its own duration measured with those events; the other forms' numbers; and the CPU oracle timed on a bounded
sample on the host cores.  `--copy-calibration` instead times a plain device copy of known size
(the reference for HBM counter scaling) and exits.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-updates/sec (Compton+BW MC step) FP32 vs FP64; p99 step latency"
HBM_PEAK = 8.0e12  # B/s, MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_bulk_kernel_plane_wave_fp64.md")


def stream_kernel_bytes(n_flags, processed, emitted, converted):
    """Algorithmic bytes of the streaming kernel for one step (optical-depth decisions).  Every
    particle slot of a tile with alive flags (photons; leptons never die in the step and have
    none): its flag (1 B).  Every live particle: p (24), E and B (48) and the optical depth (8)
    read.  Every live particle that does not emit: the optical depth written back (8); emitters
    get a fresh depth in the emitter kernel.  The particle id is not needed here: only emitters
    use it (emitter kernel)."""
    return n_flags + 80 * processed + 8 * (processed - emitted - converted)


def survey_step_bytes(processed, emitted, converted):
    """The whole step's bytes as the scope table counts them (a fixed yardstick for the step's
    roofline fraction): 96 B per particle update (p, E, B, optical depth and id read, optical
    depth written), plus per Compton emission the emitter's momentum (24 B) and a photon
    product (48 B), per conversion two lepton products (96 B), and 8 B of queue traffic per
    event."""
    return 96 * processed + (24 + 48 + 8) * emitted + (96 + 8) * converted


def pushed_stream_kernel_bytes(n_flags, processed, emitted, converted, leptons):
    """The streaming kernel with the fused momentum push: as above, plus the pushed momentum
    (24 B) written back for every live lepton that does not emit (emitters' momenta are written
    after the recoil by the emitter kernel, as without the push)."""
    return stream_kernel_bytes(n_flags, processed, emitted, converted) + 24 * (leptons - emitted)


def emit_kernel_bytes(emitted, converted):
    """Algorithmic bytes of the emitter kernel for one step.  A Compton emission reads the
    emitter's id (8) and writes its momentum and optical depth (32) and one photon product
    (p 24, tau 8, uid 8, parent 8 = 48).  A conversion reads the photon's id (8) and writes its
    alive flag (1) and two lepton products (96)."""
    return 88 * emitted + 105 * converted


def wave_stream_kernel_bytes(n_flags, processed, emitted, converted):
    """The streaming kernel with plane-wave tiles (fields computed in the kernel): as
    stream_kernel_bytes, with the wave's amplitude and phase (16 B) read instead of E and B
    (48 B)."""
    return n_flags + 48 * processed + 8 * (processed - emitted - converted)


def device_tiles(dev, sfq, h, workloads, wave=False):
    import torch

    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    tiles = []
    for w in workloads:
        n = len(w["uid"])
        uid = t(w["uid"])
        if wave:  # the same fields, E_y = B_z = a cos(phase), computed in the step
            fields = dict(field_mode=sfq.FIELDS_PLANE_WAVE, wave_amp=t(w["wave_a"]),
                          wave_phase=t(w["wave_phase"]), wave_k=(1.0, 0.0, 0.0),
                          wave_pol=(0.0, 1.0, 0.0))
        else:
            fields = dict(ex=t(w["E"][0]), ey=t(w["E"][1]), ez=t(w["E"][2]), bx=t(w["B"][0]),
                          by=t(w["B"][1]), bz=t(w["B"][2]))
        # photons convert and die; leptons never die in the step and carry no alive flags
        alive = (torch.ones(n, dtype=torch.uint8, device=dev)
                 if int(w["species"]) == sfq.PHOTON else None)
        tiles.append(sfq.TileArrays(int(w["species"]), *[t(w["p"][k]) for k in range(3)],
                                    **fields, tau=h.init_optical_depth(uid, seed=0), uid=uid,
                                    alive=alive))
    return tiles


class StateReset:
    """The tiles' evolving state (momenta, optical depths, alive flags, beyond-LCFA state) as it
    was when made (or when the reset was created), put
    back by a device copy before every timed step, outside the step's timed events, so that each
    repeat steps the same ensemble (no converted photons pile up as dead slots).  A copy through
    an unrelated buffer after it leaves the caches as a step of its own would find them."""

    def __init__(self, tiles, dev, flush_bytes=512 << 20):
        import torch

        self.pairs = []
        for t in tiles:
            for f in ("px", "py", "pz", "tau", "alive", "fperp", "dfperp", "just_created"):
                v = getattr(t, f)
                if v is not None:
                    self.pairs.append((v, v.clone()))
        self.flush_src = torch.empty(flush_bytes // 8, dtype=torch.float64, device=dev)
        self.flush_dst = torch.empty_like(self.flush_src)

    def __call__(self):
        for dst, src in self.pairs:
            dst.copy_(src)
        self.flush_dst.copy_(self.flush_src)


def time_steps(h, tiles, prods, cnt, reset, steps, warmup, push=False):
    """Warm-up steps, then `steps` steps each timed whole on the step's stream by the library's
    timing events (before the streaming kernel and after the step's last kernel; no
    system-scope fence), the state put back by `reset` before each outside the timed region,
    then up to 10 more steps timed with the streaming/emitter split (a third event between the
    two passes, whose idle gap the split times include).  Every step zeroes the product counts
    itself: the buffers hold that step's products."""
    import torch

    for s in range(warmup):
        reset()
        h.step(tiles, seed=0, step=s + 1, products=prods, counters=cnt, push=push,
               zero_product_counts=True)
    torch.cuda.synchronize()
    cnt.reset()
    h.profile(True, whole_step=True)
    h.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        reset()
        h.step(tiles, seed=0, step=warmup + s + 1, products=prods, counters=cnt, push=push,
               zero_product_counts=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    whole, _ = h.profile_read_steps(steps)
    if len(whole) != steps:
        raise RuntimeError("the step timing events did not cover every timed step")
    step_ms = whole.astype(np.float64)           # per step: streaming kernel to the step's end
    c = cnt.as_dict()
    if c["overflow"]:
        raise RuntimeError("product buffers overflowed during the benchmark")
    h.profile(True)
    nsplit = min(steps, 10)
    for s in range(nsplit):
        reset()
        h.step(tiles, seed=0, step=warmup + steps + s + 1, products=prods, counters=cnt,
               push=push, zero_product_counts=True)
    bulk, emit = h.profile_read_steps(nsplit)
    h.profile(False)
    return dict(wall=wall, device_s=float(step_ms.sum()) * 1e-3, step_ms=step_ms, counters=c,
                bulk_ms=float(bulk.mean()), emit_ms=float(emit.mean()))


def run_form(precision, workload, n, steps, warmup, dev, launch=None, push=False, wave=False,
             approx=0):
    import torch

    from paper_2301_07684_amd import autotune, inputs, sfq

    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=precision, approx=approx)
    tiles = []
    for species in (sfq.ELECTRON, sfq.PHOTON):
        if workload == "plane_wave":
            w = inputs.plane_wave(n, species=species)
        else:
            w = inputs.plane_wave(n, seed=inputs.SEED_SKEW, species=species, chi_range=(1e-4, 1e3))
        tiles += device_tiles(dev, sfq, h, [w], wave=wave)
        del w
    n_flags = sum(t.n for t in tiles if t.alive is not None)
    prods = sfq.ProductBuffers.empty(n // 2, n // 8, dev)
    cnt = sfq.Counters(dev)
    if launch is None:
        tuned = autotune.tune(h, tiles, prods, cnt, seed=0, step=1, repeats=3, cache_path=None,
                              push=push)
    else:
        h.set_launch(*launch)
        tuned = {"shape": list(launch)}
    h.reserve(2 * n, 2)
    reset = StateReset(tiles, dev)
    r = time_steps(h, tiles, prods, cnt, reset, steps, warmup, push=push)
    qbytes = h.queue_bytes()
    h.close()
    del tiles, prods, reset
    torch.cuda.empty_cache()
    return dict(r, n_total=2 * n, n_flags=n_flags, shape=tuned["shape"], queue_bytes=qbytes)


def served_stream_kernel_bytes(n_leptons, n_flags, photons_live):
    """Algorithmic bytes of the streaming kernel of the served form's step (beyond-LCFA
    electrons pushed in the kernel, plane-wave tiles, local decisions, so no optical depths).
    Every electron: p, the wave's amplitude and phase, F_perp, dF, the id and the just-created
    flag read (97 B); the pushed p, F_perp, dF and the flag written (73 B).  Every photon slot:
    its alive flag (1 B); every live photon: p, the wave's amplitude and phase and the id read
    (48 B)."""
    return 170 * n_leptons + n_flags + 48 * photons_live


def run_served_step(n, steps, warmup, dev, launch=None):
    """The served form's kernels on one large step: n electrons with beyond-LCFA state and n
    photons as plane-wave tiles, the fused push, local decisions, MIXED (the kernels a served
    batch runs, without the serving loop's small batches and concurrent lanes)."""
    import torch

    from paper_2301_07684_amd import autotune, inputs, sfq

    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=sfq.MIXED,
                   decision=sfq.LOCAL, blcfa=True)
    e = inputs.plane_wave_t(n, dev, species=sfq.ELECTRON)
    g = inputs.plane_wave_t(n, dev, species=sfq.PHOTON)
    wave = dict(field_mode=sfq.FIELDS_PLANE_WAVE, wave_k=(1.0, 0.0, 0.0),
                wave_pol=(0.0, 1.0, 0.0))
    p, k = e["p"].contiguous(), g["p"].contiguous()
    fperp = torch.zeros(3 * n, dtype=torch.float64, device=dev)
    tiles = [sfq.TileArrays(sfq.ELECTRON, p[0], p[1], p[2], uid=e["uid"], fperp=fperp,
                            dfperp=torch.zeros_like(fperp),
                            just_created=torch.ones(n, dtype=torch.uint8, device=dev),
                            wave_amp=e["a"], wave_phase=e["phi"], **wave),
             sfq.TileArrays(sfq.PHOTON, k[0], k[1], k[2], uid=g["uid"],
                            alive=torch.ones(n, dtype=torch.uint8, device=dev),
                            wave_amp=g["a"], wave_phase=g["phi"], **wave)]
    del e, g
    prods = sfq.ProductBuffers.empty(n // 2, n // 8, dev)
    cnt = sfq.Counters(dev)
    # a particle's first beyond-LCFA step only records its force: three steps (the wave's
    # phase advancing) bring every electron to where it can emit
    for s in range(3):
        for t in tiles:
            t.wave_phase0 = 2.0 * inputs.DT * s
        h.step(tiles, seed=1, step=s + 1, products=prods, counters=cnt, push=True,
               zero_product_counts=True)
    if launch is None:
        tuned = autotune.tune(h, tiles, prods, cnt, seed=0, step=1, repeats=3, cache_path=None,
                              push=True)
    else:
        h.set_launch(*launch)
        tuned = {"shape": list(launch)}
    h.reserve(2 * n, 2)
    reset = StateReset(tiles, dev)
    r = time_steps(h, tiles, prods, cnt, reset, steps, warmup, push=True)
    h.close()
    del tiles, prods, reset, p, k, fperp
    torch.cuda.empty_cache()
    return dict(r, n_leptons=n, n_flags=n, shape=tuned["shape"])


def run_batched(steps, warmup, dev):
    """64 uneven tiles, MIXED, autotuned launch shape, one graph replay per step."""
    import torch

    from paper_2301_07684_amd import autotune, inputs, sfq

    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=sfq.MIXED)
    tiles = []
    for w in inputs.tiles():
        tiles += device_tiles(dev, sfq, h, [w])
    n_total = sum(t.n for t in tiles)
    n_lep = sum(t.n for t in tiles if t.species != sfq.PHOTON)
    prods = sfq.ProductBuffers.empty(n_lep // 3 + 1, (n_total - n_lep) // 8 + 1, dev)
    cnt = sfq.Counters(dev)
    tuned = autotune.tune(h, tiles, prods, cnt, seed=0, step=1, repeats=3)
    plan = h.plan(tiles, seed=0, step=1, products=prods, counters=cnt)
    plan.capture(1)
    stream = torch.cuda.current_stream()
    reset = StateReset(tiles, dev)
    for _ in range(warmup):
        reset()
        plan.replay()
    torch.cuda.synchronize()
    cnt.reset()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        reset()
        ev[s][0].record(stream)
        plan.replay()
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([a.elapsed_time(b) for a, b in ev])
    c = cnt.as_dict()
    if c["overflow"]:
        raise RuntimeError("product buffers overflowed during the batched benchmark")
    # the streaming / emitter split, from plan launches (the graph's kernels, outside the
    # graph) timed with the library's events
    h.profile(True)
    h.profile_read()
    for s in range(min(steps, 10)):
        reset()
        plan.launch()
    bulk, emit = h.profile_read_steps()
    h.profile(False)
    plan.close()
    h.close()
    n_flags = sum(t.n for t in tiles if t.alive is not None)
    del tiles, prods, reset
    torch.cuda.empty_cache()
    return dict(wall=wall, device_s=float(step_ms.sum()) * 1e-3, step_ms=step_ms, counters=c,
                n_total=n_total, n_flags=n_flags, tuned=tuned, bulk_ms=float(np.mean(bulk)),
                emit_ms=float(np.mean(emit)))


def run_served(dev, jobs_per_client=16, steps=40):
    """Served form: 8 clients, Exp(2e6)-sized simulations (clamped to [1e4, 2e7]) arriving in a
    burst, beyond-LCFA leptons, MIXED, admission under a 12 GiB budget, 3 lanes."""
    import torch

    from paper_2301_07684_amd import serve

    warm = serve.Server(dev, hbm_budget=1 << 30, lanes=2)
    warm.add_jobs(serve.workload(clients=2, jobs_per_client=1, steps=3, mean=1e5, hi=2e5))
    warm.run()
    warm.close()
    srv = serve.Server(dev, hbm_budget=12 << 30, lanes=3)
    srv.add_jobs(serve.workload(clients=8, jobs_per_client=jobs_per_client, steps=steps,
                                think=0.002))
    res = srv.run(time_limit=300)
    srv.close()
    torch.cuda.empty_cache()
    return res


def constant_field_kernel_bytes(processed, emitted):
    """Streaming-kernel bytes of a uniform-field electron tile with the fused push (no alive
    array, optical depth): p and the optical depth read (32 B) for every particle; the pushed p
    and the new depth written (32 B) for every particle that does not emit."""
    return 32 * processed + 32 * (processed - emitted)


def run_constant_field(dev, n, warmup=2, launch=None):
    """The paper's constant-field set-up at scale: n electrons of 10 GeV at chi = 1 in a uniform
    magnetic field (one field value for the tile), 1.3 fs in 130 steps of 0.01 fs with the
    fused push and recoil, at the library's default launch shape (or `launch`), which the
    autotuner, run on the first 2^28 electrons, also picks.  Returns timings, counters and the
    photon count against N T R."""
    import torch

    from paper_2301_07684_amd import inputs, sfq

    seed = inputs.SEED_SYNC
    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT)
    K = int(round(inputs.T_SIM_FS / (inputs.DT_SECONDS * 1e15)))
    s = inputs.synchrotron_t(n, dev, seed=seed)
    g0 = inputs.GAMMA_10GEV
    W = float(h.rates(sfq.ELECTRON, torch.tensor([g0], dtype=torch.float64, device=dev),
                      torch.tensor([1.0], dtype=torch.float64, device=dev))[0])
    tau = h.init_optical_depth(s["uid"], seed=seed)
    tile = sfq.TileArrays(sfq.ELECTRON, s["p"][0], s["p"][1], s["p"][2], *s["E"], *s["B"],
                          tau=tau, uid=s["uid"], field_mode=sfq.FIELDS_UNIFORM)
    pb = sfq.ProductBuffers.empty(int(n * W * h.dt * 1.5) + 10000, 1, dev)
    cnt = sfq.Counters(dev)
    if launch is not None:
        h.set_launch(*launch)
    shape = list(h.get_launch())
    h.reserve(n, 1)
    for k in range(warmup):
        h.step([tile], seed=seed, step=k, products=pb, counters=cnt, push=True,
               zero_product_counts=True)
    # back to the initial state for the measured run
    torch.cuda.synchronize()
    s["p"][0].fill_(s["pm"])
    s["p"][1:].zero_()
    h.init_optical_depth(s["uid"], seed=seed, out=tau)
    cnt.reset()
    h.profile(True)   # the library's timing events, as in run_form
    h.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        h.step([tile], seed=seed, step=k, products=pb, counters=cnt, push=True,
               zero_product_counts=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bulk, emit = h.profile_read_steps(K)
    h.profile(False)
    if len(bulk) != K:
        raise RuntimeError("the step timing events did not cover every timed step")
    c = cnt.as_dict()
    if c["overflow"]:
        raise RuntimeError("product buffers overflowed during the constant-field run")
    h.close()
    del tile, s, tau, pb
    torch.cuda.empty_cache()
    return dict(wall=wall, K=K, n=n, counters=c, W=W, dt=inputs.DT,
                step_ms=(bulk + emit).astype(np.float64),
                bulk_ms=float(bulk.mean()), emit_ms=float(emit.mean()), shape=shape)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_sample=16384):
    """The oracle as it stands on a bounded sample of the FP64 workload (all host cores): the
    full step of every sampled particle (the workload's own emission mix), and, on the same
    sample, chi and the rate alone (a particle that does not emit) and, from the difference,
    the cost of each emitter's sampling, recoil and products."""
    from oracle import oracle as O
    from paper_2301_07684_amd import inputs

    O.build()
    rng_idx = np.random.default_rng(0).choice(1 << 24, n_sample // 2, replace=False)
    ws = [inputs.plane_wave(1 << 24, idx=rng_idx, species=sp) for sp in (O.ELECTRON, O.PHOTON)]
    t_rate = t_step = 0.0
    done = emitters = 0
    for species, w in zip((O.ELECTRON, O.PHOTON), ws):
        uid = w["uid"].view(np.uint64)
        tau0 = O.init_optical_depth(0, uid)
        t0 = time.perf_counter()
        g, c = O.chi(species, w["p"], w["E"], w["B"], inputs.LC_OVER_LR)
        O.rates(species, g, c, 1.0 / inputs.LC_OVER_LR)
        t1 = time.perf_counter()
        ref = O.step(species, w["p"], w["E"], w["B"], tau0, uid, dt=inputs.DT,
                     lc_over_lr=inputs.LC_OVER_LR, seed=0, step=1)
        t2 = time.perf_counter()
        t_rate += t1 - t0
        t_step += t2 - t1
        done += uid.size
        emitters += int(np.sum(ref["emitted"]))
    per_emitter = max(0.0, t_step - t_rate) / max(1, emitters)
    return dict(value=done / t_step, unit="particle-updates/s", cores=O.num_threads(),
                kind="oracle", cpu_model=cpu_model(),
                rate_only_updates_per_s=done / t_rate,
                seconds_per_emitter=per_emitter, emitters_in_sample=emitters,
                sample=f"{done} particles ({n_sample // 2} electrons + {n_sample // 2} photons, "
                       f"seeded random indices) of the FP64 plane-wave workload, one full step "
                       f"each ({t_step:.1f} s; chi and rate alone {t_rate:.1f} s)")


def measured_traffic():
    """HBM bytes per launch of the streaming kernel from the committed counter summary, or None
    when the kernels changed since the counters were taken."""
    from paper_2301_07684_amd import build

    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    get = lambda k: re.search(rf"^{k}:\s*(\S+)\s*$", txt, re.M)
    h, f, w = get("source_hash"), get("fetch_bytes_per_launch"), get("write_bytes_per_launch")
    if not (h and f and w) or h.group(1) != build.kernel_source_hash():
        return None
    return float(f.group(1)) + float(w.group(1))


def copy_calibration(dev, nbytes=1 << 31, reps=5):
    import torch

    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps + 1,
                      "GB_per_s": 2 * nbytes / dt / 1e9}), flush=True)


PROBE_SHAPES = ((2, 2), (3, 2), (4, 2), (2, 4))  # (blocks per CU, particles per lane)


def memory_probe(n=1 << 25, chunk=2048, repeats=12):
    """The practical ceiling of the streaming kernel's access pattern on this machine: the
    memory-only probe of csrc/mem_probe.hip (ten FP64 arrays of n read, one written back, 88 B
    per element, no arithmetic) at a few launch shapes; TB/s of read plus written bytes per
    shape, from the median of `repeats` launches, each after a cache-evicting copy."""
    import ctypes

    from paper_2301_07684_amd import build

    if not os.path.exists(build.PROBE_LIB):
        raise RuntimeError(f"{build.PROBE_LIB} is missing: run the build step first")
    lib = ctypes.CDLL(build.PROBE_LIB)
    fn = lib.sfq_probe_stream
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                   ctypes.POINTER(ctypes.c_float)]
    out = {}
    for bpc, ppl in PROBE_SHAPES:
        ms = ctypes.c_float(0.0)
        rc = fn(bpc, ppl, n, chunk, repeats, ctypes.byref(ms))
        if rc != 0:
            raise RuntimeError(f"memory probe failed with code {rc}")
        out[f"{bpc}x{chunk}, {ppl} per lane"] = 88.0 * n / (ms.value * 1e-3) / 1e12
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 24, help="particles per species")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-served-step", action="store_true",
                    help="skip the served form's kernels on one large step")
    ap.add_argument("--no-push", action="store_true")
    ap.add_argument("--no-constant-field", action="store_true")
    ap.add_argument("--no-wave", action="store_true")
    ap.add_argument("--no-mixed-same", action="store_true")
    ap.add_argument("--no-dial", action="store_true",
                    help="skip the truncated-table forms of the accuracy/speed dial")
    ap.add_argument("--constant-field-n", type=int, default=1 << 30,
                    help="electrons of the constant-field run")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-memory-probe", action="store_true",
                    help="skip the memory-only probe of the streaming kernel's access pattern")
    ap.add_argument("--launch", default=None,
                    help="fixed launch shape BLOCKS_PER_CUxCHUNK for the FP64 and MIXED forms "
                         "instead of the autotuner (e.g. for profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the QED step is independent per particle and the "
              "library runs it on a single MI355X; --gpus above 1 is not supported.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda", 0)
    if args.copy_calibration:
        copy_calibration(dev)
        return
    launch = tuple(int(v) for v in args.launch.split("x")) if args.launch else None
    f64 = run_form(0, "plane_wave", args.n, args.steps, args.warmup, dev, launch)
    print(f"# fp64 form done: {f64['wall'] / args.steps * 1e3:.3f} ms/step", file=sys.stderr,
          flush=True)
    # the memory-only reference right after the headline form, on the same machine state
    probe = None
    if not args.no_memory_probe:
        torch.cuda.empty_cache()
        try:
            probe = memory_probe()
        except (OSError, RuntimeError) as e:  # a reference figure: its failure spoils no other
            print(f"# memory probe failed: {e}", file=sys.stderr, flush=True)
    if probe is not None:
        print(f"# memory probe done: best {max(probe.values()):.2f} TB/s", file=sys.stderr,
              flush=True)
    mixed = None if args.no_mixed else run_form(1, "plane_wave_skewed", args.n, args.steps,
                                                args.warmup, dev, launch)
    if mixed is not None:
        print(f"# mixed form done: {mixed['wall'] / args.steps * 1e3:.3f} ms/step",
              file=sys.stderr, flush=True)
    mixed_same = None if args.no_mixed_same else run_form(1, "plane_wave", args.n, args.steps,
                                                          args.warmup, dev, launch)
    if mixed_same is not None:
        print(f"# mixed form on the headline workload done: "
              f"{mixed_same['wall'] / args.steps * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    batched = None if args.no_batched else run_batched(args.steps, args.warmup, dev)
    if batched is not None:
        print(f"# batched form done: {batched['wall'] / args.steps * 1e3:.3f} ms/step",
              file=sys.stderr, flush=True)
    served = None if args.no_served else run_served(dev)
    if served is not None:
        print(f"# served form done: {served['wall']:.2f} s", file=sys.stderr, flush=True)
    served_step = None if args.no_served_step else run_served_step(args.n, args.steps,
                                                                   args.warmup, dev, launch)
    if served_step is not None:
        print(f"# served form's kernels on one step done: "
              f"{served_step['wall'] / args.steps * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    # each form takes the launch shape the autotuner finds for it (or --launch): the
    # plane-wave-fields form, with more arithmetic per byte, runs best with more waves
    fused = None if args.no_push else run_form(0, "plane_wave", args.n, args.steps, args.warmup,
                                               dev, launch, push=True)
    if fused is not None:
        print(f"# fused push form done: {fused['wall'] / args.steps * 1e3:.3f} ms/step",
              file=sys.stderr, flush=True)
    wave = None if args.no_wave else run_form(0, "plane_wave", args.n, args.steps, args.warmup,
                                              dev, launch, wave=True)
    if wave is not None:
        print(f"# plane-wave fields form done: {wave['wall'] / args.steps * 1e3:.3f} ms/step",
              file=sys.stderr, flush=True)
    dial = {}
    if not args.no_dial:
        # the accuracy/speed dial's truncated forms on the headline workload
        for prec, name in ((0, "fp64_trunc"), (1, "mixed_trunc")):
            dial[name] = run_form(prec, "plane_wave", args.n, args.steps, args.warmup, dev,
                                  launch, approx=1)
            print(f"# {name} form done: {dial[name]['wall'] / args.steps * 1e3:.3f} ms/step",
                  file=sys.stderr, flush=True)
    const = None if args.no_constant_field else run_constant_field(dev, args.constant_field_n,
                                                                   launch=launch)
    if const is not None:
        print(f"# constant-field run done: {const['wall'] / const['K'] * 1e3:.3f} ms/step",
              file=sys.stderr, flush=True)

    c = f64["counters"]
    K = args.steps
    value = c["processed"] / f64["device_s"]
    per = lambda k: c[k] / K
    bulk_bytes = stream_kernel_bytes(f64["n_flags"], per("processed"), per("emitted"),
                                     per("converted"))
    emit_bytes = emit_kernel_bytes(per("emitted"), per("converted"))
    bulk_s, emit_s = f64["bulk_ms"] * 1e-3, f64["emit_ms"] * 1e-3
    achieved = bulk_bytes / bulk_s
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": f64["device_s"] / K * 1e3,
        "p50_step_ms": float(np.percentile(f64["step_ms"], 50)),
        "p99_step_ms": float(np.percentile(f64["step_ms"], 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "plane-wave FP64 plain form: 2^24 electrons + 2^24 photons, "
                               "Compton + Breit-Wheeler, optical depth, dt = 0.01 fs",
                   "particles_per_step": f64["n_total"], "precision": "fp64"},
        "emitted_per_step": per("emitted"),
        "converted_per_step": per("converted"),
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": measured_traffic(),
                     "kernel": "bulk_kernel<false, false, false, false, false> (the streaming "
                               "kernel alone; the whole step is step_roofline)",
                     "kernel_ms": f64["bulk_ms"], "algorithmic_bytes_per_launch": bulk_bytes},
        "emitter_pass": {"kernels": "emit_kernel<false, false, false> + "
                                    "defer_kernel (returns at once when nothing was deferred)",
                         "ms": f64["emit_ms"], "algorithmic_bytes_per_launch": emit_bytes,
                         "achieved_GB_per_s": emit_bytes / emit_s / 1e9},
        "launch_shape": f64["shape"],
        # the whole step (streaming kernel, emitter pass) against the HBM peak: with the
        # per-update yardstick (the headline figure), and with the kernels' own algorithmic
        # bytes (which leave out what this optical-depth form does not need, e.g. the uid of
        # non-emitters)
        "step_roofline": {"bytes_per_step": survey_step_bytes(per("processed"), per("emitted"),
                                                              per("converted")),
                          "frac": survey_step_bytes(per("processed"), per("emitted"),
                                                    per("converted"))
                                  / (f64["device_s"] / K) / HBM_PEAK,
                          "counting": "96 B per particle update + 80 B per emission + 104 B per "
                                      "conversion",
                          "kernel_algorithmic_bytes_per_step": bulk_bytes + emit_bytes,
                          "frac_kernel_algorithmic": (bulk_bytes + emit_bytes)
                                                     / (f64["device_s"] / K) / HBM_PEAK},
        "timing": "each step between the library's timing-only HIP events on the step's "
                  "stream (one before the streaming kernel, one after the step's last kernel); "
                  "before every timed step the particle state is put back by an untimed device "
                  "copy (and a 512 MiB copy evicts it from the caches), so each repeat steps the "
                  "same ensemble; the streaming/emitter split comes from 10 further steps timed "
                  "with a third event between the two",
        "wall_ms_per_step_incl_reset": f64["wall"] / K * 1e3,
        "emitter_queue_bytes": f64["queue_bytes"],
    }
    if mixed is not None:
        cm = mixed["counters"]
        pm = lambda k: cm[k] / K
        bb = stream_kernel_bytes(mixed["n_flags"], pm("processed"), pm("emitted"), pm("converted"))
        out["mixed"] = {"value": cm["processed"] / mixed["device_s"], "unit": "particle-updates/s",
                        "dtype": "f32 (f64 chi, optical depth and tails)",
                        "workload": "plane-wave skewed chi log-uniform [1e-4, 1e3], 2^24 + 2^24",
                        "ms_per_step": mixed["device_s"] / K * 1e3,
                        "p50_step_ms": float(np.percentile(mixed["step_ms"], 50)),
                        "p99_step_ms": float(np.percentile(mixed["step_ms"], 99)),
                        "bulk_kernel_ms": mixed["bulk_ms"], "emitter_pass_ms": mixed["emit_ms"],
                        "launch_shape": mixed["shape"],
                        "bulk_roofline_frac": bb / (mixed["bulk_ms"] * 1e-3) / HBM_PEAK,
                        "emitted_per_step": pm("emitted"),
                        "converted_per_step": pm("converted")}
    if mixed_same is not None:
        cs_ = mixed_same["counters"]
        ps_ = lambda k: cs_[k] / K
        bs_ = stream_kernel_bytes(mixed_same["n_flags"], ps_("processed"), ps_("emitted"),
                                  ps_("converted"))
        out["mixed_headline_workload"] = {
            "value": cs_["processed"] / mixed_same["device_s"], "unit": "particle-updates/s",
            "dtype": "f32 (f64 chi, optical depth and tails)",
            "workload": "the headline workload (plane wave, 2^24 + 2^24) in the MIXED form",
            "ms_per_step": mixed_same["device_s"] / K * 1e3,
            "p50_step_ms": float(np.percentile(mixed_same["step_ms"], 50)),
            "p99_step_ms": float(np.percentile(mixed_same["step_ms"], 99)),
            "bulk_kernel_ms": mixed_same["bulk_ms"], "emitter_pass_ms": mixed_same["emit_ms"],
            "bulk_roofline_frac": bs_ / (mixed_same["bulk_ms"] * 1e-3) / HBM_PEAK,
            "speedup_over_fp64": (cs_["processed"] / mixed_same["device_s"]) / value,
            "emitted_per_step": ps_("emitted"), "converted_per_step": ps_("converted")}
    if batched is not None:
        cb = batched["counters"]
        pb = lambda k: cb[k] / K
        sb = stream_kernel_bytes(batched["n_flags"], pb("processed"), pb("emitted"),
                                 pb("converted")) + emit_kernel_bytes(pb("emitted"),
                                                                      pb("converted"))
        out["batched"] = {"value": cb["processed"] / batched["device_s"], "unit": "particle-updates/s",
                          "dtype": "f32 (f64 chi, optical depth and tails)",
                          "workload": f"64 uneven tiles, {batched['n_total']} particles, "
                                      "e-/e+/photon, static B, chi log-uniform [1e-3, 1e2]",
                          "ms_per_step": batched["device_s"] / K * 1e3,
                          "p50_step_ms": float(np.percentile(batched["step_ms"], 50)),
                          "p99_step_ms": float(np.percentile(batched["step_ms"], 99)),
                          "launch_shape": batched["tuned"]["shape"],
                          "autotune_ms": batched["tuned"].get("timings"),
                          "step_roofline": {
                              "frac": survey_step_bytes(pb("processed"), pb("emitted"),
                                                        pb("converted"))
                                      / (float(np.mean(batched["step_ms"])) * 1e-3) / HBM_PEAK,
                              "frac_kernel_algorithmic":
                                  sb / (float(np.mean(batched["step_ms"])) * 1e-3) / HBM_PEAK},
                          "bulk_kernel_ms": batched["bulk_ms"],
                          "emitter_pass_ms": batched["emit_ms"],
                          "split_from": "plan launches with the library's timing events",
                          "emitted_per_step": pb("emitted"),
                          "converted_per_step": pb("converted")}
    if served is not None:
        cs = served["counters"]
        out["served"] = {"value": served["updates_per_s"], "unit": "particle-updates/s",
                         "dtype": "f32 (f64 chi, optical depth, tails and beyond-LCFA state)",
                         "workload": f"8 clients, {served['jobs']} simulations of Exp(2e6) "
                                     "particles (clamped [1e4, 2e7], half electrons with "
                                     "beyond-LCFA state, half photons), 40 steps each, burst "
                                     "arrivals, 12 GiB HBM budget, 3 lanes",
                         "p50_request_ms": served["p50_ms"], "p99_request_ms": served["p99_ms"],
                         "requests": served["requests"], "batches": served["batches"],
                         "mean_batch_requests": served["mean_batch"],
                         "admission_wait_p50_ms": served["admission_wait_p50_ms"],
                         "admission_wait_max_ms": served["admission_wait_max_ms"],
                         "jobs_that_waited_for_memory": served["waited"],
                         "wall_s": served["wall"], "emitted": cs["emitted"],
                         "blcfa_rejected": cs["blcfa_rejected"], "converted": cs["converted"]}
    if served_step is not None:
        cv = served_step["counters"]
        pv = lambda k: cv[k] / K
        vb = served_stream_kernel_bytes(served_step["n_leptons"], served_step["n_flags"],
                                        pv("processed") - served_step["n_leptons"])
        out["served_kernels_one_step"] = {
            "value": cv["processed"] / served_step["device_s"], "unit": "particle-updates/s",
            "dtype": "f32 (f64 chi, tails and beyond-LCFA state)",
            "workload": "the served form's kernels on one large step: 2^24 electrons with "
                        "beyond-LCFA state + 2^24 photons, plane-wave tiles, fused push, local "
                        "decisions",
            "ms_per_step": served_step["device_s"] / K * 1e3,
            "p50_step_ms": float(np.percentile(served_step["step_ms"], 50)),
            "p99_step_ms": float(np.percentile(served_step["step_ms"], 99)),
            "bulk_kernel_ms": served_step["bulk_ms"], "emitter_pass_ms": served_step["emit_ms"],
            "bulk_algorithmic_bytes": vb,
            "bulk_roofline_frac": vb / (served_step["bulk_ms"] * 1e-3) / HBM_PEAK,
            "launch_shape": served_step["shape"],
            "emitted_per_step": pv("emitted"), "blcfa_rejected_per_step": pv("blcfa_rejected"),
            "converted_per_step": pv("converted")}
    if fused is not None:
        cf = fused["counters"]
        pf = lambda k: cf[k] / K
        fb = pushed_stream_kernel_bytes(fused["n_flags"], pf("processed"), pf("emitted"),
                                        pf("converted"), fused["n_total"] // 2)
        out["fused_push"] = {"value": cf["processed"] / fused["device_s"],
                             "unit": "particle-updates/s", "dtype": "f64",
                             "workload": "the headline workload, electrons pushed (Boris) "
                                         "through their fields inside the streaming kernel",
                             "ms_per_step": fused["device_s"] / K * 1e3,
                             "p50_step_ms": float(np.percentile(fused["step_ms"], 50)),
                             "p99_step_ms": float(np.percentile(fused["step_ms"], 99)),
                             "bulk_kernel_ms": fused["bulk_ms"],
                             "emitter_pass_ms": fused["emit_ms"],
                             "bulk_algorithmic_bytes": fb,
                             "bulk_roofline_frac": fb / (fused["bulk_ms"] * 1e-3) / HBM_PEAK,
                             "launch_shape": fused["shape"],
                             "emitted_per_step": pf("emitted"),
                             "converted_per_step": pf("converted")}
    if wave is not None:
        cw = wave["counters"]
        pw = lambda k: cw[k] / K
        wb = wave_stream_kernel_bytes(wave["n_flags"], pw("processed"), pw("emitted"),
                                      pw("converted"))
        out["plane_wave_fields"] = {
            "value": cw["processed"] / wave["device_s"], "unit": "particle-updates/s", "dtype": "f64",
            "workload": "the headline workload with its fields given as the plane wave they come "
                        "from (per-particle amplitude and phase, E and B computed in the kernel)",
            "ms_per_step": wave["device_s"] / K * 1e3,
            "p50_step_ms": float(np.percentile(wave["step_ms"], 50)),
            "p99_step_ms": float(np.percentile(wave["step_ms"], 99)),
            "bulk_kernel_ms": wave["bulk_ms"], "emitter_pass_ms": wave["emit_ms"],
            "bulk_algorithmic_bytes": wb,
            "bulk_roofline_frac": wb / (wave["bulk_ms"] * 1e-3) / HBM_PEAK,
            "launch_shape": wave["shape"],
            "emitted_per_step": pw("emitted"), "converted_per_step": pw("converted")}
    if dial:
        from paper_2301_07684_amd import autotune

        errs = autotune.form_errors()
        out["dial"] = {"reported_error_bounds": {
            autotune.FORM_NAMES[k]: {"rate": v["rate"], "sample": v["sample"]}
            for k, v in errs.items()}, "forms": {}}
        for name, r in dial.items():
            cd = r["counters"]
            out["dial"]["forms"][name] = {
                "value": cd["processed"] / r["device_s"], "unit": "particle-updates/s",
                "workload": "the headline workload (plane wave, 2^24 + 2^24)",
                "ms_per_step": r["device_s"] / K * 1e3,
                "bulk_kernel_ms": r["bulk_ms"], "emitter_pass_ms": r["emit_ms"],
                "launch_shape": r["shape"], "speedup_over_fp64": (cd["processed"] / r["device_s"])
                                                                 / value}
    if const is not None:
        cc = const["counters"]
        kb = constant_field_kernel_bytes(cc["processed"] / const["K"], cc["emitted"] / const["K"])
        n_a = const["n"] * const["K"] * const["W"] * const["dt"]
        out["constant_field"] = {
            "value": cc["processed"] / const["wall"], "unit": "particle-updates/s",
            "dtype": "f64",
            "workload": f"{const['n']} electrons of 10 GeV at chi = 1 in a uniform magnetic field "
                        "(one value per tile), 1.3 fs = 130 steps, fused push, recoil",
            "ms_per_step": const["wall"] / const["K"] * 1e3,
            "p50_step_ms": float(np.percentile(const["step_ms"], 50)),
            "p99_step_ms": float(np.percentile(const["step_ms"], 99)),
            "bulk_kernel_ms": const["bulk_ms"], "emitter_pass_ms": const["emit_ms"],
            "launch_shape": const["shape"],
            "bulk_algorithmic_bytes": kb,
            "bulk_roofline_frac": kb / (const["bulk_ms"] * 1e-3) / HBM_PEAK,
            "photons": cc["emitted"], "N_T_R": n_a, "photons_over_N_T_R": cc["emitted"] / n_a}
    if probe is not None:
        best = max(probe.values())
        out["memory_probe"] = {
            "what": "the streaming kernel's bytes (ten FP64 arrays read, one written back) with no "
                    "arithmetic: the practical ceiling of its access pattern on this machine",
            "unit": "TB/s", "by_shape": probe, "best": best,
            "streaming_kernel_fraction_of_best": (out["roofline"]["traffic"] or bulk_bytes)
                                                 / bulk_s / 1e12 / best}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
