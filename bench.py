#!/usr/bin/env python3
"""Benchmark of the QED Monte Carlo step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Workload (the plain FP64 form at scale): 2^24 electrons + 2^24 photons counter-propagating
through a linearly polarised plane wave (a ~ U[10, 500], random phase, gamma log-uniform
[1e2, 1e5]), nonlinear Compton and Breit-Wheeler both active, optical-depth decisions,
dt = 0.01 fs, FP64 SoA arrays resident in HBM.  A step is one sfq_step over both tiles
(chi, rates, decisions, sampling, recoil, products).  The same is then timed in the MIXED form
on the skewed-chi ensemble (chi log-uniform [1e-4, 1e3]).

Prints ONE JSON line: value = FP64 particle-updates/s; p50/p99 step latency; the MIXED form's
numbers; the HBM roofline of the step kernel (algorithmic bytes / kernel time, measured with HIP
events on the launch stream); and the CPU oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-updates/sec (Compton+BW MC step) FP32 vs FP64; p99 step latency"
HBM_PEAK = 8.0e12  # B/s, MI355X HBM3E


def algorithmic_bytes(processed, emitted, converted):
    """Bytes a perfect implementation must move for one step.
    Per alive particle: read p, E, B (72), tau (8), uid (8), alive (1); write tau (8) = 97.
    Per Compton emission: write the emitter momentum (24) and a photon product
    (p 24, tau 8, uid 8, parent 8 = 48).  Per conversion: write alive (1) and two lepton
    products (96)."""
    return 97 * processed + (24 + 48) * emitted + (1 + 96) * converted


def build_state(dev, sfq, inputs, n, workload):
    import torch

    tiles, keep = [], []
    for species in (sfq.ELECTRON, sfq.PHOTON):
        if workload == "plane_wave":
            w = inputs.plane_wave(n, species=species)
        else:
            w = inputs.plane_wave(n, seed=inputs.SEED_SKEW, species=species, chi_range=(1e-4, 1e3))
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        arrs = dict(p=[t(w["p"][k]) for k in range(3)], E=[t(w["E"][k]) for k in range(3)],
                    B=[t(w["B"][k]) for k in range(3)], uid=t(w["uid"]))
        del w
        keep.append(arrs)
    return keep


def run_form(precision, workload, n, steps, warmup, dev):
    import torch

    from paper_2301_07684_amd import inputs, sfq

    h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=inputs.DT, precision=precision)
    state = build_state(dev, sfq, inputs, n, workload)
    tiles = []
    for species, a in zip((sfq.ELECTRON, sfq.PHOTON), state):
        tau = h.init_optical_depth(a["uid"], seed=0)
        alive = torch.ones(n, dtype=torch.uint8, device=dev)
        tiles.append(sfq.TileArrays(species, *a["p"], *a["E"], *a["B"], tau=tau, uid=a["uid"],
                                    alive=alive))
    prods = sfq.ProductBuffers.empty(n // 4, n // 16, dev)
    cnt = sfq.Counters(dev)
    stream = torch.cuda.current_stream()
    for s in range(warmup):
        prods.reset()
        h.step(tiles, seed=0, step=s + 1, products=prods, counters=cnt)
    torch.cuda.synchronize()
    cnt.reset()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        prods.reset()
        ev[s][0].record(stream)
        h.step(tiles, seed=0, step=warmup + s + 1, products=prods, counters=cnt)
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([a.elapsed_time(b) for a, b in ev])
    c = cnt.as_dict()
    if c["overflow"]:
        raise RuntimeError("product buffers overflowed during the benchmark")
    h.close()
    del tiles, state, prods
    torch.cuda.empty_cache()
    return dict(wall=wall, step_ms=step_ms, counters=c)


def cpu_baseline(n_sample=4096):
    """The oracle as it stands on a bounded sample of the FP64 workload (all host cores)."""
    from oracle import oracle as O
    from paper_2301_07684_amd import inputs

    O.build()
    rng_idx = np.random.default_rng(0).choice(1 << 24, n_sample // 2, replace=False)
    t0 = time.perf_counter()
    done = 0
    for species in (O.ELECTRON, O.PHOTON):
        w = inputs.plane_wave(1 << 24, idx=rng_idx, species=species)
        uid = w["uid"].view(np.uint64)
        tau0 = O.init_optical_depth(0, uid)
        O.step(species, w["p"], w["E"], w["B"], tau0, uid, dt=inputs.DT,
               lc_over_lr=inputs.LC_OVER_LR, seed=0, step=1)
        done += uid.size
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="particle-updates/s", cores=O.num_threads(), kind="oracle",
                sample=f"{done} particles ({n_sample // 2} electrons + {n_sample // 2} photons) of "
                       f"the FP64 plane-wave workload, one full step each, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 24, help="particles per species")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the QED step is independent per particle and this "
              "build runs on a single MI355X; --gpus above 1 is not supported.", file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda", 0)
    f64 = run_form(0, "plane_wave", args.n, args.steps, args.warmup, dev)
    mixed = None if args.no_mixed else run_form(1, "plane_wave_skewed", args.n, args.steps,
                                                args.warmup, dev)

    c = f64["counters"]
    updates = c["processed"]
    value = updates / f64["wall"]
    ms = f64["wall"] / args.steps * 1e3
    kern_s = float(np.mean(f64["step_ms"])) * 1e-3
    bytes_per_step = algorithmic_bytes(c["processed"], c["emitted"], c["converted"]) / args.steps
    achieved = bytes_per_step / kern_s
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "p50_step_ms": float(np.percentile(f64["step_ms"], 50)),
        "p99_step_ms": float(np.percentile(f64["step_ms"], 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "plane-wave FP64 plain form: 2^24 electrons + 2^24 photons, "
                               "Compton + Breit-Wheeler, optical depth, dt = 0.01 fs",
                   "particles_per_step": 2 * args.n, "precision": "fp64"},
        "emitted_per_step": c["emitted"] / args.steps,
        "converted_per_step": c["converted"] / args.steps,
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": None,
                     "kernel": "step_kernel<false>", "kernel_ms": kern_s * 1e3,
                     "algorithmic_bytes_per_launch": bytes_per_step},
    }
    if mixed is not None:
        cm = mixed["counters"]
        km = float(np.mean(mixed["step_ms"])) * 1e-3
        bm = algorithmic_bytes(cm["processed"], cm["emitted"], cm["converted"]) / args.steps
        out["mixed"] = {"value": cm["processed"] / mixed["wall"], "unit": "particle-updates/s",
                        "dtype": "f32 (f64 chi, optical depth and tails)",
                        "workload": "plane-wave skewed chi log-uniform [1e-4, 1e3], 2^24 + 2^24",
                        "ms_per_step": mixed["wall"] / args.steps * 1e3,
                        "p50_step_ms": float(np.percentile(mixed["step_ms"], 50)),
                        "p99_step_ms": float(np.percentile(mixed["step_ms"], 99)),
                        "roofline_frac": bm / km / HBM_PEAK,
                        "emitted_per_step": cm["emitted"] / args.steps,
                        "converted_per_step": cm["converted"] / args.steps}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
