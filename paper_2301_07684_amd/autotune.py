"""Launch-shape autotuner for the step kernels.

For a given set of tiles it times each candidate launch shape (blocks per compute unit x chunk
length, see sfq_set_launch) on the real data with a plan, keeps the fastest and caches the
choice in a JSON file keyed by the device, the precision and a coarse signature of the workload
(total particles and number of tiles rounded to powers of two, species mix).  The particle
state, the products already in the caller's buffers and the counters are snapshotted before
tuning and restored afterwards, so a tuned run gives the same results as an untuned one
(results never depend on the launch shape).
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Sequence, Tuple

import torch

from . import sfq

DEFAULT_CANDIDATES = [(2, 1024), (2, 2048), (2, 4096), (4, 2048), (4, 4096), (8, 1024), (8, 2048),
                      (16, 1024)]
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "autotune.json")

_STATE_FIELDS = ("px", "py", "pz", "tau", "alive", "fperp", "dfperp", "just_created")


def signature(handle: sfq.Handle, tiles: Sequence[sfq.TileArrays], push: bool = False) -> str:
    total = sum(t.n for t in tiles)
    species = sorted({int(t.species) for t in tiles})
    fields = sorted({int(t.field_mode) for t in tiles})
    props = torch.cuda.get_device_properties(handle.device)
    b = lambda v: 2 ** max(0, math.ceil(math.log2(max(v, 1))))
    return (f"{props.name}|cu{props.multi_processor_count}|prec{handle.precision}|"
            f"blcfa{int(handle.blcfa)}|n{b(total)}|t{b(len(tiles))}|s{'-'.join(map(str, species))}|"
            f"f{'-'.join(map(str, fields))}|push{int(push)}")


def _snapshot(tiles):
    return [{f: getattr(t, f).clone() for f in _STATE_FIELDS if getattr(t, f) is not None}
            for t in tiles]


def _restore(tiles, snap):
    for t, s in zip(tiles, snap):
        for f, v in s.items():
            getattr(t, f).copy_(v)


_PRODUCT_FIELDS = ("px", "py", "pz", "tau", "uid", "parent")
_PRODUCT_SPECIES = ("photons", "electrons", "positrons")


def _snapshot_products(products: sfq.ProductBuffers):
    """The products already in the buffers (the timed launches write theirs from slot 0)."""
    counts = products.host_counts()
    snap = []
    for k, name in enumerate(_PRODUCT_SPECIES):
        ps = getattr(products, name)
        m = min(counts[k], ps.capacity)
        snap.append({f: getattr(ps, f)[:m].clone() for f in _PRODUCT_FIELDS} if m > 0 else {})
    return products.counts.clone(), snap


def _restore_products(products: sfq.ProductBuffers, saved):
    counts, snap = saved
    for name, s in zip(_PRODUCT_SPECIES, snap):
        ps = getattr(products, name)
        for f, v in s.items():
            getattr(ps, f)[:v.numel()].copy_(v)
    products.counts.copy_(counts)


def load_cache(path: str = DEFAULT_CACHE) -> Dict[str, List[int]]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache, path: str = DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(handle: sfq.Handle, tiles: Sequence[sfq.TileArrays], products: sfq.ProductBuffers,
         counters: sfq.Counters, *, seed: int = 0, step: int = 1,
         candidates: Sequence[Tuple[int, int]] = DEFAULT_CANDIDATES, repeats: int = 4,
         cache_path: str | None = DEFAULT_CACHE, force: bool = False,
         push: bool = False) -> Dict:
    """Sets the fastest launch shape on `handle` and returns {'shape', 'ms', 'timings', ...}.
    Each candidate is timed on the step the caller will run: with `push`, the kernels that push
    the leptons inside the step."""
    key = signature(handle, tiles, push)
    cache = load_cache(cache_path) if cache_path else {}
    if not force and key in cache:
        bpc, chunk = cache[key]["shape"]
        handle.set_launch(bpc, chunk)
        return dict(cache[key], cached=True, key=key)
    snap = _snapshot(tiles)
    prod0 = _snapshot_products(products)
    cnt0 = counters.t.clone()
    timings = {}
    was_profiling = getattr(handle, "profiling", False)
    if was_profiling:
        handle.profile_read_steps()      # the caller's pending timings are not the candidates'
    handle.profile(True)                 # each launch timed by the library's timing-only events
    for bpc, chunk in candidates:
        handle.set_launch(bpc, chunk)
        plan = handle.plan(tiles, seed=seed, step=step, products=products, counters=counters,
                           push=push)
        plan.launch()
        torch.cuda.synchronize()
        handle.profile_read_steps()
        for k in range(repeats):
            plan.launch()
        a, b = handle.profile_read_steps()
        ms = sorted((a + b).tolist())    # per launch: streaming kernel to emitter pass end
        timings[f"{bpc}x{chunk}"] = ms[len(ms) // 2]
        plan.close()
        _restore(tiles, snap)
    handle.profile(was_profiling)
    best = min(timings, key=timings.get)
    bpc, chunk = (int(v) for v in best.split("x"))
    handle.set_launch(bpc, chunk)
    _restore_products(products, prod0)
    counters.t.copy_(cnt0)
    torch.cuda.synchronize()
    entry = {"shape": [bpc, chunk], "ms": timings[best], "timings": timings,
             "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
    if cache_path:
        cache[key] = entry
        save_cache(cache, cache_path)
    return dict(entry, cached=False, key=key)


# ------------------------------------------------------------------------------------------------
# Accuracy/speed dial
# ------------------------------------------------------------------------------------------------
FORM_NAMES = {(sfq.FP64, sfq.APPROX_FULL): "fp64", (sfq.FP64, sfq.APPROX_TRUNCATED): "fp64_trunc",
              (sfq.MIXED, sfq.APPROX_FULL): "mixed", (sfq.MIXED, sfq.APPROX_TRUNCATED): "mixed_trunc"}
# rounding of the kernels' own arithmetic after the table evaluation (products, powers, the
# energy fractions), per form: a few units in the last place of the evaluation precision
_FINAL_ULPS = {sfq.FP64: 8 * 2.0 ** -53, sfq.MIXED: 8 * 2.0 ** -24}


def tables_report_path() -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "sfq_tables_report.json")


def form_errors(report_path: str | None = None) -> Dict[Tuple[int, int], Dict[str, float]]:
    """Relative error bound of each arithmetic form (precision x table evaluation), from the
    table generator's measured report for the tables the library loads: twice the largest
    error it measured on its check points for the rates (against the quadrature of Eqs. (wtilde),
    (wtilde_pair)) and for the samples (against the exact inversion of Eqs. (again),
    (again_pp)), plus the rounding of the kernels' final arithmetic."""
    with open(report_path or tables_report_path()) as f:
        forms = json.load(f)["forms"]
    out = {}
    for (prec, approx), name in FORM_NAMES.items():
        m = forms[name]
        a = _FINAL_ULPS[prec]
        out[(prec, approx)] = {"rate": 2.0 * m["rate"] + a, "sample": 2.0 * m["sample"] + a,
                               # per process: photon emission by leptons, pair creation by photons
                               "emission_rate": 2.0 * m["photon_rate"] + a,
                               "pair_rate": 2.0 * m["pair_rate"] + a,
                               "measured_rate": m["rate"], "measured_sample": m["sample"],
                               "rate_terms": m["rate_terms"], "patch_terms": m["patch_terms"]}
    return out


# bw_fast (App. A function 7) is not a relative error: pair creation is dropped below chi = 0.3,
# where the pair rate is below 9.1e-6 alpha lambda_r / (lambda_C gamma) (Sec. 4.2).
BW_FAST_BOUND = "pair creation dropped for chi < 0.3, where W_pair < 9.1e-6 alpha lambda_r/(lambda_C gamma)"


def select_form(handle_kwargs: Dict, tiles: Sequence[sfq.TileArrays],
                products: sfq.ProductBuffers, counters: sfq.Counters, *, max_rel_error: float,
                allow_bw_fast: bool = False, seed: int = 0, step: int = 1,
                candidates: Sequence[Tuple[int, int]] = DEFAULT_CANDIDATES,
                repeats: int = 4, push: bool = False) -> Dict:
    """The accuracy/speed dial (the analogue of the paper's choice of coefficient counts, Sec. 4.5,
    and of its _fast pair functions, App. A functions 7 and 11): times every arithmetic form --
    FP64 or MIXED, with the full or the truncated tables -- whose measured error bound
    (form_errors) is within `max_rel_error`, each also with bw_fast when `allow_bw_fast`, each at
    its own best launch shape, on the caller's tiles, and returns the fastest as {'handle',
    'precision', 'approx', 'bw_fast', 'name', 'shape', 'ms', 'error_bound', 'timings'}.  The
    other handles are closed; the particle state, products and counters are restored.
    handle_kwargs are the sfq.Handle arguments other than precision, approx and bw_fast (units,
    dt, decision, blcfa, device); `push` times the steps with the leptons' push."""
    errors = form_errors()
    forms = [f for f in FORM_NAMES if max(errors[f]["rate"], errors[f]["sample"]) <= max_rel_error]
    if not forms:
        best = errors[(sfq.FP64, sfq.APPROX_FULL)]
        raise ValueError(f"no form meets a relative error of {max_rel_error:g} "
                         f"(FP64: {max(best['rate'], best['sample']):g})")
    fast = (False, True) if allow_bw_fast else (False,)
    snap = _snapshot(tiles)
    timings, best, handles = {}, None, []
    try:
        for prec, approx in forms:
            for bw in fast:
                h = sfq.Handle(**handle_kwargs, precision=prec, approx=approx, bw_fast=bw)
                handles.append(h)
                r = tune(h, tiles, products, counters, seed=seed, step=step,
                         candidates=candidates, repeats=repeats, cache_path=None, push=push)
                _restore(tiles, snap)
                name = FORM_NAMES[(prec, approx)] + ("+bw_fast" if bw else "")
                timings[name] = r["ms"]
                if best is None or r["ms"] < best["ms"]:
                    best = dict(handle=h, precision=prec, approx=approx, bw_fast=bw,
                                shape=r["shape"], ms=r["ms"], name=name)
    finally:
        for h in handles:
            if best is None or h is not best["handle"]:
                h.close()
    torch.cuda.synchronize()
    e = errors[(best["precision"], best["approx"])]
    bound = {"rate": e["rate"], "sample": e["sample"]}
    if best["bw_fast"]:
        bound["bw_fast"] = BW_FAST_BOUND
    best.update(error_bound=bound, timings=timings)
    return best
