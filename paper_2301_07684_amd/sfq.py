"""Python binding of the C ABI in include/sfq.h (argument marshalling only).

Every computation runs in the HIP library ``libsfq.so`` built from ``csrc/sfq.hip``; this
module only checks tensor shapes/dtypes/devices, passes ``tensor.data_ptr()`` and the current
HIP stream, and raises on a non-zero status.  There is no CPU fallback: if the library is
missing, ``load()`` raises.  PyTorch is used for device memory and streams only.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfq.so")

ELECTRON, POSITRON, PHOTON = 0, 1, 2
FP64, MIXED = 0, 1
OPTICAL_DEPTH, LOCAL = 0, 1
APPROX_FULL, APPROX_TRUNCATED = 0, 1
FIELDS_ARRAYS, FIELDS_UNIFORM, FIELDS_PLANE_WAVE = 0, 1, 2
P_INIT, P_EMIT, P_CHILD, P_CHILD2, P_LOCAL = 0, 1, 2, 3, 4
MAX_TILES = 4096

STATUS = {0: "SFQ_OK", 1: "SFQ_E_ARG", 2: "SFQ_E_STATE", 3: "SFQ_E_NOMEM", 4: "SFQ_E_CAPACITY",
          5: "SFQ_E_DEVICE", 6: "SFQ_E_TABLES"}

# every symbol declared in include/sfq.h
EXPORTS = ("sfq_create", "sfq_destroy", "sfq_last_error", "sfq_units", "sfq_chi", "sfq_rates",
           "sfq_sample_photon", "sfq_sample_pair", "sfq_philox", "sfq_init_optical_depth",
           "sfq_step", "sfq_step_noalloc", "sfq_set_launch", "sfq_get_launch", "sfq_plan_create",
           "sfq_plan_destroy",
           "sfq_plan_launch", "sfq_plan_set_step", "sfq_plan_capture", "sfq_plan_replay",
           "sfq_reserve", "sfq_set_queue", "sfq_queue_bytes", "sfq_profile_enable",
           "sfq_profile_read", "sfq_profile_read_steps")


class Config(C.Structure):
    _fields_ = [("ref_omega", C.c_double), ("ref_length", C.c_double), ("dt", C.c_double),
                ("precision", C.c_int32), ("decision", C.c_int32), ("blcfa", C.c_int32),
                ("bw_fast", C.c_int32), ("device", C.c_int32), ("approx", C.c_int32),
                ("tables_path", C.c_char_p)]


_P = C.c_void_p


class Tile(C.Structure):
    _fields_ = [("species", C.c_int32), ("product_set", C.c_int32), ("n", C.c_uint64),
                ("px", _P), ("py", _P), ("pz", _P), ("ex", _P), ("ey", _P), ("ez", _P),
                ("bx", _P), ("by", _P), ("bz", _P), ("tau", _P), ("uid", _P), ("alive", _P),
                ("px_prev", _P), ("py_prev", _P), ("pz_prev", _P), ("fperp", _P),
                ("dfperp", _P), ("just_created", _P), ("chi_out", _P), ("rate_out", _P),
                ("step_offset", C.c_uint64), ("field_mode", C.c_int32),
                ("reserved3", C.c_int32), ("wave_amp", _P), ("wave_phase", _P),
                ("wave_k", C.c_double * 3), ("wave_pol", C.c_double * 3),
                ("wave_phase0", C.c_double)]


class ProductsC(C.Structure):
    _fields_ = [("px", _P), ("py", _P), ("pz", _P), ("tau", _P), ("uid", _P), ("parent", _P),
                ("capacity", C.c_uint64)]


class ProductSetC(C.Structure):
    _fields_ = [("photons", ProductsC), ("electrons", ProductsC), ("positrons", ProductsC),
                ("product_counts", _P)]


class StepDesc(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("step", C.c_uint64), ("ntiles", C.c_int32),
                ("nsets", C.c_int32), ("tiles", C.POINTER(Tile)), ("photons", ProductsC),
                ("electrons", ProductsC), ("positrons", ProductsC), ("product_counts", _P),
                ("counters", _P), ("product_sets", C.POINTER(ProductSetC)),
                ("push", C.c_int32), ("zero_product_counts", C.c_int32)]


_TILE_POINTERS = tuple(nm for nm, _ in Tile._fields_[3:23])

COUNTER_NAMES = ("processed", "emitted", "converted", "blcfa_rejected", "out_of_domain",
                 "clamped", "overflow", "deferred")

_lib = None


def load(path: str = LIB_PATH):
    """Load libsfq.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run `python -m paper_2301_07684_amd.build`)")
    L = C.CDLL(path)
    st, vp, sz, dp, u64 = C.c_int, C.c_void_p, C.c_size_t, C.c_void_p, C.c_uint64
    L.sfq_create.restype = st
    L.sfq_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
    L.sfq_destroy.restype = None
    L.sfq_destroy.argtypes = [vp]
    L.sfq_last_error.restype = C.c_char_p
    L.sfq_last_error.argtypes = [vp]
    L.sfq_units.restype = st
    L.sfq_units.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.sfq_chi.restype = st
    L.sfq_chi.argtypes = [vp, C.c_int, sz] + [dp] * 11 + [vp]
    L.sfq_rates.restype = st
    L.sfq_rates.argtypes = [vp, C.c_int, sz, dp, dp, dp, vp]
    L.sfq_sample_photon.restype = st
    L.sfq_sample_photon.argtypes = [vp, sz, dp, dp, dp, dp, dp, vp]
    L.sfq_sample_pair.restype = st
    L.sfq_sample_pair.argtypes = [vp, sz, dp, dp, dp, dp, dp, vp]
    L.sfq_philox.restype = st
    L.sfq_philox.argtypes = [vp, sz, dp, u64, u64, C.c_uint32, dp, dp, vp]
    L.sfq_init_optical_depth.restype = st
    L.sfq_init_optical_depth.argtypes = [vp, sz, dp, u64, dp, vp]
    L.sfq_step.restype = st
    L.sfq_step.argtypes = [vp, C.POINTER(StepDesc), vp]
    L.sfq_step_noalloc.restype = st
    L.sfq_step_noalloc.argtypes = [vp, C.POINTER(StepDesc), vp]
    L.sfq_set_launch.restype = st
    L.sfq_set_launch.argtypes = [vp, C.c_int, C.c_int]
    L.sfq_get_launch.restype = st
    L.sfq_get_launch.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.sfq_plan_create.restype = st
    L.sfq_plan_create.argtypes = [vp, C.POINTER(StepDesc), C.c_int, C.POINTER(vp)]
    L.sfq_plan_destroy.restype = None
    L.sfq_plan_destroy.argtypes = [vp]
    L.sfq_plan_launch.restype = st
    L.sfq_plan_launch.argtypes = [vp, vp]
    L.sfq_plan_set_step.restype = st
    L.sfq_plan_set_step.argtypes = [vp, u64, vp]
    L.sfq_plan_capture.restype = st
    L.sfq_plan_capture.argtypes = [vp, C.c_int]
    L.sfq_plan_replay.restype = st
    L.sfq_plan_replay.argtypes = [vp, vp]
    L.sfq_reserve.restype = st
    L.sfq_reserve.argtypes = [vp, u64, C.c_int]
    L.sfq_set_queue.restype = st
    L.sfq_set_queue.argtypes = [vp, C.c_double, C.c_int]
    L.sfq_queue_bytes.restype = st
    L.sfq_queue_bytes.argtypes = [vp, C.POINTER(C.c_uint64)]
    L.sfq_profile_enable.restype = st
    L.sfq_profile_enable.argtypes = [vp, C.c_int]
    L.sfq_profile_read.restype = st
    L.sfq_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_uint64)]
    L.sfq_profile_read_steps.restype = st
    L.sfq_profile_read_steps.argtypes = [vp, C.c_uint64, C.POINTER(C.c_float),
                                         C.POINTER(C.c_float), C.POINTER(C.c_uint64)]
    _lib = L
    return L


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, dtype, n=None, name="array"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return t


class SFQError(RuntimeError):
    pass


class Handle:
    """An initialised library context (paper App. A functions 1/2 and 14)."""

    def __init__(self, *, ref_length: float | None = None, ref_omega: float | None = None,
                 dt: float, precision: int = FP64, decision: int = OPTICAL_DEPTH,
                 blcfa: bool = False, bw_fast: bool = False, device: int = 0,
                 tables_path: str | None = None, approx: int = APPROX_FULL):
        self._L = load()
        cfg = Config(ref_omega=ref_omega or 0.0, ref_length=ref_length or 0.0, dt=dt,
                     precision=precision, decision=decision, blcfa=int(blcfa),
                     bw_fast=int(bw_fast), device=device, approx=int(approx),
                     tables_path=None if tables_path is None else tables_path.encode())
        h = C.c_void_p()
        self._check(self._L.sfq_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self.profiling = False
        self.precision, self.decision, self.blcfa, self.bw_fast = precision, decision, blcfa, bw_fast
        self.approx = approx
        self.device = torch.device("cuda", device)
        lc, lr = C.c_double(), C.c_double()
        self._check(self._L.sfq_units(self._h, C.byref(lc), C.byref(lr)))
        self.lc_over_lr, self.lr_over_lc, self.dt = lc.value, lr.value, dt

    def _check(self, st):
        if st != 0:
            msg = self._L.sfq_last_error(None).decode()
            raise SFQError(f"{STATUS.get(st, st)}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            self._L.sfq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, blocks_per_cu: int, chunk: int):
        self._check(self._L.sfq_set_launch(self._h, blocks_per_cu, chunk))

    def get_launch(self):
        a, b = C.c_int(), C.c_int()
        self._check(self._L.sfq_get_launch(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def reserve(self, max_particles: int, max_tiles: int = 1):
        """Pre-size the emitter queue so steps within these limits allocate nothing."""
        self._check(self._L.sfq_reserve(self._h, max_particles, max_tiles))

    def set_queue(self, expected_fraction: float, adaptive: bool = True):
        """Emitter-queue sizing: the fraction of a step's particles expected to emit (slices hold
        twice that plus one share of a chunk), grown from observations when `adaptive`.  Shares
        that do not fit are stepped by a further kernel of the same step: same results."""
        self._check(self._L.sfq_set_queue(self._h, float(expected_fraction), int(bool(adaptive))))

    def queue_bytes(self) -> int:
        """Device bytes the emitter queue holds now."""
        v = C.c_uint64()
        self._check(self._L.sfq_queue_bytes(self._h, C.byref(v)))
        return v.value

    def profile(self, enable: bool = True, whole_step: bool = False):
        """Start/stop timing every step with HIP events: the streaming kernel and the emitter
        pass apart, or with `whole_step` the step as a whole (one event record fewer between
        the kernels; the emitter-pass times read as 0)."""
        mode = (2 if whole_step else 1) if enable else 0
        self._check(self._L.sfq_profile_enable(self._h, mode))
        self.profiling = bool(enable)

    def profile_read(self):
        """(stream-kernel ms, emitter-kernel ms, steps) summed since the previous read."""
        a, b, n = C.c_double(), C.c_double(), C.c_uint64()
        self._check(self._L.sfq_profile_read(self._h, C.byref(a), C.byref(b), C.byref(n)))
        return a.value, b.value, n.value

    def profile_read_steps(self, max_steps: int = 100000):
        """Per-step (stream-kernel ms, emitter-pass ms) arrays of the steps timed since the
        previous read (numpy float32, in launch order)."""
        a = np.zeros(max_steps, dtype=np.float32)
        b = np.zeros(max_steps, dtype=np.float32)
        n = C.c_uint64()
        fp = C.POINTER(C.c_float)
        self._check(self._L.sfq_profile_read_steps(self._h, max_steps, a.ctypes.data_as(fp),
                                                   b.ctypes.data_as(fp), C.byref(n)))
        return a[:n.value].copy(), b[:n.value].copy()

    # ---- batched calls ------------------------------------------------------------------------
    def chi(self, species, p, E, B, stream=None):
        """p, E, B: sequences of three float64 device tensors.  Returns (gamma, chi)."""
        n = p[0].numel()
        arrs = [_dev(a, torch.float64, n, "p/E/B") for a in (*p, *E, *B)]
        gamma = torch.empty(n, dtype=torch.float64, device=arrs[0].device)
        chi = torch.empty_like(gamma)
        self._check(self._L.sfq_chi(self._h, species, n, *[_ptr(a) for a in arrs], _ptr(gamma),
                                    _ptr(chi), _stream(stream)))
        return gamma, chi

    def rates(self, species, gamma, chi, out=None, stream=None):
        n = gamma.numel()
        _dev(gamma, torch.float64, n, "gamma")
        _dev(chi, torch.float64, n, "chi")
        out = torch.empty_like(gamma) if out is None else _dev(out, torch.float64, n, "out")
        self._check(self._L.sfq_rates(self._h, species, n, _ptr(gamma), _ptr(chi), _ptr(out),
                                      _stream(stream)))
        return out

    def sample_photon(self, gamma, chi, r, stream=None):
        n = gamma.numel()
        for nm, a in (("gamma", gamma), ("chi", chi), ("r", r)):
            _dev(a, torch.float64, n, nm)
        gph, gem = torch.empty_like(gamma), torch.empty_like(gamma)
        self._check(self._L.sfq_sample_photon(self._h, n, _ptr(gamma), _ptr(chi), _ptr(r),
                                              _ptr(gph), _ptr(gem), _stream(stream)))
        return gph, gem

    def sample_pair(self, gamma, chi, r, stream=None):
        n = gamma.numel()
        for nm, a in (("gamma", gamma), ("chi", chi), ("r", r)):
            _dev(a, torch.float64, n, nm)
        ge, gp = torch.empty_like(gamma), torch.empty_like(gamma)
        self._check(self._L.sfq_sample_pair(self._h, n, _ptr(gamma), _ptr(chi), _ptr(r),
                                            _ptr(ge), _ptr(gp), _stream(stream)))
        return ge, gp

    def philox(self, uid, seed, step, purpose, stream=None):
        """uid: int64 device tensor (bit pattern of the uint64 ids).  Returns (a, b) int64."""
        n = uid.numel()
        _dev(uid, torch.int64, n, "uid")
        a, b = torch.empty_like(uid), torch.empty_like(uid)
        self._check(self._L.sfq_philox(self._h, n, _ptr(uid), seed, step, purpose, _ptr(a),
                                       _ptr(b), _stream(stream)))
        return a, b

    def init_optical_depth(self, uid, seed, out=None, stream=None):
        n = uid.numel()
        _dev(uid, torch.int64, n, "uid")
        out = torch.empty(n, dtype=torch.float64, device=uid.device) if out is None else out
        self._check(self._L.sfq_init_optical_depth(self._h, n, _ptr(uid), seed, _ptr(out),
                                                   _stream(stream)))
        return out

    @staticmethod
    def _desc(tiles, seed, step, products, counters, product_sets=None, push=False,
              zero_product_counts=False):
        """Step descriptor.  With `product_sets` (a list of ProductBuffers), tile k's products go
        to product_sets[tiles[k].product_set] and `products` may be None.  push=True gives every
        alive lepton the Boris push through its tile's fields before the step."""
        nt = len(tiles)
        if nt == 0 or nt > MAX_TILES:
            raise ValueError("1 <= len(tiles) <= MAX_TILES")
        arr = (Tile * nt)()
        for k, t in enumerate(tiles):
            arr[k] = t.to_c()
        if product_sets:
            sets = (ProductSetC * len(product_sets))()
            for k, pb in enumerate(product_sets):
                sets[k] = ProductSetC(photons=pb.photons.to_c(), electrons=pb.electrons.to_c(),
                                      positrons=pb.positrons.to_c(), product_counts=_ptr(pb.counts))
            nsets = len(product_sets)
        else:
            if products is None:
                raise ValueError("products or product_sets is required")
            sets, nsets = None, 0
            for t in tiles:
                if t.product_set != 0:
                    raise ValueError("product_set indices need product_sets")
        none = ProductsC()
        desc = StepDesc(seed=seed, step=step, ntiles=nt, nsets=nsets, tiles=arr,
                        photons=products.photons.to_c() if products else none,
                        electrons=products.electrons.to_c() if products else none,
                        positrons=products.positrons.to_c() if products else none,
                        product_counts=_ptr(products.counts) if products else None,
                        counters=_ptr(counters.t), product_sets=sets, push=int(bool(push)),
                        zero_product_counts=int(bool(zero_product_counts)))
        return desc, (arr, sets)

    def step(self, tiles: Sequence["TileArrays"], *, seed: int, step: int,
             products: Optional["ProductBuffers"] = None, counters: "Counters",
             product_sets: Optional[Sequence["ProductBuffers"]] = None, push: bool = False,
             zero_product_counts: bool = False, stream=None):
        """One Monte Carlo step over all tiles (one launch sequence on `stream`); with
        push=True the leptons' momenta are first pushed through their fields (fused); with
        zero_product_counts=True the product buffers receive this step's products only."""
        desc, _keep = self._desc(tiles, seed, step, products, counters, product_sets, push,
                                 zero_product_counts)
        self._check(self._L.sfq_step(self._h, C.byref(desc), _stream(stream)))

    def step_noalloc(self, tiles: Sequence["TileArrays"], *, seed: int, step: int,
                     products: Optional["ProductBuffers"] = None, counters: "Counters",
                     product_sets: Optional[Sequence["ProductBuffers"]] = None,
                     push: bool = False, zero_product_counts: bool = False, stream=None):
        """step() through sfq_step_noalloc: no allocation in the call (its scratch is the
        library's static device array); calls that overlap on one device race."""
        desc, _keep = self._desc(tiles, seed, step, products, counters, product_sets, push,
                                 zero_product_counts)
        self._check(self._L.sfq_step_noalloc(self._h, C.byref(desc), _stream(stream)))

    def plan(self, tiles, *, seed: int, step: int, products: Optional["ProductBuffers"] = None,
             counters: "Counters", zero_product_counts: bool = True,
             product_sets: Optional[Sequence["ProductBuffers"]] = None,
             push: bool = False) -> "Plan":
        return Plan(self, tiles, seed=seed, step=step, products=products, counters=counters,
                    zero_product_counts=zero_product_counts, product_sets=product_sets,
                    push=push)


class Plan:
    """A fixed set of tiles stepped repeatedly (sfq_plan_*): kernels only per launch, the step
    index advancing on the device, optionally captured in a HIP graph."""

    def __init__(self, handle: Handle, tiles, *, seed, step, products, counters,
                 zero_product_counts=True, product_sets=None, push=False):
        self._handle = handle
        self._L = handle._L
        self.tiles, self.products, self.counters = list(tiles), products, counters
        self.product_sets = list(product_sets) if product_sets else None
        desc, _keep = Handle._desc(self.tiles, seed, step, products, counters, product_sets,
                                   push)
        p = C.c_void_p()
        handle._check(self._L.sfq_plan_create(handle._h, C.byref(desc), int(zero_product_counts),
                                              C.byref(p)))
        self._p = p

    def launch(self, stream=None):
        self._handle._check(self._L.sfq_plan_launch(self._p, _stream(stream)))

    def set_step(self, step, stream=None):
        self._handle._check(self._L.sfq_plan_set_step(self._p, step, _stream(stream)))

    def capture(self, steps: int):
        self._handle._check(self._L.sfq_plan_capture(self._p, steps))

    def replay(self, stream=None):
        self._handle._check(self._L.sfq_plan_replay(self._p, _stream(stream)))

    def close(self):
        if getattr(self, "_p", None):
            self._L.sfq_plan_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class TileArrays:
    """Device SoA arrays of one tile (see sfq_tile in include/sfq.h)."""
    species: int
    px: torch.Tensor
    py: torch.Tensor
    pz: torch.Tensor
    ex: Optional[torch.Tensor] = None
    ey: Optional[torch.Tensor] = None
    ez: Optional[torch.Tensor] = None
    bx: Optional[torch.Tensor] = None
    by: Optional[torch.Tensor] = None
    bz: Optional[torch.Tensor] = None
    tau: Optional[torch.Tensor] = None
    uid: Optional[torch.Tensor] = None
    alive: Optional[torch.Tensor] = None
    px_prev: Optional[torch.Tensor] = None
    py_prev: Optional[torch.Tensor] = None
    pz_prev: Optional[torch.Tensor] = None
    fperp: Optional[torch.Tensor] = None
    dfperp: Optional[torch.Tensor] = None
    just_created: Optional[torch.Tensor] = None
    chi_out: Optional[torch.Tensor] = None
    rate_out: Optional[torch.Tensor] = None
    product_set: int = 0
    step_offset: int = 0
    # how the fields are given: FIELDS_ARRAYS (ex..bz of n), FIELDS_UNIFORM (ex..bz of one
    # value each), FIELDS_PLANE_WAVE (E = wave_amp cos(wave_phase + wave_phase0) wave_pol,
    # B = wave_k x E, computed in the step)
    field_mode: int = FIELDS_ARRAYS
    wave_amp: Optional[torch.Tensor] = None
    wave_phase: Optional[torch.Tensor] = None
    wave_k: Sequence[float] = (1.0, 0.0, 0.0)
    wave_pol: Sequence[float] = (0.0, 1.0, 0.0)
    wave_phase0: float = 0.0

    def __post_init__(self):
        n = self.px.numel()
        f64 = ("px", "py", "pz", "ex", "ey", "ez", "bx", "by", "bz", "tau", "px_prev", "py_prev",
               "pz_prev", "chi_out", "rate_out", "wave_amp", "wave_phase")
        fields = ("ex", "ey", "ez", "bx", "by", "bz")
        uniform = self.field_mode == FIELDS_UNIFORM
        for nm in f64:
            a = getattr(self, nm)
            if a is not None:
                _dev(a, torch.float64, 1 if (uniform and nm in fields) else n, nm)
        for nm in ("fperp", "dfperp"):
            a = getattr(self, nm)
            if a is not None:
                _dev(a, torch.float64, 3 * n, nm)
        if self.uid is not None:
            _dev(self.uid, torch.int64, n, "uid")
        for nm in ("alive", "just_created"):
            a = getattr(self, nm)
            if a is not None:
                _dev(a, torch.uint8, n, nm)

    @property
    def n(self):
        return self.px.numel()

    def to_c(self) -> Tile:
        ptrs = [None if a is None else a.data_ptr() for a in
                (getattr(self, nm) for nm in _TILE_POINTERS)]
        wa, wp = self.wave_amp, self.wave_phase
        return Tile(self.species, self.product_set, self.n, *ptrs, self.step_offset,
                    int(self.field_mode), 0, None if wa is None else wa.data_ptr(),
                    None if wp is None else wp.data_ptr(), (C.c_double * 3)(*self.wave_k),
                    (C.c_double * 3)(*self.wave_pol), float(self.wave_phase0))


@dataclass
class ProductSpecies:
    px: torch.Tensor
    py: torch.Tensor
    pz: torch.Tensor
    tau: torch.Tensor
    uid: torch.Tensor
    parent: torch.Tensor

    @staticmethod
    def empty(capacity: int, device) -> "ProductSpecies":
        f = lambda: torch.empty(max(capacity, 1), dtype=torch.float64, device=device)
        i = lambda: torch.empty(max(capacity, 1), dtype=torch.int64, device=device)
        return ProductSpecies(f(), f(), f(), f(), i(), i())

    @property
    def capacity(self):
        return self.px.numel()

    def to_c(self) -> ProductsC:
        return ProductsC(px=_ptr(self.px), py=_ptr(self.py), pz=_ptr(self.pz), tau=_ptr(self.tau),
                         uid=_ptr(self.uid), parent=_ptr(self.parent), capacity=self.capacity)


@dataclass
class ProductBuffers:
    photons: ProductSpecies
    electrons: ProductSpecies
    positrons: ProductSpecies
    counts: torch.Tensor = field(default=None)

    @staticmethod
    def empty(capacity_photons: int, capacity_pairs: int, device) -> "ProductBuffers":
        pb = ProductBuffers(ProductSpecies.empty(capacity_photons, device),
                            ProductSpecies.empty(capacity_pairs, device),
                            ProductSpecies.empty(capacity_pairs, device))
        pb.counts = torch.zeros(3, dtype=torch.int64, device=device)
        return pb

    def reset(self):
        self.counts.zero_()

    def host_counts(self):
        return [int(v) for v in self.counts.cpu()]


class Counters:
    def __init__(self, device):
        self.t = torch.zeros(8, dtype=torch.int64, device=device)

    def reset(self):
        self.t.zero_()

    def as_dict(self):
        v = self.t.cpu().tolist()
        return dict(zip(COUNTER_NAMES, v))

    def results(self):
        """The counters that describe the step's results: all but `deferred`, which depends on
        how the work was scheduled (the size of the emitter queue), not on the results."""
        return {k: v for k, v in self.as_dict().items() if k != "deferred"}
