"""Served form of the QED step on one GPU: continuous batching of step requests.

Several client simulations (PIC codes, each with its own resident particles) ask for one QED
step per tick of their own time loop.  The server

* admits a simulation when its device footprint (particle state, beyond-LCFA state and product
  buffers) fits the HBM budget.  Admission is first-come first-served, so a large simulation is
  not overtaken forever by small ones;
* batches every step request that is ready into one ``sfq_step`` call on a free lane.  A lane is
  a HIP stream with its own library handle and emitter queue, reserved once and charged to the
  HBM budget.  Each simulation's
  tiles carry their own Philox step offset and product set, so its results do not depend on
  what it was batched with (draws depend only on seed, uid, step and purpose);
* keeps one batch in flight per lane, so requests that become ready while others run on the GPU
  are dispatched as soon as a lane frees up, and their work overlaps on the device;
* records each request's latency, from submission until its results are ready (the batch's
  completion event observed), plus throughput and admission waits.

The clients are a test harness, not part of the library.  Each simulation holds electrons with
beyond-LCFA state (paper Sec. 5) and photons in a linearly polarised plane wave travelling along
+x, E = a cos(phi + 2 t) y, B = E_y z (each particle's amplitude a and phase phi; the phase
advances by 2 dt per step for particles meeting the wave head-on).  The step computes those
fields itself (plane-wave tiles) and pushes the electrons (Boris) before the QED step, which
supplies p^{(n-1/2)} and p^{(n+1/2)} to the beyond-LCFA force update: a client's tick enqueues
no GPU work of its own.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

from . import inputs, sfq


# Device bytes per particle of a simulation (the footprint admission charges)
LEPTON_BYTES = 8 * 3 * 3 + 8 + 1 + 8 + 8  # p, F_perp, dF; uid; just_created; wave a, phi
PHOTON_BYTES = 8 * 3 + 8 + 1 + 8 + 8       # p; uid; alive; wave a, phi
PRODUCT_BYTES = 6 * 8                      # p, tau, uid, parent
# launch shape of the lanes' steps (blocks per compute unit, particles per chunk): the best of
# 8 x 2048, 3 x 4096, 4 x 2048 and 3 x 2048 on the served workload (batches of about 24M
# particles in beyond-LCFA kernels of 3 waves per SIMD), by a few percent
LANE_LAUNCH = (4, 2048)
# expected emitter fraction the lanes' emitter queues are sized for (fixed, so that their memory
# is known when admitting; a batch with more emitters is still stepped exactly, more slowly)
LANE_QUEUE_FRACTION = 1.0 / 16.0


@dataclass
class JobSpec:
    """One client simulation: its particle counts, number of steps and arrival time (s)."""
    job_id: int
    n_leptons: int
    n_photons: int
    steps: int
    arrival: float = 0.0
    client: int = 0

    @property
    def seed(self) -> int:
        # inputs seeds: electrons use seed, photons seed + 2 (distinct uids per job)
        return inputs.SEED_SERVE * 10000 + 4 * self.job_id

    @property
    def photon_capacity(self) -> int:
        return max(256, self.n_leptons // 4)

    @property
    def pair_capacity(self) -> int:
        return max(256, self.n_photons // 8)

    @property
    def footprint(self) -> int:
        return (self.n_leptons * LEPTON_BYTES + self.n_photons * PHOTON_BYTES
                + PRODUCT_BYTES * (self.photon_capacity + 2 * self.pair_capacity) + 4096)


# ------------------------------------------------------------------------------------------------
# Host-side scheduling (no GPU): admission by budget and batch formation
# ------------------------------------------------------------------------------------------------
class Scheduler:
    """Admission (FIFO under an HBM budget) and batch formation (FIFO under size limits)."""

    def __init__(self, budget: int, max_batch_particles: int, max_batch_tiles: int):
        self.budget, self.used = budget, 0
        self.max_batch_particles, self.max_batch_tiles = max_batch_particles, max_batch_tiles
        self.waiting: Deque[JobSpec] = collections.deque()
        self.ready: Deque[object] = collections.deque()
        self.deferred = set()  # jobs that had to wait for memory at least once
        self._unmarked = 0     # jobs at the end of `waiting` not yet in `deferred`

    def arrive(self, spec: JobSpec):
        if spec.footprint > self.budget:
            raise ValueError(f"job {spec.job_id} needs {spec.footprint} B, more than the whole "
                             f"HBM budget of {self.budget} B")
        self.waiting.append(spec)
        self._unmarked += 1

    def admit(self) -> List[JobSpec]:
        """Jobs admitted now, in arrival order; stops at the first that does not fit."""
        out = []
        while self.waiting and self.used + self.waiting[0].footprint <= self.budget:
            spec = self.waiting.popleft()
            self.used += spec.footprint
            out.append(spec)
        # the jobs left waiting had to wait for memory; only the latest arrivals are new
        k = min(self._unmarked, len(self.waiting))
        for i in range(len(self.waiting) - k, len(self.waiting)):
            self.deferred.add(self.waiting[i].job_id)
        self._unmarked = 0
        return out

    def release(self, spec: JobSpec):
        self.used -= spec.footprint
        assert self.used >= 0

    def submit(self, request):
        self.ready.append(request)

    def next_batch(self, particles: Callable[[object], int],
                   tiles: Callable[[object], int]) -> list:
        """Ready requests in FIFO order up to the batch limits (at least one if any)."""
        batch, n, t = [], 0, 0
        while self.ready:
            r = self.ready[0]
            pn, pt = particles(r), tiles(r)
            if batch and (n + pn > self.max_batch_particles or t + pt > self.max_batch_tiles):
                break
            batch.append(self.ready.popleft())
            n, t = n + pn, t + pt
        return batch


def percentile(values: Sequence[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    if not values:
        return float("nan")
    v = sorted(values)
    k = max(0, min(len(v) - 1, math.ceil(q / 100.0 * len(v)) - 1))
    return v[k]


# ------------------------------------------------------------------------------------------------
# Device side
# ------------------------------------------------------------------------------------------------
class Simulation:
    """Device-resident state of one client simulation (created at admission)."""

    def __init__(self, spec: JobSpec, dev, stream):
        import torch

        self.spec, self.dev, self.stream = spec, dev, stream
        self.step = 0                 # steps done = the Philox step offset of the next one
        self.in_flight = False
        self.last_batch = 0           # requests in the batch of the last step
        self._tiles = None
        with torch.cuda.stream(stream):
            e = inputs.plane_wave_t(spec.n_leptons, dev, seed=spec.seed, species=sfq.ELECTRON)
            self.p = e["p"].contiguous()
            self.a, self.phi = e["a"], e["phi"]
            self.e_uid = e["uid"]
            self.fperp = torch.zeros(3 * spec.n_leptons, dtype=torch.float64, device=dev)
            self.dfperp = torch.zeros_like(self.fperp)
            self.just_created = torch.ones(spec.n_leptons, dtype=torch.uint8, device=dev)
            g = inputs.plane_wave_t(spec.n_photons, dev, seed=spec.seed, species=sfq.PHOTON)
            self.k = g["p"].contiguous()
            self.ka, self.kphi = g["a"], g["phi"]
            self.g_uid = g["uid"]
            self.alive = torch.ones(spec.n_photons, dtype=torch.uint8, device=dev)
            self.products = sfq.ProductBuffers.empty(spec.photon_capacity, spec.pair_capacity, dev)
            del e, g
        # the set-up ran on the client's stream: the first step waits for it
        self.ready_event = torch.cuda.Event()
        self.ready_event.record(stream)

    def wave_phase0(self, dt: float) -> float:
        """The phase the wave has advanced by at the current step (2 dt per step)."""
        return 2.0 * dt * self.step

    def tiles(self, product_set: int, dt: float) -> List[sfq.TileArrays]:
        """The simulation's tiles for a batched step (built once; the product set, the Philox
        step offset and the wave's phase change per step).  Both species are plane-wave tiles:
        the step computes their fields and pushes the electrons."""
        if self._tiles is None:
            wave = dict(field_mode=sfq.FIELDS_PLANE_WAVE, wave_k=(1.0, 0.0, 0.0),
                        wave_pol=(0.0, 1.0, 0.0))
            lep = sfq.TileArrays(sfq.ELECTRON, self.p[0], self.p[1], self.p[2], uid=self.e_uid,
                                 fperp=self.fperp, dfperp=self.dfperp,
                                 just_created=self.just_created, wave_amp=self.a,
                                 wave_phase=self.phi, **wave)
            pho = sfq.TileArrays(sfq.PHOTON, self.k[0], self.k[1], self.k[2], uid=self.g_uid,
                                 alive=self.alive, wave_amp=self.ka, wave_phase=self.kphi, **wave)
            self._tiles = [t for t in (lep, pho) if t.n > 0]
        for t in self._tiles:
            t.product_set = product_set
            t.step_offset = self.step
            t.wave_phase0 = self.wave_phase0(dt)
        return self._tiles

    @property
    def particles(self) -> int:
        return self.spec.n_leptons + self.spec.n_photons


@dataclass
class Request:
    sim: Simulation
    t_submit: float
    t_dispatch: float = 0.0


@dataclass
class Lane:
    handle: object
    stream: object
    counters: object
    event: object = None
    batch: list = field(default_factory=list)


class Server:
    """Continuous-batching server of QED steps on one GPU (see the module docstring)."""

    def __init__(self, dev=None, *, hbm_budget: int = 3 << 30, lanes: int = 2,
                 precision: int = sfq.MIXED, seed: int = 0, max_batch_particles: int = 1 << 25,
                 max_batch_tiles: int = 256, clients: int = 8,
                 on_step: Optional[Callable[[Simulation], None]] = None,
                 launch: Tuple[int, int] = LANE_LAUNCH):
        import torch

        self.dev = dev or torch.device("cuda", 0)
        self.seed, self.on_step = seed, on_step
        self.dt = inputs.DT
        self.lanes: List[Lane] = []
        for _ in range(lanes):
            h = sfq.Handle(ref_length=inputs.LAMBDA_R, dt=self.dt, precision=precision,
                           decision=sfq.LOCAL, blcfa=True, device=self.dev.index or 0)
            h.set_launch(*launch)
            h.set_queue(LANE_QUEUE_FRACTION, adaptive=False)
            h.reserve(max_batch_particles, max_batch_tiles)
            self.lanes.append(Lane(h, torch.cuda.Stream(device=self.dev), sfq.Counters(self.dev)))
        # the lanes' emitter queues are charged to the budget before any simulation
        self.queue_bytes = sum(lane.handle.queue_bytes() for lane in self.lanes)
        if self.queue_bytes >= hbm_budget:
            raise ValueError(f"the lanes' emitter queues ({self.queue_bytes} B) do not fit the "
                             f"HBM budget of {hbm_budget} B")
        self.sched = Scheduler(hbm_budget - self.queue_bytes, max_batch_particles,
                               max_batch_tiles)
        self.client_streams = [torch.cuda.Stream(device=self.dev) for _ in range(clients)]
        self.pending: List[JobSpec] = []
        self.active: Dict[int, Simulation] = {}
        self.latencies: List[float] = []
        self.admission_waits: List[float] = []
        self.batch_sizes: List[int] = []
        self.done_jobs = 0
        self.t0 = None

    # ---- client arrivals -----------------------------------------------------------------------
    def add_jobs(self, specs: Sequence[JobSpec]):
        self.pending.extend(sorted(specs, key=lambda s: s.arrival))

    def _now(self):
        return time.perf_counter() - self.t0

    def _arrivals(self, now):
        while self.pending and self.pending[0].arrival <= now:
            self.sched.arrive(self.pending.pop(0))

    def _admit(self, now):
        for spec in self.sched.admit():
            self.admission_waits.append(max(0.0, now - spec.arrival))
            stream = self.client_streams[spec.client % len(self.client_streams)]
            self.active[spec.job_id] = Simulation(spec, self.dev, stream)

    def _clients(self):
        # a client's tick: the next step request (its fields and push are part of the step)
        for sim in self.active.values():
            if not sim.in_flight and sim.step < sim.spec.steps:
                sim.in_flight = True
                self.sched.submit(Request(sim, self._now()))

    def _dispatch(self):
        for lane in self.lanes:
            if lane.batch or not self.sched.ready:
                continue
            batch = self.sched.next_batch(lambda r: r.sim.particles, lambda r: 2)
            tiles, sets = [], []
            for k, req in enumerate(batch):
                if req.sim.ready_event is not None:  # its set-up, on its client's stream
                    lane.stream.wait_event(req.sim.ready_event)
                    req.sim.ready_event = None
                sets.append(req.sim.products)
                tiles += req.sim.tiles(k, self.dt)
            # every set receives this step's products only (zeroed by the step itself); a
            # simulation's previous step is complete (observed before its request was made)
            lane.handle.step(tiles, seed=self.seed, step=0, counters=lane.counters,
                             product_sets=sets, push=True, zero_product_counts=True,
                             stream=lane.stream)
            lane.event = _event(lane.stream)
            now = self._now()
            for req in batch:
                req.t_dispatch = now
                req.sim.last_batch = len(batch)
            lane.batch = batch
            self.batch_sizes.append(len(batch))

    def _complete(self):
        for lane in self.lanes:
            if lane.batch and lane.event.query():
                now = self._now()
                for req in lane.batch:
                    sim = req.sim
                    self.latencies.append(now - req.t_submit)
                    sim.step += 1
                    sim.in_flight = False
                    if self.on_step is not None:
                        self.on_step(sim)
                    if sim.step >= sim.spec.steps:
                        self._release(sim)
                lane.batch = []

    def _release(self, sim: Simulation):
        del self.active[sim.spec.job_id]
        self.sched.release(sim.spec)
        self.done_jobs += 1

    def run(self, time_limit: float = 600.0) -> Dict:
        """Serves every added job to completion (or until time_limit seconds)."""
        import torch

        torch.cuda.synchronize(self.dev)
        for lane in self.lanes:
            lane.counters.reset()
        n_jobs = len(self.pending)
        self.t0 = time.perf_counter()
        while self.done_jobs < n_jobs:
            now = self._now()
            if now > time_limit:
                raise RuntimeError(f"serving did not finish within {time_limit} s")
            self._complete()
            self._arrivals(now)
            self._admit(now)
            self._clients()
            self._dispatch()
        torch.cuda.synchronize(self.dev)
        wall = self._now()
        c = collections.Counter()
        for lane in self.lanes:
            c.update(lane.counters.as_dict())
        return dict(wall=wall, jobs=n_jobs, requests=len(self.latencies), counters=dict(c),
                    updates_per_s=c["processed"] / wall,
                    p50_ms=percentile(self.latencies, 50) * 1e3,
                    p99_ms=percentile(self.latencies, 99) * 1e3,
                    mean_batch=sum(self.batch_sizes) / max(1, len(self.batch_sizes)),
                    batches=len(self.batch_sizes),
                    admission_wait_p50_ms=percentile(self.admission_waits, 50) * 1e3,
                    admission_wait_max_ms=max(self.admission_waits, default=0.0) * 1e3,
                    waited=len(self.sched.deferred), lane_queue_bytes=self.queue_bytes)

    def close(self):
        for lane in self.lanes:
            lane.handle.close()


def _event(stream):
    import torch

    e = torch.cuda.Event()
    e.record(stream)
    return e


def workload(clients: int = 8, jobs_per_client: int = 6, steps: int = 20, mean: float = 2e6,
             lo: float = 1e4, hi: float = 2e7, think: float = 0.005,
             seed: int = inputs.SEED_SERVE) -> List[JobSpec]:
    """Served-form job mix: the simulations of each client arrive as a Poisson process (mean
    gap `think` seconds); sizes ~ Exp(mean) clamped to [lo, hi], half electrons and half
    photons; every simulation takes `steps` steps."""
    import numpy as np

    specs, jid = [], 0
    for c in range(clients):
        t = 0.0
        for j in range(jobs_per_client):
            u = inputs.uniforms(seed, 200 + c, np.array([2 * j, 2 * j + 1]))
            t += -think * math.log(u[0])
            n = int(min(hi, max(lo, -mean * math.log(u[1]))))
            specs.append(JobSpec(jid, n // 2, n - n // 2, steps, arrival=t, client=c))
            jid += 1
    return specs
