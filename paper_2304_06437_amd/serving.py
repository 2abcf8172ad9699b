"""Continuous batching of independent lattice Boltzmann simulations.

A request is one simulation (lattice, domain, relaxation time, initial flow,
storage precision, number of steps).  The server

  * admits queued requests in arrival order while their device footprint
    (``lb_required_bytes``) fits the HBM budget, whenever memory frees up;
  * keeps every admitted simulation resident on the GPU and advances all of
    them together, ``chunk_steps`` at a time, through ``lb_batch_step``
    (simulations of the same kernel configuration share one launch per
    sweep; fixed-membership runs are replayed from a captured HIP graph);
  * reads each finished simulation's moments back, records its
    time-to-solution (arrival to moments on the host) and releases its memory.

Requests that arrive while others are running join at the next chunk
boundary.  A request whose footprint exceeds the whole budget is rejected; a
request whose set-up or read-out fails (or whose state became non-finite) is
marked failed without affecting the others.

With ``overlap=True`` the set-up of admitted requests and the read-back of
finished ones run on a worker thread while the main thread steps the batch:
the GPU backend does that work on a stream of its own and hands each
simulation to the batch's stream (``lb_set_stream``) once it is initialised,
and back for the read-back, with that stream ordered after the batch's
stream after every chunk.

Not part of the paper: the serving loop is how this library runs many small
independent simulations on one GPU.
"""
from __future__ import annotations

import math
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import inputs


@dataclass
class JobSpec:
    job_id: int
    lattice: int                  # 9, 19 or 27
    shape: tuple                  # (nx, ny, nz); nz = 1 for D2Q9
    steps: int
    storage: str = "f32"          # f32, f16s, bf16s, f64
    flow: str = "tg"              # "tg" (Taylor-Green) or "channel"
    tau: float = 0.6
    arrival: float = 0.0          # seconds after the start of the run
    amplitude: float = 0.01       # Taylor-Green velocity amplitude u0

    @property
    def nodes(self) -> int:
        return self.shape[0] * self.shape[1] * self.shape[2]

    def fields(self):
        """Initial density and velocity of the request's flow."""
        nx, ny, nz = self.shape
        D = 2 if self.lattice == 9 else 3
        if self.flow == "tg":
            if D == 2:
                return inputs.taylor_green_2d(nx, ny, self.amplitude)
            return inputs.taylor_green_3d(nx, ny, nz, self.amplitude)
        if self.flow == "channel":
            return inputs.channel_noise(nx, ny, nz, D, seed=12345 + self.job_id)
        raise ValueError(self.flow)

    def force(self):
        return (1e-6, 0.0, 0.0) if self.flow == "channel" else (0.0, 0.0, 0.0)

    def bc(self):
        if self.flow != "channel":
            return (0, 0, 0)
        return (0, 1, 0) if self.lattice == 9 else (0, 0, 1)


@dataclass
class JobResult:
    job_id: int
    status: str                   # done, failed, rejected
    arrival: float
    admitted: float = math.nan
    finished: float = math.nan
    lattice_updates: int = 0
    error: str = ""
    moments: dict | None = None

    @property
    def time_to_solution(self) -> float:
        return self.finished - self.arrival


@dataclass
class ServeReport:
    results: list
    makespan: float
    max_active: int
    peak_bytes: int
    chunks: int = 0
    phase_s: dict = field(default_factory=dict)  # host time: create, step, read, idle

    def _tts(self):
        return np.array([r.time_to_solution for r in self.results if r.status == "done"])

    @property
    def p50(self) -> float:
        t = self._tts()
        return float(np.percentile(t, 50)) if t.size else math.nan

    @property
    def p99(self) -> float:
        t = self._tts()
        return float(np.percentile(t, 99)) if t.size else math.nan

    @property
    def lattice_updates(self) -> int:
        return sum(r.lattice_updates for r in self.results if r.status == "done")

    @property
    def mlups(self) -> float:
        return self.lattice_updates / self.makespan / 1e6 if self.makespan > 0 else math.nan

    def summary(self) -> dict:
        st = [r.status for r in self.results]
        return {
            "jobs": len(st), "done": st.count("done"), "failed": st.count("failed"),
            "rejected": st.count("rejected"), "p50_s": round(self.p50, 4),
            "p99_s": round(self.p99, 4), "aggregate_MLUPS": round(self.mlups, 1),
            "makespan_s": round(self.makespan, 3), "max_active": self.max_active,
            "peak_GB": round(self.peak_bytes / 1e9, 3), "chunks": self.chunks,
            "phase_s": {k: round(v, 3) for k, v in self.phase_s.items()},
        }


class _Active:
    __slots__ = ("spec", "handle", "remaining", "nbytes", "result")

    def __init__(self, spec, handle, nbytes, result):
        self.spec = spec
        self.handle = handle
        self.remaining = spec.steps
        self.nbytes = nbytes
        self.result = result


class GpuBackend:
    """liblb.so simulations in torch-owned device memory on one stream."""

    def __init__(self, device=None, graphs: bool = True, keep_moments: bool = False):
        import torch

        from . import lb

        self.torch = torch
        self.lb = lb
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        self.stream = torch.cuda.current_stream(self.device)
        # set-up and read-back stream of the overlapped server (default priority)
        self.side = torch.cuda.Stream(self.device)
        self.batch = lb.lb_batch_create(self.stream.cuda_stream)
        lb.lb_batch_set_graphs(self.batch, graphs)
        self.keep_moments = keep_moments

    def params(self, spec: JobSpec):
        from .sim import make_params

        return make_params(lattice=spec.lattice, shape=spec.shape, tau=spec.tau,
                           force=spec.force(), bc=spec.bc(), storage=spec.storage)

    def required_bytes(self, spec: JobSpec) -> int:
        n = self.lb.lb_required_bytes(self.params(spec))
        if n == 0:
            raise ValueError(f"invalid request {spec}")
        return n

    def prepare(self, spec: JobSpec):
        """Host-side initial fields (runs on the server's worker thread)."""
        return spec.fields()

    def create(self, spec: JobSpec, prepared=None):
        from .sim import Simulation

        sim = Simulation(self.params(spec), device=self.device, stream=self.stream)
        rho, u = prepared if prepared is not None else spec.fields()
        sim.init(rho, u)
        return sim

    def create_aside(self, spec: JobSpec, prepared=None):
        """create() on the side stream (worker thread); lb_init is synchronous,
        so the simulation is ready for the batch's stream when this returns."""
        from .sim import Simulation

        with self.torch.cuda.stream(self.side):
            sim = Simulation(self.params(spec), device=self.device, stream=self.side)
            rho, u = prepared if prepared is not None else spec.fields()
            sim.init(rho, u)
        sim.set_stream(self.stream)
        return sim

    def step(self, handles, nsteps):
        self.lb.lb_batch_step(self.batch, [s.handle for s in handles], nsteps)

    def blown_up(self, handles) -> list:
        """Indices of the simulations whose mass or momentum (FP64 device
        reduction, one round trip for all) is no longer finite."""
        if not handles:
            return []
        sums, st = self.lb.lb_batch_conserved(self.batch, [s.handle for s in handles])
        if st == self.lb.LB_OK:
            return []
        return [i for i in range(len(handles)) if not np.isfinite(sums[i, :4]).all()]

    def chunk_done(self):
        """Order the side stream after everything enqueued on the batch's
        stream so far.  Called by the main thread between batch steps, when
        no graph capture is active on the batch's stream: HIP rejects a wait
        on that stream's work while it is being captured, even for work
        recorded before the capture began."""
        self.side.wait_stream(self.stream)

    def read(self, sim, spec: JobSpec) -> dict:
        out = sim.moments(rho=self.keep_moments, u=True, pineq=False, allow_nonfinite=True)
        if out["status"] != self.lb.LB_OK or not np.isfinite(out["u"]).all():
            raise FloatingPointError("non-finite state")
        return out

    def read_aside(self, sim, spec: JobSpec) -> dict:
        """read() on the side stream (worker thread), which chunk_done() has
        ordered after the simulation's last chunk; the handle stays on the
        side stream for destroy()."""
        sim.set_stream(self.side)
        with self.torch.cuda.stream(self.side):
            return self.read(sim, spec)

    def destroy(self, sim):
        sim.close()

    def close(self):
        if self.batch is not None:
            self.lb.lb_batch_destroy(self.batch)
            self.batch = None


class Server:
    """check_finite: after every chunk, stop the simulations whose state is
    no longer finite (marked failed at that chunk, memory released), using
    the backend's blown_up() when it has one.  progress: optional callable
    taking a dict of counters (time, chunks, active, finished), called after
    every chunk."""

    def __init__(self, backend, hbm_budget: int, chunk_steps: int = 200,
                 max_active: int = 256, keep_moments: bool = False, clock=time.perf_counter,
                 sleep=time.sleep, overlap: bool = False, check_finite: bool = True,
                 progress=None):
        self.check_finite = check_finite
        # progress(dict): called after every chunk with the run's counters
        self.progress = progress
        self.backend = backend
        self.budget = int(hbm_budget)
        self.chunk = int(chunk_steps)
        self.max_active = int(max_active)
        self.keep_moments = keep_moments
        self.clock = clock
        self.sleep = sleep
        self.overlap = overlap

    def run(self, specs) -> ServeReport:
        prep = getattr(self.backend, "prepare", None)
        pool = ThreadPoolExecutor(max_workers=2) if prep is not None else None
        try:
            if self.overlap:
                return self._run_overlapped(specs, pool, prep)
            return self._run(specs, pool, prep)
        finally:
            if pool is not None:
                pool.shutdown(wait=True, cancel_futures=True)

    def _admit_check(self, spec, results, futures):
        """(need, None) for a request that may be admitted, (None, result) for
        one rejected outright."""
        res = JobResult(spec.job_id, "queued", spec.arrival)
        try:
            need = self.backend.required_bytes(spec)
        except Exception as e:  # invalid request
            res.status, res.error = "rejected", str(e)
        else:
            if need <= self.budget:
                return need, res
            res.status, res.error = "rejected", f"needs {need} B > budget {self.budget} B"
        futures.pop(spec.job_id, None)
        results[spec.job_id] = res
        return None, res

    def _run_overlapped(self, specs, pool, prep) -> ServeReport:
        """As _run, with set-up and read-back on one worker thread while the
        main thread steps the resident batch.  Memory counts against the
        budget from admission until the read-back has released it."""
        from concurrent.futures import FIRST_COMPLETED, wait

        be = self.backend
        create = getattr(be, "create_aside", be.create)
        read = getattr(be, "read_aside", be.read)
        chunk_done = getattr(be, "chunk_done", lambda: None)
        worker = ThreadPoolExecutor(max_workers=1)
        pending = deque(sorted(specs, key=lambda s: (s.arrival, s.job_id)))
        queue: deque = deque()
        active: list = []
        creating: list = []   # (future, spec, need, result)
        reading: list = []    # (future, _Active)
        results = {}
        futures = {}
        used = peak = 0
        max_active = chunks = 0
        phase = {"create": 0.0, "step": 0.0, "read": 0.0, "idle": 0.0, "wait": 0.0}
        t0 = self.clock()

        def now():
            return self.clock() - t0

        def setup_task(spec, fut):
            tc = self.clock()
            try:
                return create(spec, fut.result()) if fut is not None else create(spec)
            finally:
                phase["create"] += self.clock() - tc

        def read_task(a):
            tr = self.clock()
            try:
                out = read(a.handle, a.spec)
            finally:
                self._release(a)
                phase["read"] += self.clock() - tr
            return out

        try:
            while pending or queue or active or creating or reading:
                t = now()
                while pending and pending[0].arrival <= t:
                    spec = pending.popleft()
                    queue.append(spec)
                    if pool is not None:
                        futures[spec.job_id] = pool.submit(prep, spec)
                # finished read-backs release their memory
                still = []
                for fut, a in reading:
                    if not fut.done():
                        still.append((fut, a))
                        continue
                    try:
                        out = fut.result()
                        a.result.status = "done"
                        a.result.lattice_updates = a.spec.nodes * a.spec.steps
                        if self.keep_moments:
                            a.result.moments = out
                    except Exception as e:
                        a.result.status, a.result.error = "failed", repr(e)
                    a.result.finished = now()
                    results[a.spec.job_id] = a.result
                    used -= a.nbytes
                reading = still
                # admission in arrival order while the head of the queue fits
                while queue and len(active) + len(creating) < self.max_active:
                    need, res = self._admit_check(queue[0], results, futures)
                    if need is None:
                        queue.popleft()
                        continue
                    if used + need > self.budget:
                        break
                    spec = queue.popleft()
                    res.admitted = now()
                    used += need
                    peak = max(peak, used)
                    creating.append((worker.submit(setup_task, spec, futures.pop(spec.job_id, None)),
                                     spec, need, res))
                # set-ups that have finished join the batch
                still = []
                for fut, spec, need, res in creating:
                    if not fut.done():
                        still.append((fut, spec, need, res))
                        continue
                    try:
                        active.append(_Active(spec, fut.result(), need, res))
                    except Exception as e:
                        res.status, res.error, res.finished = "failed", repr(e), now()
                        results[spec.job_id] = res
                        used -= need
                creating = still
                max_active = max(max_active, len(active))
                if not active:
                    if creating or reading:
                        tw = self.clock()
                        wait([f for f, *_ in creating] + [f for f, _ in reading],
                             return_when=FIRST_COMPLETED)
                        phase["wait"] += self.clock() - tw
                    elif pending and not queue:
                        ti = self.clock()
                        self.sleep(max(0.0, min(pending[0].arrival - now(), 0.05)))
                        phase["idle"] += self.clock() - ti
                    continue
                nsteps = [min(self.chunk, a.remaining) for a in active]
                ts = self.clock()
                try:
                    be.step([a.handle for a in active], nsteps)
                    chunk_done()  # read-backs below are ordered after this chunk
                    phase["step"] += self.clock() - ts
                except Exception as e:
                    for a in active:
                        a.result.status, a.result.error, a.result.finished = "failed", repr(e), now()
                        results[a.spec.job_id] = a.result
                        self._release(a)
                        used -= a.nbytes
                    active = []
                    continue
                chunks += 1
                if self.progress is not None:
                    self.progress({"t": now(), "chunks": chunks, "active": len(active),
                                   "finished": len(results)})
                kept, failed = self._blown_up(active, nsteps)
                for a, done in failed:
                    a.result.status = "failed"
                    a.result.error = f"non-finite state within {done} steps"
                    a.result.finished = now()
                    results[a.spec.job_id] = a.result
                    self._release(a)
                    used -= a.nbytes
                if failed:
                    keep = {id(a) for a in kept}
                    nsteps = [k for a, k in zip(active, nsteps) if id(a) in keep]
                    active = kept
                still = []
                for a, k in zip(active, nsteps):
                    a.remaining -= k
                    if a.remaining > 0:
                        still.append(a)
                    else:
                        reading.append((worker.submit(read_task, a), a))
                active = still
        finally:
            worker.shutdown(wait=True)
        ordered = [results[s.job_id] for s in sorted(specs, key=lambda s: s.job_id)]
        return ServeReport(ordered, now(), max_active, peak, chunks, phase)

    def _run(self, specs, pool, prep) -> ServeReport:
        pending = deque(sorted(specs, key=lambda s: (s.arrival, s.job_id)))
        queue: deque = deque()
        active: list = []
        results = {}
        futures = {}
        used = peak = 0
        max_active = chunks = 0
        phase = {"create": 0.0, "step": 0.0, "read": 0.0, "idle": 0.0}
        t0 = self.clock()

        def now():
            return self.clock() - t0

        while pending or queue or active:
            t = now()
            while pending and pending[0].arrival <= t:
                spec = pending.popleft()
                queue.append(spec)
                if pool is not None:
                    # host-side preparation overlaps the GPU work of the running chunk
                    futures[spec.job_id] = pool.submit(prep, spec)
            # admission: arrival order, as long as the head of the queue fits
            while queue and len(active) < self.max_active:
                spec = queue[0]
                res = JobResult(spec.job_id, "queued", spec.arrival)
                try:
                    need = self.backend.required_bytes(spec)
                except Exception as e:  # invalid request
                    queue.popleft()
                    res.status, res.error = "rejected", str(e)
                    results[spec.job_id] = res
                    futures.pop(spec.job_id, None)
                    continue
                if need > self.budget:
                    futures.pop(spec.job_id, None)
                    queue.popleft()
                    res.status, res.error = "rejected", f"needs {need} B > budget {self.budget} B"
                    results[spec.job_id] = res
                    continue
                if used + need > self.budget:
                    break
                queue.popleft()
                res.admitted = now()
                tc = self.clock()
                try:
                    fut = futures.pop(spec.job_id, None)
                    if fut is not None:
                        handle = self.backend.create(spec, fut.result())
                    else:
                        handle = self.backend.create(spec)
                except Exception as e:
                    res.status, res.error, res.finished = "failed", repr(e), now()
                    results[spec.job_id] = res
                    continue
                finally:
                    phase["create"] += self.clock() - tc
                used += need
                peak = max(peak, used)
                active.append(_Active(spec, handle, need, res))
            max_active = max(max_active, len(active))
            if not active:
                if pending and not queue:
                    ti = self.clock()
                    self.sleep(max(0.0, min(pending[0].arrival - now(), 0.05)))
                    phase["idle"] += self.clock() - ti
                continue
            # one chunk for every resident simulation
            nsteps = [min(self.chunk, a.remaining) for a in active]
            ts = self.clock()
            try:
                self.backend.step([a.handle for a in active], nsteps)
                phase["step"] += self.clock() - ts
            except Exception as e:
                # a launch failure poisons the whole batch: fail every member
                for a in active:
                    a.result.status, a.result.error, a.result.finished = "failed", repr(e), now()
                    results[a.spec.job_id] = a.result
                    self._release(a)
                    used -= a.nbytes
                active = []
                continue
            chunks += 1
            if self.progress is not None:
                self.progress({"t": now(), "chunks": chunks, "active": len(active),
                               "finished": len(results)})
            kept, failed = self._blown_up(active, nsteps)
            for a, done in failed:
                a.result.status = "failed"
                a.result.error = f"non-finite state within {done} steps"
                a.result.finished = now()
                results[a.spec.job_id] = a.result
                self._release(a)
                used -= a.nbytes
            if failed:
                keep = {id(a) for a in kept}
                nsteps = [k for a, k in zip(active, nsteps) if id(a) in keep]
                active = kept
            still = []
            for a, k in zip(active, nsteps):
                a.remaining -= k
                if a.remaining > 0:
                    still.append(a)
                    continue
                tr = self.clock()
                try:
                    out = self.backend.read(a.handle, a.spec)
                    a.result.status = "done"
                    a.result.lattice_updates = a.spec.nodes * a.spec.steps
                    if self.keep_moments:
                        a.result.moments = out
                except Exception as e:
                    a.result.status, a.result.error = "failed", repr(e)
                phase["read"] += self.clock() - tr
                a.result.finished = now()
                results[a.spec.job_id] = a.result
                self._release(a)
                used -= a.nbytes
            active = still
        ordered = [results[s.job_id] for s in sorted(specs, key=lambda s: s.job_id)]
        return ServeReport(ordered, now(), max_active, peak, chunks, phase)

    def _blown_up(self, active, stepped_now):
        """Jobs of `active` (each advanced by stepped_now[i] this chunk) whose
        state has blown up: returns (kept, failed), failed as (job, steps
        done so far)."""
        probe = getattr(self.backend, "blown_up", None)
        if not self.check_finite or probe is None or not active:
            return active, []
        bad = set(probe([a.handle for a in active]))
        kept, failed = [], []
        for i, a in enumerate(active):
            if i in bad:
                failed.append((a, a.spec.steps - a.remaining + stepped_now[i]))
            else:
                kept.append(a)
        return kept, failed

    def _release(self, a):
        try:
            self.backend.destroy(a.handle)
        except Exception:
            pass


def poisson_mix(n_jobs: int, rate: float, seed: int = 2026, edge_min: int = 64,
                edge_max: int = 256, steps=(200, 2000), lattices=(9, 19),
                storages=("f32", "f16s"), flows=("tg", "channel")) -> list:
    """Seeded request stream: exponential inter-arrival gaps (mean 1/rate),
    lattice / flow / storage uniform, edge n = round(exp U[ln min, ln max])
    (n^2 for D2Q9, n^3 otherwise), step count uniform in [steps]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    specs = []
    for i in range(n_jobs):
        t += rng.exponential(1.0 / rate)
        lat = int(rng.choice(lattices))
        n = int(round(math.exp(rng.uniform(math.log(edge_min), math.log(edge_max)))))
        shape = (n, n, 1) if lat == 9 else (n, n, n)
        specs.append(JobSpec(job_id=i, lattice=lat, shape=shape,
                             steps=int(rng.integers(steps[0], steps[1] + 1)),
                             storage=str(rng.choice(storages)), flow=str(rng.choice(flows)),
                             tau=0.6, arrival=t))
    return specs
