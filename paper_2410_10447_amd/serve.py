"""Continuous-batching serving loop for docking jobs (host side).

A docking job is one ligand, one resident receptor grid set and a population
of individuals (runs x population) that each get `iterations` ADADELTA steps
plus a final evaluation (Sec. 2.1 local search; each ligand is an independent
docking task, Sec. 1). Jobs arrive over time. The server

* admits a queued job when the in-flight individuals and the device bytes
  its state needs fit the configured budgets (FIFO: a job that does not fit
  blocks the ones behind it, so large jobs are not starved);
* runs the local search in chunks of `chunk_iters` steps: every chunk is ONE
  persistent launch over all in-flight jobs (each job an item with its own
  remaining step count; the final evaluation is requested only in a job's last
  chunk). Jobs join and leave at chunk boundaries, so requests that arrive
  while others are on the GPU start at the next chunk and their work overlaps
  in the same launch;
* keeps up to `depth` chunks enqueued so the device never idles while the host
  plans the next one; completion is observed through events;
* lets a client withdraw a job (`cancel`, or `JobSpec.cancel_at`): a queued job
  leaves the queue; an admitted one gets no further chunk, and its state is
  released once no enqueued chunk carries it (a chunk already on the device
  finishes; its work on the job is discarded).

Because the kernel computes every individual independently and in a fixed
order, and a chunked search equals an unchunked one bit for bit, a job's
result does not depend on which other jobs shared its launches.

The executor is an interface so that the admission and scheduling logic can
be tested on a CPU with a simulated device (`FakeExecutor`).
"""
from __future__ import annotations

import collections
import heapq
import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class JobSpec:
    job_id: int
    ligand: object            # synth.Ligand (or any object with the ligand fields)
    grid_id: int
    genotypes: object         # float32 [n, 7 + T] starting points, or a function that
                              # returns them when the job is admitted (then `n` is set)
    arrival: float            # seconds, on the server clock
    iterations: int = 300
    n: int = 0                # individuals, when `genotypes` is a function
    cancel_at: float = math.inf   # seconds, on the server clock: the client withdraws the job

    @property
    def count(self) -> int:
        return self.n if callable(self.genotypes) else int(self.genotypes.shape[0])

    def starting_points(self) -> np.ndarray:
        return self.genotypes() if callable(self.genotypes) else self.genotypes


@dataclass
class JobRecord:
    spec: JobSpec
    admitted: float = math.nan
    done: float = math.nan
    iters_done: int = 0
    footprint: int = 0
    handle: object = None      # executor-side state
    chunks: int = 0
    error: str = ""
    result: object = None
    cancelled: bool = False    # withdrawn; released at the next chunk boundary

    @property
    def latency(self) -> float:
        return self.done - self.spec.arrival


@dataclass
class ServeStats:
    completed: list = field(default_factory=list)
    failed: list = field(default_factory=list)
    cancelled: list = field(default_factory=list)
    evals: int = 0
    wall: float = 0.0
    peak_device_bytes: int = 0
    mean_device_bytes: float = 0.0
    resident_grid_bytes: int = 0
    chunks: int = 0
    max_queue: int = 0

    def latencies(self):
        return np.array([r.latency for r in self.completed])

    def summary(self) -> dict:
        lat = self.latencies()
        out = {"jobs": len(self.completed), "failed": len(self.failed),
               "cancelled": len(self.cancelled), "evals": self.evals,
               "wall_s": self.wall,
               "evals_per_s": self.evals / self.wall if self.wall > 0 else 0.0,
               "chunks": self.chunks, "max_queue": self.max_queue,
               "peak_state_bytes": self.peak_device_bytes,
               "mean_state_bytes": self.mean_device_bytes,
               "resident_grid_bytes": self.resident_grid_bytes}
        if len(lat):
            out.update({"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                        "mean_s": float(lat.mean())})
        return out


def state_bytes(n: int, n_genes: int) -> int:
    """Device bytes of one job's local-search state (see the C ABI item)."""
    return n * (4 * n_genes * 4 + 3 * 4)


class Server:
    def __init__(self, executor, max_individuals: int, device_budget: int,
                 chunk_iters: int = 50, depth: int = 2, clock=None,
                 chunk_timeout: float = math.inf):
        if chunk_iters < 1 or depth < 1:
            raise ValueError("chunk_iters and depth must be >= 1")
        self.ex = executor
        self.max_individuals = max_individuals
        self.budget = device_budget
        self.chunk_iters = chunk_iters
        self.depth = depth
        self.chunk_timeout = chunk_timeout
        self.clock = clock or time.perf_counter
        self.queue = collections.deque()
        self.inflight: list[JobRecord] = []
        self.pending = collections.deque()   # (token, [(record, iters, final)])
        self.stats = ServeStats()
        self.used_individuals = 0
        self.used_bytes = 0
        self._t0 = None
        self._occ_area = 0.0
        self._occ_t = None

    # -- admission -------------------------------------------------------
    def submit(self, spec: JobSpec):
        rec = JobRecord(spec)
        rec.footprint = self.ex.footprint(spec)
        if spec.count > self.max_individuals or rec.footprint > self.budget:
            raise ValueError(f"job {spec.job_id} can never fit the budgets")
        self.queue.append(rec)
        self.stats.max_queue = max(self.stats.max_queue, len(self.queue))

    def _admit(self, now):
        while self.queue:
            rec = self.queue[0]
            n = rec.spec.count
            if self.used_individuals + n > self.max_individuals or \
                    self.used_bytes + rec.footprint > self.budget:
                break
            self.queue.popleft()
            rec.handle = self.ex.prepare(rec.spec)
            rec.admitted = now
            self.used_individuals += n
            self.used_bytes += rec.footprint
            self.stats.peak_device_bytes = max(self.stats.peak_device_bytes, self.used_bytes)
            self.inflight.append(rec)

    # -- cancellation ----------------------------------------------------
    def cancel(self, job_id, now=None) -> bool:
        """Withdraw a queued or admitted job; False if it is not (or no
        longer) queued or in flight."""
        if now is None:
            now = self.clock() - (self._t0 if self._t0 is not None else 0.0)
        for rec in self.queue:
            if rec.spec.job_id == job_id:
                self.queue.remove(rec)
                rec.cancelled = True
                rec.error = "cancelled"
                rec.done = now
                self.stats.cancelled.append(rec)
                return True
        for rec in self.inflight:
            if rec.spec.job_id == job_id and not rec.cancelled:
                rec.cancelled = True
                self._drop_cancelled(now)
                return True
        return False

    def _drop_cancelled(self, now):
        """Release withdrawn jobs that no enqueued chunk carries any more."""
        carried = {id(r) for _, plan, _ in self.pending for r, _, _ in plan}
        for rec in [r for r in self.inflight if r.cancelled and id(r) not in carried]:
            self.inflight.remove(rec)
            self.used_individuals -= rec.spec.count
            self.used_bytes -= rec.footprint
            self.ex.release(rec.handle)
            rec.error = "cancelled"
            rec.done = now
            self.stats.cancelled.append(rec)

    # -- chunks ----------------------------------------------------------
    def _planned_iters(self, rec):
        """Steps already enqueued for rec (done + in pending chunks)."""
        return rec.iters_done + sum(it for _, plan, _ in self.pending for r, it, _ in plan if r is rec)

    def _launch_chunk(self):
        plan = []
        for rec in self.inflight:
            if rec.cancelled:
                continue
            planned = self._planned_iters(rec)
            remaining = rec.spec.iterations - planned
            finished_enqueued = any(r is rec and fin for _, p, _ in self.pending for r, _, fin in p)
            if remaining <= 0 and finished_enqueued:
                continue
            k = min(self.chunk_iters, remaining)
            final = (planned + k) >= rec.spec.iterations
            plan.append((rec, k, final))
        if not plan:
            return False
        try:
            token = self.ex.launch([(r.handle, k, fin) for r, k, fin in plan], self.chunk_iters)
        except Exception as e:  # a failed launch fails only the jobs it carried
            for r, _, _ in plan:
                self._fail(r, f"launch failed: {e}")
            return True
        self.pending.append((token, plan, self.clock() - self._t0))
        self.stats.chunks += 1
        for r, _, _ in plan:
            r.chunks += 1
        return True

    def _fail(self, rec, why):
        rec.error = why
        rec.done = self.clock() - self._t0
        if rec in self.inflight:
            self.inflight.remove(rec)
            self.used_individuals -= rec.spec.count
            self.used_bytes -= rec.footprint
            try:
                self.ex.release(rec.handle)
            except Exception:
                pass
        self.stats.failed.append(rec)

    def _retire(self, now):
        progressed = False
        # watchdog: a chunk that does not complete in time fails its jobs
        while self.pending and not self.ex.done(self.pending[0][0]) and \
                now - self.pending[0][2] > self.chunk_timeout:
            _, plan, _ = self.pending.popleft()
            for rec, _, _ in plan:
                if rec in self.inflight:
                    self._fail(rec, "chunk timed out")
        while self.pending and self.ex.done(self.pending[0][0]):
            token, plan, _ = self.pending.popleft()
            progressed = True
            for rec, k, final in plan:
                if rec not in self.inflight:
                    continue
                rec.iters_done += k
                n = rec.spec.count
                self.stats.evals += n * (k + (1 if final else 0))
                if final and not rec.cancelled:
                    rec.done = now
                    rec.result = self.ex.result(rec.handle)
                    self.ex.release(rec.handle)
                    self.inflight.remove(rec)
                    self.used_individuals -= n
                    self.used_bytes -= rec.footprint
                    self.stats.completed.append(rec)
        self._drop_cancelled(now)
        return progressed

    def _account(self, now):
        if self._occ_t is not None:
            self._occ_area += self.used_bytes * (now - self._occ_t)
        self._occ_t = now

    # -- driver ----------------------------------------------------------
    def run(self, specs, poll: float = 2e-4, until_empty: bool = True, horizon: float = math.inf,
            progress=None, progress_every: float = 30.0):
        """Serve `specs` (arrival times relative to the start of run).
        `progress(now, stats)` is called every `progress_every` seconds."""
        arrivals = sorted(specs, key=lambda s: s.arrival)
        i = 0
        t0 = self.clock()
        self._t0 = t0
        self._occ_t = 0.0
        next_report = progress_every
        while True:
            now = self.clock() - t0
            if progress is not None and now >= next_report:
                progress(now, self.stats)
                next_report += progress_every
            while i < len(arrivals) and arrivals[i].arrival <= now and arrivals[i].arrival <= horizon:
                self.submit(arrivals[i])
                i += 1
            for rec in [r for r in (*self.queue, *self.inflight) if r.spec.cancel_at <= now and not r.cancelled]:
                self.cancel(rec.spec.job_id, now)
            self._retire(now)
            self._admit(now)
            self._account(now)
            while len(self.pending) < self.depth and self._launch_chunk():
                pass
            no_more = i >= len(arrivals) or arrivals[i].arrival > horizon
            if no_more and not self.queue and not self.inflight and not self.pending:
                break
            if not until_empty and no_more and now > horizon:
                break
            if self.pending and not self.ex.done(self.pending[0][0]):
                self.ex.wait(self.pending[0][0], poll)
                now2 = self.clock() - t0
                if now2 - self.pending[0][2] > self.chunk_timeout:
                    continue
            elif i < len(arrivals):
                dt = arrivals[i].arrival - (self.clock() - t0)
                if dt > 0 and not self.pending:
                    time.sleep(min(dt, poll)) if self.clock is time.perf_counter else self.ex.idle(dt)
        self.stats.wall = self.clock() - t0
        self.stats.mean_device_bytes = self._occ_area / self.stats.wall if self.stats.wall > 0 else 0.0
        return self.stats


def poisson_arrivals(rate: float, duration: float, seed: int):
    """Arrival times of a Poisson process with `rate` per second on [0, duration)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return out
        out.append(t)


# ---------------------------------------------------------------------------
# Executors
# ---------------------------------------------------------------------------

class GpuExecutor:
    """Runs chunks through the C ABI on one stream; grid sets stay resident."""

    def __init__(self, grid_sets, ff, variant: int = 0, device="cuda", use_table: bool = False):
        import torch
        from . import dock
        self.dock = dock
        self.torch = torch
        self.device = device
        self.variant = variant
        self.use_table = use_table   # each job takes its size bucket's tuned variant and
                                     # threads per individual
        self.ff = ff
        self.grids = [dock.Grids.from_synth(g, device) for g in grid_sets]
        self.grid_bytes = sum(g.nbytes() for g in self.grids)
        self.stream = torch.cuda.current_stream()
        # results leave on a side stream (default priority) so that reading a
        # finished job does not wait for the chunks queued after it
        self.side = torch.cuda.Stream()
        self._ws_pool = []

    def footprint(self, spec):
        G = 7 + int(len(spec.ligand.rot_bonds))
        return state_bytes(spec.count, G) + 8192

    def prepare(self, spec):
        torch = self.torch
        L = self.dock.Ligand(spec.ligand, self.ff, device=self.device, upload=False)
        L.upload(self.device, stream=self.stream)
        host = torch.from_numpy(np.ascontiguousarray(spec.starting_points())).pin_memory()
        with torch.cuda.stream(self.stream):
            gen = host.to(self.device, non_blocking=True)
            st = self.dock.LSState.start(gen)
        var, tpi, plain, two = -1, 0, False, False
        if self.use_table:
            from . import autotune
            pick = autotune.choose(L.n_atoms, L.n_torsions)
            var = int(pick["variant"])
            tpi = int(pick.get("threads_per_ind", 64))
            plain = bool(pick.get("plain_maps", False))
            two = bool(pick.get("two_per_wave", False))
        return {"ligand": L, "state": st, "grids": self.grids[spec.grid_id], "host": host,
                "variant": var, "threads_per_ind": tpi, "plain_maps": plain,
                "two_per_wave": two if self.use_table else False}

    def launch(self, plan, max_iters):
        jobs = [self.dock.LsJob(h["grids"], h["ligand"], h["state"], h["variant"], k, 1 if fin else 0,
                                threads_per_ind=h.get("threads_per_ind", 0),
                                plain_maps=h.get("plain_maps", False),
                                two_per_wave=h.get("two_per_wave", False))
                for h, k, fin in plan]
        need = self.dock.workspace_bytes(len(jobs))
        # a workspace per in-flight chunk: reuse one whose chunk has completed
        ws = None
        for cand, ev in self._ws_pool:
            if cand.numel() >= need and ev.query():
                ws = cand
                self._ws_pool.remove((cand, ev))
                break
        if ws is None:
            ws = self.torch.empty(max(need, 4096), dtype=self.torch.uint8, device=self.device)
        self.dock.local_search(jobs, max_iters, variant=self.variant, workspace=ws,
                               stream=self.stream)
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        self._ws_pool.append((ws, ev))
        return ev

    def done(self, token):
        return token.query()

    def wait(self, token, poll):
        time.sleep(poll)

    def idle(self, dt):
        time.sleep(min(dt, 1e-3))

    def result(self, handle):
        torch = self.torch
        st = handle["state"]
        with torch.cuda.stream(self.side):
            be = torch.empty(st.best_energy.shape, dtype=st.best_energy.dtype, pin_memory=True)
            bg = torch.empty(st.best_genotype.shape, dtype=st.best_genotype.dtype, pin_memory=True)
            be.copy_(st.best_energy, non_blocking=True)
            bg.copy_(st.best_genotype, non_blocking=True)
        self.side.synchronize()
        return {"best_energy": be.numpy(), "best_genotype": bg.numpy()}

    def release(self, handle):
        handle.clear()


class FakeExecutor:
    """Simulated device for CPU tests: a chunk takes `cost * evals` seconds of a
    virtual clock, chunks run one after another, and results are a
    deterministic function of the job alone."""

    def __init__(self, sec_per_eval: float = 1e-8, fail_on=None):
        self.t = 0.0
        self.busy_until = 0.0
        self.sec_per_eval = sec_per_eval
        self.launched = []
        self.fail_on = fail_on or set()
        self.live = {}

    def clock(self):
        return self.t

    def footprint(self, spec):
        return state_bytes(spec.count, spec.starting_points().shape[1])

    def prepare(self, spec):
        h = {"spec": spec, "iters": 0, "final": False}
        self.live[spec.job_id] = h
        return h

    def launch(self, plan, max_iters):
        evals = 0
        for h, k, fin in plan:
            if h["spec"].job_id in self.fail_on:
                raise RuntimeError(f"injected failure for job {h['spec'].job_id}")
            assert not h["final"], "job launched after its final evaluation"
            h["iters"] += k
            h["final"] = fin
            evals += h["spec"].count * (k + (1 if fin else 0))
        start = max(self.t, self.busy_until)
        self.busy_until = start + evals * self.sec_per_eval
        self.launched.append([(h["spec"].job_id, k, fin) for h, k, fin in plan])
        return self.busy_until

    def done(self, token):
        return self.t >= token

    def wait(self, token, poll):
        self.t = max(self.t + poll, min(token, self.t + 1.0))
        if self.t < token:
            self.t = token

    def idle(self, dt):
        self.t += dt

    def result(self, handle):
        spec = handle["spec"]
        rng = np.random.default_rng(spec.job_id)
        return {"iters": handle["iters"], "final": handle["final"],
                "value": float(rng.normal()) + float(spec.starting_points().sum())}

    def release(self, handle):
        self.live.pop(handle["spec"].job_id, None)
