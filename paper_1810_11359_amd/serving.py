"""Continuous-batching request loop for RIR jobs.

Jobs (one room, its sources and receivers) arrive over time. The scheduler
admits waiting jobs while their device footprint fits a byte budget and a
stream slot is free, launches each group of admitted jobs as one batch on its
own stream (so batches overlap on the device), and retires batches as their
completion events fire, freeing memory and the slot for the next admissions.
It records arrival, admission, launch and finish times per job and reports
p50/p99 latency beside throughput.

The loop is independent of the device: an executor provides ``footprint``,
``launch``, ``done`` and ``finish``. ``GpuExecutor`` runs batches through
``ism_batch_prepare``/``ism_batch_run``; tests drive the same loop with a fake
executor and a virtual clock.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Any, Callable, Deque, Dict, List, Optional

import numpy as np


@dataclass
class Job:
    jid: int
    room: Any            # ism.Room
    src: np.ndarray      # [n_src, 3] float32
    rcv: np.ndarray      # [n_rcv, 3] float32
    arrival: float       # seconds on the scheduler clock
    admitted: float = float("nan")
    launched: float = float("nan")
    finished: float = float("nan")
    footprint: int = 0   # device bytes while in flight
    out: Any = None      # result tensor once finished

    @property
    def n_rirs(self) -> int:
        return int(self.src.shape[0] * self.rcv.shape[0])

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class Stats:
    n_jobs: int
    n_rirs: int
    makespan_s: float
    rirs_per_s: float
    jobs_per_s: float
    p50_ms: float
    p99_ms: float
    mean_batch_jobs: float
    max_in_flight_bytes: int

    def as_dict(self) -> Dict[str, float]:
        return dict(self.__dict__)


class Scheduler:
    """Admission by device-memory budget and free slots; one batch per slot.

    ``max_batch_jobs`` caps how many waiting jobs join one batch; a batch is
    launched as soon as a slot is free (no waiting to fill it), which keeps
    latency low at light load and batches grow naturally under heavy load.
    """

    def __init__(self, executor, budget_bytes: int, n_slots: int = 2, max_batch_jobs: int = 64,
                 clock: Callable[[], float] = time.perf_counter):
        if n_slots < 1 or budget_bytes <= 0 or max_batch_jobs < 1:
            raise ValueError("n_slots, budget_bytes and max_batch_jobs must be positive")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.n_slots = n_slots
        self.max_batch_jobs = max_batch_jobs
        self.clock = clock
        self.waiting: Deque[Job] = deque()
        self.in_flight: List[tuple] = []     # (slot, handle, jobs)
        self.free_slots = list(range(n_slots))
        self.used = 0
        self.max_used = 0
        self.done: List[Job] = []
        self.batch_sizes: List[int] = []

    def submit(self, job: Job) -> None:
        job.footprint = int(self.ex.footprint(job))
        if job.footprint > self.budget:
            raise ValueError(f"job {job.jid} needs {job.footprint} bytes, more than the whole budget")
        self.waiting.append(job)

    def _retire(self) -> int:
        n = 0
        still = []
        for slot, handle, jobs in self.in_flight:
            if self.ex.done(handle):
                now = self.clock()
                self.ex.finish(handle, jobs)
                for j in jobs:
                    j.finished = now
                    self.used -= j.footprint
                    self.done.append(j)
                self.free_slots.append(slot)
                n += 1
            else:
                still.append((slot, handle, jobs))
        self.in_flight = still
        return n

    def _admit_and_launch(self) -> int:
        launched = 0
        while self.free_slots and self.waiting:
            batch = []
            while self.waiting and len(batch) < self.max_batch_jobs and \
                    self.used + self.waiting[0].footprint <= self.budget:
                j = self.waiting.popleft()
                j.admitted = self.clock()
                self.used += j.footprint
                batch.append(j)
            if not batch:
                break  # memory full: wait for a retirement
            self.max_used = max(self.max_used, self.used)
            slot = self.free_slots.pop(0)
            now = self.clock()
            for j in batch:
                j.launched = now
            handle = self.ex.launch(batch, slot)
            self.in_flight.append((slot, handle, batch))
            self.batch_sizes.append(len(batch))
            launched += 1
        return launched

    def step(self) -> bool:
        """One scheduling pass; returns True if anything changed."""
        return bool(self._retire() + self._admit_and_launch())

    def idle(self) -> bool:
        return not self.waiting and not self.in_flight

    def stats(self) -> Stats:
        lat = np.array([j.latency for j in self.done]) * 1e3
        t0 = min(j.arrival for j in self.done)
        t1 = max(j.finished for j in self.done)
        span = max(t1 - t0, 1e-12)
        n_rirs = sum(j.n_rirs for j in self.done)
        return Stats(len(self.done), n_rirs, span, n_rirs / span, len(self.done) / span,
                     float(np.percentile(lat, 50)), float(np.percentile(lat, 99)),
                     float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0, self.max_used)


def replay(scheduler: Scheduler, jobs: List[Job], sleep: Callable[[float], None] = time.sleep,
           poll_s: float = 2e-5) -> Stats:
    """Feed ``jobs`` (sorted by arrival, times relative to the start) into the
    scheduler at their arrival times and run until all are finished."""
    start = scheduler.clock()
    pending = deque(sorted(jobs, key=lambda j: j.arrival))
    for j in pending:
        j.arrival += start
    while pending or not scheduler.idle():
        now = scheduler.clock()
        while pending and pending[0].arrival <= now:
            scheduler.submit(pending.popleft())
        if not scheduler.step():
            nxt = pending[0].arrival - scheduler.clock() if pending else poll_s
            sleep(max(min(nxt, poll_s), 0.0))
    return scheduler.stats()


class GpuExecutor:
    """Runs each batch with ism_batch_prepare + ism_batch_run on the slot's stream.

    Outputs and workspaces are torch tensors allocated per batch (device
    resident); a batch's completion is a recorded stream event.
    """

    def __init__(self, n_slots: int, device: str = "cuda"):
        import torch

        from . import ism

        self.torch = torch
        self.ism = ism
        self.device = device
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]

    def footprint(self, job: Job) -> int:
        """Device bytes the job holds while in flight: its output and its
        share of the batch workspace (``ism_batch_workspace_size`` of the job
        alone; the tables of a group, padded per job here, take no more)."""
        out = job.n_rirs * job.room.n_samples * 4
        return out + self.ism.batch_workspace_size([(job.room, job.src.shape[0], job.rcv.shape[0])])

    def launch(self, jobs: List[Job], slot: int):
        torch = self.torch
        st = self.streams[slot]
        with torch.cuda.stream(st):
            sim = self.ism.BatchSimulator([(j.room, j.src, j.rcv) for j in jobs], device=self.device, check=False,
                                          stream=st)
            sim.run(stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        return (sim, ev)

    def done(self, handle) -> bool:
        return handle[1].query()

    def finish(self, handle, jobs: List[Job]) -> None:
        sim, _ = handle
        for j, o in zip(jobs, sim.outs):
            j.out = o
