"""Continuous-batching request loop over the batched step of libsol.

Requests (cases with an arrival time and a step count) are admitted in
arrival order while their device footprint (sol_footprint_bytes) fits the
memory budget and the batch has a free slot.  A request whose footprint
exceeds the whole budget is refused on its own (listed under "rejected",
with the reason) and the rest of the stream is served.  Admitted cases stay on the
device; every tick advances all admitted cases together in one batched
launch sequence per step (sol_batch_step), until the next event: a case
finishing its steps, or an arrival that a free slot could take (judged
from the measured step time).  A case that has done its steps
leaves the batch, its fields are read back, its memory is released and the
next waiting request can take the slot, while the others keep running.
Latency = time from arrival until the fields are on the host.

Every step runs in the library's kernels; this module only schedules.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from .binding import Batch, Case, sol_footprint_bytes


@dataclass
class Request:
    case: dict
    steps: int
    arrival: float                    # seconds after the start of the run
    rid: int = 0
    cells: int = 0
    footprint: int = 0
    admitted: float = -1.0
    finished: float = -1.0
    result: dict | None = None
    steps_done: int = 0
    error: str | None = None          # set when the request is refused
    handle: Case | None = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    def __init__(self, device=None, hbm_budget_bytes: int = 270 * 2 ** 30, max_active: int = 64,
                 graph: bool = False, keep_results: bool = True, multi_step: bool = True,
                 backfill: bool = True, max_wait_s: float = 2.0):
        self.device = device
        self.backfill = backfill
        self.max_wait_s = float(max_wait_s)
        self.budget = int(hbm_budget_bytes)
        self.max_active = int(max_active)
        self.graph = graph
        self.keep_results = keep_results
        # a tick advances the batch until its next event (a request finishes,
        # or the next arrival could be admitted) instead of by one step
        self.multi_step = multi_step
        self.log = []                 # (time, event, request id)

    def run(self, requests, clock=time.perf_counter, sleep=time.sleep):
        pending = deque()
        rejected = []
        for r in sorted(requests, key=lambda r: r.arrival):
            g = r.case["grid"]
            r.cells = g["nx"] * g["ny"] * (g["nz"] if g["dim"] == 3 else 1)
            r.footprint = sol_footprint_bytes(r.case)
            if r.footprint > self.budget:
                # can never be admitted: refused on its own, the stream goes on
                r.error = f"needs {r.footprint} B of device memory, over the budget of {self.budget} B"
                rejected.append(r)
                self.log.append((r.arrival, "reject", r.rid))
            else:
                pending.append(r)
        waiting, active, done = deque(), [], []
        used = 0
        batch = None
        members = None
        t0 = clock()
        cell_steps = 0
        step_s = None                 # running estimate of one batched step (s)
        while pending or waiting or active:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admission in arrival order, by footprint and free slots; when
            # the oldest waiting request does not fit the memory left, later
            # ones that do fit may go ahead of it (backfill) until it has
            # waited max_wait_s, after which admission holds for it
            while waiting and len(active) < self.max_active:
                head = waiting[0]
                if used + head.footprint <= self.budget:
                    r = waiting.popleft()
                elif self.backfill and now - head.arrival < self.max_wait_s:
                    r = next((x for x in waiting if used + x.footprint <= self.budget), None)
                    if r is None:
                        break
                    waiting.remove(r)
                else:
                    break
                r.handle = Case(r.case, device=self.device)
                if self.graph:
                    r.handle.set_graph(True)
                r.admitted = clock() - t0
                used += r.footprint
                active.append(r)
                self.log.append((r.admitted, "admit", r.rid))
            if not active:
                if pending:
                    sleep(max(0.0, min(0.01, pending[0].arrival - (clock() - t0))))
                continue
            ids = [r.rid for r in active]
            if batch is None or members != ids:
                if batch is not None:
                    batch.close()
                batch = Batch([r.handle for r in active])
                members = ids
            k = 1
            if self.multi_step:
                k = min(r.steps - r.steps_done for r in active)
                # an arrival that could be admitted is not kept waiting past
                # its time by more than one step
                # (requests already waiting are held by the memory budget or
                # the slots, and wait for a finish either way)
                if pending and not waiting and len(active) < self.max_active:
                    ahead = pending[0].arrival - (clock() - t0)
                    k = min(k, max(1, int(ahead / step_s))) if step_s else 1
            ts = clock()
            batch.step([k] * len(active))
            dt = (clock() - ts) / k
            step_s = dt if step_s is None else 0.7 * step_s + 0.3 * dt
            for r in active:
                r.steps_done += k
                cell_steps += r.cells * k
            finished = [r for r in active if r.steps_done >= r.steps]
            if finished:
                batch.close()
                batch = None
                members = None
                for r in finished:
                    fields = r.handle.read_fields()
                    r.finished = clock() - t0
                    r.result = fields if self.keep_results else None
                    r.handle.close()
                    r.handle = None
                    used -= r.footprint
                    active.remove(r)
                    done.append(r)
                    self.log.append((r.finished, "finish", r.rid))
        if batch is not None:
            batch.close()
        wall = clock() - t0
        if not done:
            return dict(requests=0, rejected=rejected, wall_s=wall, cell_updates_per_s=0.0,
                        p50_latency_s=float("nan"), p99_latency_s=float("nan"), mean_latency_s=float("nan"),
                        offered_cell_updates_per_s=0.0, done=done)
        lat = np.array([r.latency for r in done])
        span = max(r.arrival for r in done) - min(r.arrival for r in done) if len(done) > 1 else 0.0
        offered = sum(r.cells * r.steps for r in done) / span if span > 0 else float("inf")
        return dict(
            requests=len(done), rejected=rejected, wall_s=wall,
            cell_updates_per_s=cell_steps / wall if wall > 0 else 0.0,
            p50_latency_s=float(np.percentile(lat, 50)), p99_latency_s=float(np.percentile(lat, 99)),
            mean_latency_s=float(lat.mean()), offered_cell_updates_per_s=offered,
            done=done,
        )
