"""Serving loop for many discharges (continuous batching).

Requests -- the parameters of one discharge each -- wait in a queue.  They are
admitted while the device memory their particle stores need stays within a
budget, advanced together one quantum at a time (``step_batch``: one launch
per kernel for every active discharge, all standing at the same phase of the
step sequence), and retired when their steady-state detector fires or they
reach their cycle limit; the memory they free admits the next requests.  The
quantum is the launch period of the step sequence (twice the least common
multiple of the sort and Coulomb intervals; it divides an rf cycle), so an
arrival waits at most one period for admission, and a discharge admitted at
a period boundary stands at the same phase as the running ones.

Steady state, as Sec. II defines the end of a run: the moments no longer
change when averaged over an rf cycle.  The detector watches the
cycle-averaged number of ions (O- and O2+) and declares steady state when its
relative change between cycle k and cycle k - window stays below tol in two
consecutive cycles.

The loop is plain host code around the library's C ABI; every discharge ends
exactly as it would if it ran alone (the batched launches are bit-identical
to single ones).
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque

import numpy as np

# device bytes per store slot: two particle buffers (cell, off, vx, vy, vz,
# id), the candidate list and the birth records, rounded up
BYTES_PER_SLOT = {"fp32": 96, "fp64": 160}
BYTES_FIXED = 8 << 20


@dataclasses.dataclass
class Request:
    rid: int
    workload: object            # pic_inputs.Workload (resolved)
    max_cycles: int = 1000
    window: int = 50
    tol: float = 0.01
    arrival: float | None = None


@dataclasses.dataclass
class Result:
    rid: int
    cycles: int
    steady: bool                # retired by the steady-state detector (else by the cycle limit)
    t_arrival: float
    t_admit: float
    t_done: float               # when the detector fired or the limit was reached
    ions: list                  # cycle-averaged ion count per completed cycle
    pushes: int = 0             # particle pushes of the discharge


class SteadyState:
    """Relative change of a per-cycle value against the value `window` cycles
    earlier, below `tol` in two consecutive cycles."""

    def __init__(self, window: int, tol: float):
        self.window = window
        self.tol = tol
        self.values: list[float] = []
        self.hits = 0

    def feed(self, x: float) -> bool:
        self.values.append(float(x))
        if len(self.values) <= self.window:
            return False
        ref = self.values[-1 - self.window]
        change = abs(self.values[-1] - ref) / max(abs(ref), 1e-300)
        self.hits = self.hits + 1 if change < self.tol else 0
        return self.hits >= 2


def launch_period(wl) -> int:
    """Steps after which the library's launch sequence repeats: twice the
    least common multiple of the sort and Coulomb intervals."""
    a = int(wl.sort_every)
    b = int(wl.coulomb_every) if wl.coulomb_every > 0 else 1
    return 2 * (a // math.gcd(a, b)) * b


def capacity(wl) -> list:
    """Store capacity per species the server gives a discharge."""
    return [4 * int(n) + (1 << 20) for n in wl.n_init]


def bytes_needed(wl, precision: str) -> int:
    return BYTES_PER_SLOT[precision] * sum(capacity(wl)) + BYTES_FIXED


def cycle_ions(m, wl) -> float:
    """Cycle-averaged number of ion macro particles from the moments'
    cycle-averaged densities (trapezoidal node volumes)."""
    dens = np.asarray(m["density"])
    n = dens.shape[1] - 1
    dx = wl.gap_m / n
    vol = np.full(n + 1, wl.area_m2 * dx)
    vol[0] *= 0.5
    vol[-1] *= 0.5
    return float((dens[1] * vol).sum() + (dens[2] * vol).sum()) / wl.weight


def percentile(values, q: float) -> float:
    return float(np.percentile(np.asarray(values, dtype=float), q)) if len(values) else float("nan")


class Server:
    """Continuous batching of discharges under a device-memory budget.

    backend(workload, sigma, threshold, loss, precision=..., capacity=...)
    builds a discharge (paper_0705_0495_amd.Discharge); step_batch(list, n)
    advances a list of them (paper_0705_0495_amd.step_batch).  Both are
    parameters so that the scheduling can be tested without a GPU."""

    def __init__(self, tables, budget_bytes: int, precision: str = "fp32", backend=None, step_batch=None,
                 clock=time.perf_counter):
        if backend is None or step_batch is None:
            from . import Discharge, step_batch as sb
            backend = backend or Discharge
            step_batch = step_batch or sb
        self.tables = tables
        self.budget = int(budget_bytes)
        self.precision = precision
        self.backend = backend
        self.step_batch = step_batch
        self.clock = clock
        self.queue: deque = deque()
        self.active: list = []          # [request, discharge, detector, t_admit, bytes, steps]
        self.results: list[Result] = []
        self.used = 0
        self.cycle_steps = None
        self.quantum = None
        self.period = None

    def submit(self, req: Request) -> None:
        wl = req.workload
        key = (wl.steps_per_period, wl.sort_every, wl.coulomb_every)
        if self.cycle_steps is None:
            q = launch_period(wl)
            if wl.steps_per_period % q != 0:
                raise ValueError("the launch period must divide an rf cycle")
            self.cycle_steps, self.quantum, self.period = wl.steps_per_period, q, key
        elif key != self.period:
            raise ValueError("requests of one server share steps per rf cycle, sort and Coulomb periods")
        if bytes_needed(wl, self.precision) > self.budget:
            raise ValueError(f"request {req.rid} needs more than the whole budget")
        if req.arrival is None:
            req.arrival = self.clock()
        if self.queue and req.arrival < self.queue[-1].arrival:
            raise ValueError("requests must be submitted in arrival order")
        self.queue.append(req)

    def _admit(self) -> None:
        while self.queue:
            req = self.queue[0]
            if req.arrival > self.clock():
                return  # not arrived yet (requests are kept in arrival order)
            need = bytes_needed(req.workload, self.precision)
            if self.used + need > self.budget:
                return
            self.queue.popleft()
            d = self.backend(req.workload, *self.tables, precision=self.precision, capacity=capacity(req.workload))
            self.used += need
            self.active.append([req, d, SteadyState(req.window, req.tol), self.clock(), need, 0])

    def step_quantum(self) -> list:
        """Admit what fits, advance every active discharge by one launch
        period, feed the detectors of those that completed an rf cycle,
        retire the finished ones; returns the results retired now."""
        self._admit()
        if not self.active:
            return []
        self.step_batch([a[1] for a in self.active], self.quantum)
        done, keep = [], []
        for a in self.active:
            a[5] += self.quantum
            req, d, det, t_admit, need, steps = a
            if steps % self.cycle_steps != 0:
                keep.append(a)
                continue
            m = d.moments()
            steady = det.feed(cycle_ions(m, req.workload))
            if steady or m["cycles"] >= req.max_cycles:
                done.append(Result(req.rid, int(m["cycles"]), steady, req.arrival, t_admit, self.clock(),
                                   list(det.values), int(m.get("particle_steps", 0))))
                d.close()
                self.used -= need
            else:
                keep.append(a)
        self.active = keep
        self.results.extend(done)
        return done

    def step_cycle(self) -> list:
        """Advance by whole launch periods until one rf cycle has passed."""
        done = []
        for _ in range(self.cycle_steps // self.quantum if self.quantum else 1):
            done += self.step_quantum()
        return done

    def run(self) -> list:
        """Serve until the queue and the active set are empty."""
        while self.queue or self.active:
            if not self.active and self.queue and self.queue[0].arrival > self.clock():
                time.sleep(min(1.0, self.queue[0].arrival - self.clock()))
                continue
            self.step_quantum()
            if not self.active and self.queue and self.queue[0].arrival <= self.clock():
                raise RuntimeError("a queued request cannot be admitted")
        return self.results

    def latency(self) -> dict:
        """Time from arrival to retirement over the served requests, and time
        from arrival to the periodic steady state over those whose detector
        fired."""
        t = [r.t_done - r.t_arrival for r in self.results]
        ss = [r.t_done - r.t_arrival for r in self.results if r.steady]
        return {"p50_s": percentile(t, 50), "p99_s": percentile(t, 99), "served": len(t),
                "steady": len(ss), "ss_p50_s": percentile(ss, 50), "ss_p99_s": percentile(ss, 99)}
