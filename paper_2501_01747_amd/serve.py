"""Continuous-batching request server over the batched ADG engine (adg_batch_*).

Requests (one ADG solve each: a problem, its initial state and a number of time
steps) arrive over time.  The server keeps every admitted instance's states and
delay history resident in one device workspace and advances all of them
together, a few time steps per scheduling round:

  * admission: arrived requests are admitted in arrival order as long as the
    batch has a free slot and a free workspace region of the request's
    footprint (adg_batch_add refuses with ADG_ERR_NOMEM otherwise); a request
    that does not fit waits, and so does every later one (no overtaking);
  * each round enqueues min(chunk, fewest remaining steps of any admitted
    request) steps for the whole batch; an instance stops by itself on the
    device when it reaches its own step count;
  * after the round the server polls the step counters, retires finished
    requests (result copied out, slot and region released) and admits again.

Latency = completion - arrival, queueing included.  The scheduler is host
logic only; every step of every solve runs in the library's kernels.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    case: dict
    w0: np.ndarray
    steps: int
    arrival: float = 0.0          # seconds after the start of the run


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    completed: float
    steps: int
    dof: int
    ok: bool
    state: np.ndarray | None = None

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


def request_dof(case: dict) -> int:
    d = case["disc"]
    return d["n_elem"] * (d["order_p"] + 1) * (3 + case["physics"]["n_species"])


class Server:
    """`batch` is an adg.Batch (or any object with its add/remove/step/poll/state
    interface); `clock` returns seconds; `sleep` waits."""

    def __init__(self, batch, chunk: int = 10, keep_states: bool = False, clock=time.perf_counter,
                 sleep=time.sleep, nomem_code: int = -2, graph_steps: int = 0):
        self.batch = batch
        # graph_steps > 0: the batch replays captured graphs of that many steps (captured again
        # only when the composition changes: most rounds keep the previous round's), so a round
        # costs a few graph launches instead of every launch and stream join of its steps
        if graph_steps > 0:
            batch.set_graph(graph_steps)
        self.chunk = int(chunk)
        self.keep_states = keep_states
        self.clock = clock
        self.sleep = sleep
        self.nomem_code = nomem_code
        self.rounds = 0
        self.max_active = 0
        # wall seconds of the loop's parts: enqueueing steps, waiting for them (poll), copying
        # finished states out and releasing them, admitting (placement and upload)
        self.time_in = {"enqueue": 0.0, "wait": 0.0, "retire": 0.0, "admit": 0.0}

    def run(self, requests: list[Request]) -> list[Result]:
        arrivals = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting: collections.deque[Request] = collections.deque()
        active: dict[int, list] = {}     # slot -> [request, admission time, steps enqueued]
        done: list[Result] = []
        t0 = self.clock()
        now = 0.0
        while arrivals or waiting or active:
            now = self.clock() - t0
            while arrivals and arrivals[0].arrival <= now:
                waiting.append(arrivals.popleft())
            t_adm0 = self.clock()
            while waiting:
                r = waiting[0]
                try:
                    slot = self.batch.add(r.case, r.w0, n_steps=r.steps)
                except Exception as e:      # AdgError; NOMEM means "wait for space"
                    if getattr(e, "code", None) == self.nomem_code and active:
                        break
                    waiting.popleft()
                    t = self.clock() - t0
                    done.append(Result(r.rid, r.arrival, t, t, 0, request_dof(r.case), False))
                    continue
                waiting.popleft()
                active[slot] = [r, self.clock() - t0, 0]
            self.time_in["admit"] += self.clock() - t_adm0
            self.max_active = max(self.max_active, len(active))
            if not active:
                if arrivals:
                    self.sleep(max(0.0, arrivals[0].arrival - (self.clock() - t0)))
                continue
            n = max(1, min(self.chunk, min(a[0].steps - a[2] for a in active.values())))
            t1 = self.clock()
            self.batch.step(n)
            t2 = self.clock()
            self.rounds += 1
            for a in active.values():
                a[2] = min(a[0].steps, a[2] + n)
            steps_now, errs = self.batch.poll()
            t3 = self.clock()
            self.time_in["enqueue"] += t2 - t1
            self.time_in["wait"] += t3 - t2
            t_done = t3 - t0
            for slot in list(active):
                r, t_adm, _ = active[slot]
                if errs[slot] or steps_now[slot] >= r.steps:
                    state = None
                    ok = not errs[slot]
                    if self.keep_states and ok:
                        state = self.batch.state(slot)
                    self.batch.remove(slot)
                    del active[slot]
                    done.append(Result(r.rid, r.arrival, t_adm, t_done, int(steps_now[slot]),
                                       request_dof(r.case), ok, state))
            self.time_in["retire"] += self.clock() - t3
        return sorted(done, key=lambda x: x.rid)


def summarize(results: list[Result]) -> dict:
    """Latency percentiles and aggregate throughput of a served stream."""
    ok = [r for r in results if r.ok]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    span = max(r.completed for r in results) - min(r.arrival for r in results) if results else 0.0
    work = sum(r.dof * 3 * r.steps for r in ok)
    return {
        "requests": len(results), "completed_ok": len(ok), "failed": len(results) - len(ok),
        "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()),
        "mean_queue_s": float(np.mean([r.admitted - r.arrival for r in ok])) if ok else 0.0,
        "makespan_s": span, "requests_per_s": len(ok) / span if span > 0 else 0.0,
        "dof_updates_per_s": work / span if span > 0 else 0.0,
    }
