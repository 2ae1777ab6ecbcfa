"""Continuous-batching server for phase-field solves.

Requests (a domain shape, a precision, a parameter set, a Voronoi seed and a
number of steps) arrive over time.  The server keeps every admitted domain's
fields resident in device memory, admits queued requests whenever a slot and
enough of the memory budget are free, and advances all admitted domains of
one precision together: each round replays the captured pack step
(prologue + phi-sweep + mu-sweep over all members, one launch per kernel)
`round_steps` times.  The FP32 and FP64 packs run on two streams, so their
work overlaps on the device.  Finished domains leave at round boundaries,
their diagnostics (and optionally fields) are read back and their memory is
freed; newly admitted domains join at the next round.

The scheduler is written against a small backend interface so that its
admission and bookkeeping logic can be exercised without a GPU
(``SimBackend``); ``GpuBackend`` is the production backend over the C ABI.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque
from typing import Callable

import numpy as np


@dataclasses.dataclass
class Request:
    id: int
    arrival: float  # seconds after the start of the run
    shape: tuple    # (nz, ny, nx)
    prec: str       # "fp32" | "fp64"
    steps: int
    params: dict
    seed: int
    nseeds: int
    solid_height: int
    keep_fields: bool = False
    host_state: tuple | None = None  # (phi, mu) instead of a Voronoi state
    cancel_at: float | None = None   # withdrawn at this time (seconds after the start)


@dataclasses.dataclass
class Result:
    id: int
    arrival: float
    admitted: float
    finished: float
    cells: int
    steps: int
    prec: str
    ok: bool
    error: str = ""
    diag: dict | None = None
    fields: tuple | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def request_from_trace(d: dict, keep_fields: bool = False) -> Request:
    return Request(id=d["id"], arrival=d["arrival"], shape=tuple(d["shape"]), prec=d["prec"],
                   steps=d["steps"], params=d["params"], seed=d["seed"], nseeds=d["nseeds"],
                   solid_height=d["solid_height"], keep_fields=keep_fields)


# ------------------------------------------------------------------ backends

class GpuBackend:
    """Domains and packs through the C ABI; memory lent by torch."""

    def __init__(self, max_domains: int = 256):
        import torch

        import paper_1506_01684_amd as pf

        self.torch = torch
        self.pf = pf
        self.streams = {"fp32": torch.cuda.Stream(), "fp64": torch.cuda.Stream()}
        self.packs = {p: pf.Pack(p, stream=self.streams[p], max_domains=max_domains)
                      for p in ("fp32", "fp64")}
        self.handles = {}

    def required_bytes(self, r: Request) -> int:
        return self.pf.required_bytes(r.shape, r.prec)

    def open(self, r: Request):
        torch = self.torch
        nbytes = self.required_bytes(r)
        buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        dom = self.pf.Domain(r.shape, r.prec, buffer=buf, stream=self.streams[r.prec])
        dom.set_params(r.params)
        if r.host_state is not None:
            dom.init_host(*r.host_state)
        else:
            dom.init_voronoi(r.seed, r.nseeds, r.solid_height)
        self.packs[r.prec].add(dom, r.steps)
        self.handles[r.id] = (dom, buf)

    def step(self, prec: str, rounds: int):
        """Enqueue `rounds` pack steps (asynchronous)."""
        if self.packs[prec].members and rounds > 0:
            self.packs[prec].step(rounds)

    def close(self, r: Request) -> tuple[dict | None, tuple | None, str]:
        dom, buf = self.handles.pop(r.id)
        pk = self.packs[r.prec]
        left = pk.remaining(dom)  # synchronises the pack's stream
        if left != 0:
            raise RuntimeError(f"request {r.id}: device reports {left} steps left")
        pk.remove(dom)
        err = ""
        diag = None
        fields = None
        try:
            diag = dom.diagnostics(raise_nonfinite=False)
            if diag["nonfinite"] > 0:
                err = f"{diag['nonfinite']} non-finite cells"
            if r.keep_fields:
                fields = dom.read()
        finally:
            dom.close()
            del buf
        return diag, fields, err

    def cancel(self, r: Request):
        """Drop an admitted request before it finishes: it leaves its pack
        at this round boundary and its memory is freed."""
        dom, buf = self.handles.pop(r.id)
        self.packs[r.prec].remove(dom)
        dom.close()
        del buf

    def shutdown(self):
        for pk in self.packs.values():
            pk.close()


class SimBackend:
    """CPU stand-in: a device that advances `rate` lattice updates per
    second of a virtual clock.  Used to test the scheduler without a GPU."""

    def __init__(self, clock: "VirtualClock", rate: float = 2e10, bytes_per_cell: int = 100):
        self.clock = clock
        self.rate = rate
        self.bpc = bytes_per_cell
        self.left = {}
        self.cells = {}
        self.prec_of = {}
        self.opened = []

    def required_bytes(self, r: Request) -> int:
        nz, ny, nx = r.shape
        return nz * ny * nx * self.bpc * (2 if r.prec == "fp64" else 1)

    def open(self, r: Request):
        self.left[r.id] = r.steps
        nz, ny, nx = r.shape
        self.cells[r.id] = nz * ny * nx
        self.prec_of[r.id] = r.prec
        self.opened.append(r.id)

    def step(self, prec: str, rounds: int):
        ids = [i for i, p in self.prec_of.items() if p == prec and self.left[i] > 0]
        lups = sum(self.cells[i] * min(rounds, self.left[i]) for i in ids)
        for i in ids:
            self.left[i] = max(0, self.left[i] - rounds)
        self.clock.advance(lups / self.rate)

    def close(self, r: Request):
        del self.left[r.id], self.cells[r.id], self.prec_of[r.id]
        return {"nonfinite": 0}, None, ""

    def cancel(self, r: Request):
        del self.left[r.id], self.cells[r.id], self.prec_of[r.id]

    def shutdown(self):
        pass


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self) -> float:
        return self.t

    def advance(self, dt: float):
        self.t += dt

    def sleep(self, dt: float):
        self.t += max(dt, 0.0)


# ------------------------------------------------------------------ server

class Server:
    """Admission + continuous batching over a backend.

    budget_bytes: device memory the admitted domains may hold together.
    max_slots: admitted domains at most.
    round_steps: steps each pack advances between scheduling decisions.
    backfill: admit later requests that fit while the queue head does not.
    policy: "fifo" admits in arrival order; "sjf" admits the request with
        the least expected service time minus time already waited (shortest
        job first with aging, so that long jobs are not starved).
    target_cells: with a value, a pack admits a request only while its
        members hold fewer cells than this (one request is always admitted
        into an empty pack): beyond the cells that fill the device, more
        members only stretch every member's latency.
    rate: assumed throughput (cells x steps per second) for the "sjf"
        service-time estimate; FP64 work counts twice.
    """

    def __init__(self, backend, budget_bytes: float = 200e9, max_slots: int = 64,
                 round_steps: int = 25, backfill: bool = True,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep,
                 policy: str = "fifo", target_cells: float | None = None,
                 rate: float = 2e10, log: Callable[[str], None] | None = None):
        if policy not in ("fifo", "sjf"):
            raise ValueError(f"unknown policy {policy!r}")
        self.b = backend
        self.budget = budget_bytes
        self.max_slots = max_slots
        self.round_steps = round_steps
        self.backfill = backfill
        self.clock = clock
        self.sleep = sleep
        self.policy = policy
        self.target_cells = target_cells
        self.rate = rate
        self.log = log
        self.events: list[tuple] = []

    def _service(self, r: Request) -> float:
        return float(np.prod(r.shape)) * r.steps * (2.0 if r.prec == "fp64" else 1.0) / self.rate

    def run(self, requests: list[Request]) -> list[Result]:
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.id)))
        queue: deque[Request] = deque()
        # id -> [request, admitted time, bytes, steps left]
        active: dict[int, list] = {}
        used = 0
        results: list[Result] = []
        for r in requests:
            if self.b.required_bytes(r) > self.budget:
                raise ValueError(f"request {r.id} needs more than the whole budget")
        t0 = self.clock()
        while pending or queue or active:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # withdrawn requests: queued ones leave the queue, admitted ones
            # leave their pack at this round boundary; others are unaffected
            for r in [q for q in queue if q.cancel_at is not None and q.cancel_at <= now]:
                queue.remove(r)
                results.append(Result(r.id, r.arrival, now, now, int(np.prod(r.shape)), r.steps,
                                      r.prec, False, "cancelled"))
            for i in [i for i, a in active.items()
                      if a[0].cancel_at is not None and a[0].cancel_at <= now]:
                r, adm, need, left = active.pop(i)
                try:
                    self.b.cancel(r)
                    err = f"cancelled with {left} steps left"
                except Exception as e:
                    err = f"cancel failed: {e}"
                used -= need
                results.append(Result(r.id, r.arrival, adm, now, int(np.prod(r.shape)),
                                      r.steps - left, r.prec, False, err))
                self.events.append(("cancel", r.id, now, used))
            # admission in arrival order (or, with "sjf", by expected service
            # time minus time waited); with backfill, later requests that fit
            # may pass a head request that does not
            order = list(queue)
            if self.policy == "sjf":
                order.sort(key=lambda q: (self._service(q) - (now - q.arrival), q.arrival, q.id))
            cells = {"fp32": 0, "fp64": 0}
            for a in active.values():
                cells[a[0].prec] += int(np.prod(a[0].shape))
            for r in order:
                need = self.b.required_bytes(r)
                c = int(np.prod(r.shape))
                room = (self.target_cells is None or cells[r.prec] == 0
                        or cells[r.prec] + c <= self.target_cells)
                if len(active) < self.max_slots and used + need <= self.budget and room:
                    queue.remove(r)
                    try:
                        self.b.open(r)
                    except Exception as e:  # failure isolation: only this request fails
                        results.append(Result(r.id, r.arrival, now, self.clock() - t0,
                                              int(np.prod(r.shape)), r.steps, r.prec, False,
                                              f"admission failed: {e}"))
                        continue
                    active[r.id] = [r, now, need, r.steps]
                    used += need
                    cells[r.prec] += c
                    self.events.append(("admit", r.id, now, used))
                elif not self.backfill:
                    break
            if not active:
                if pending:
                    self.sleep(max(0.0, pending[0].arrival - (self.clock() - t0)))
                continue
            # one round: each pack advances by at most round_steps steps (no
            # more than its longest member still needs); the two packs run on
            # their own streams and overlap
            rounds = {}
            for prec in ("fp32", "fp64"):
                left = [a[3] for a in active.values() if a[0].prec == prec]
                rounds[prec] = min(self.round_steps, max(left)) if left else 0
                self.b.step(prec, rounds[prec])
            for i in list(active):
                a = active[i]
                a[3] = max(0, a[3] - rounds[a[0].prec])
                if a[3] > 0:
                    continue
                r, adm, need, _ = active.pop(i)
                try:
                    diag, fields, err = self.b.close(r)
                except Exception as e:
                    diag, fields, err = None, None, f"close failed: {e}"
                used -= need
                fin = self.clock() - t0
                results.append(Result(r.id, r.arrival, adm, fin, int(np.prod(r.shape)),
                                      r.steps, r.prec, not err, err, diag, fields))
                self.events.append(("finish", r.id, fin, used))
                if self.log:
                    self.log(f"[serve] t={fin:.1f}s finished request {r.id} "
                             f"({len(results)}/{len(requests)}, latency {fin - r.arrival:.2f}s)")
        return sorted(results, key=lambda x: x.id)


def run_serial_gpu(requests: list[Request], clock: Callable[[], float] = time.perf_counter,
                   sleep: Callable[[float], None] = time.sleep) -> list[Result]:
    """Baseline: first come, first served, one domain at a time, each stepped
    by plain single-domain launches (pf_step)."""
    import paper_1506_01684_amd as pf

    out = []
    t0 = clock()
    for r in sorted(requests, key=lambda q: (q.arrival, q.id)):
        now = clock() - t0
        if now < r.arrival:
            sleep(r.arrival - now)
        start = clock() - t0
        d = pf.Domain(r.shape, r.prec)
        try:
            d.set_params(r.params)
            if r.host_state is not None:
                d.init_host(*r.host_state)
            else:
                d.init_voronoi(r.seed, r.nseeds, r.solid_height)
            d.step(r.steps)
            d.sync()
            diag = d.diagnostics(raise_nonfinite=False)
            fields = d.read() if r.keep_fields else None
            err = f"{diag['nonfinite']} non-finite cells" if diag["nonfinite"] else ""
        finally:
            d.close()
        out.append(Result(r.id, r.arrival, start, clock() - t0, int(np.prod(r.shape)), r.steps,
                          r.prec, not err, err, diag, fields))
    return out


def summarize(results: list[Result], makespan: float | None = None) -> dict:
    ok = [r for r in results if r.ok]
    lat = np.array([r.latency for r in ok]) if ok else np.array([math.nan])
    lups = sum(r.cells * r.steps for r in ok)
    span = makespan if makespan is not None else max((r.finished for r in results), default=0.0)
    return {
        "requests": len(results), "failed": len(results) - len(ok),
        "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(np.mean(lat)), "makespan_s": span,
        "throughput_mlups": lups / span / 1e6 if span > 0 else math.nan,
    }
