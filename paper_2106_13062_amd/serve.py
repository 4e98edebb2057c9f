"""Serving loop for fast count sketch requests on one device.

Requests of mixed kinds arrive over time:
  * ``contract``  T(I, u, v) against a sketch kept resident on the device
                  (Section 4.1: median over D sketches of the free-mode
                  contraction),
  * ``cp``        a CP sketch build (Section 3.1),
  * ``coo``       a COO sketch of a sparse tensor (Section 3.2).

The ``Scheduler`` (pure host logic) keeps the waiting requests, admits them
while the device-memory footprint of everything in flight stays under a cap,
and forms launch groups: waiting ``contract`` requests against the same
resident sketch are merged into one multi-pair launch (continuous batching:
whatever arrived while the device was busy goes out together), builds go out
one per launch.  The ``Server`` owns the device side: a cache of bound plans
per (seed, shape, hash lengths, D, L) so hash tables stay resident (bounded,
least recently used unpinned plans go first), the
resident sketch spectra, several streams of default priority on which
launch groups overlap, and completion events from which latency is taken
(arrival on the host clock to the first host poll that sees the group's
event complete).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any

import numpy as np
import torch

from . import _lib as C
from .fcs import Plan


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                    # "contract", "cp" or "coo"
    arrival: float               # seconds on the driver's clock
    key: Any = None              # contract: resident sketch name; cp/coo: input name
    index: int = 0               # contract: vector pair index in the bank
    footprint: int = 0           # device bytes while in flight
    sketches: int = 0            # sketches the request builds
    done: float | None = None    # completion time on the driver's clock
    result: Any = None           # (tensor, row) or tensor


class AdmissionError(C.FcsError):
    """A request whose footprint alone exceeds the admission cap (status
    FCS_EADMIT)."""

    def __init__(self, message: str):
        super().__init__(C.FCS_EADMIT, message)


class Scheduler:
    """Admission by device-memory footprint and launch grouping (no device
    calls, so it is testable on the host)."""

    def __init__(self, cap_bytes: float, max_group: int = 256, max_inflight: int = 8):
        self.cap = float(cap_bytes)
        self.max_group = int(max_group)
        self.max_inflight = int(max_inflight)
        self.waiting: collections.deque[Request] = collections.deque()
        self.inflight_bytes = 0
        self.inflight_groups = 0
        self.resident_bytes = 0

    def submit(self, req: Request):
        if req.footprint + self.resident_bytes > self.cap:
            raise AdmissionError(f"request {req.rid} needs {req.footprint} bytes, more than the cap allows")
        self.waiting.append(req)

    def fits(self, nbytes: int) -> bool:
        return self.resident_bytes + self.inflight_bytes + nbytes <= self.cap

    def next_groups(self, window: int = 1024):
        """Launch groups that may start now, oldest request first.  A group
        is admitted only if its whole footprint fits; requests behind a
        request that does not fit wait (no overtaking).  Contraction
        requests against the head's resident sketch are gathered from the
        first `window` waiting requests."""
        groups = []
        while self.waiting and self.inflight_groups + len(groups) < self.max_inflight:
            head = self.waiting[0]
            if head.kind == "contract":
                scanned, members, nbytes = [], [], 0
                full = False
                while self.waiting and len(scanned) < window:
                    r = self.waiting.popleft()
                    if (not full and r.kind == "contract" and r.key == head.key
                            and len(members) < self.max_group and self.fits(nbytes + r.footprint)):
                        members.append(r)
                        nbytes += r.footprint
                    else:
                        if r.kind == "contract" and r.key == head.key:
                            full = True      # keep arrival order among the rest
                        scanned.append(r)
                self.waiting.extendleft(reversed(scanned))
                if not members:
                    break
            else:
                if not self.fits(head.footprint):
                    break
                members, nbytes = [self.waiting.popleft()], head.footprint
            self.inflight_bytes += nbytes
            groups.append((members, nbytes))
        self.inflight_groups += len(groups)
        return groups

    def release(self, nbytes: int):
        self.inflight_bytes -= nbytes
        self.inflight_groups -= 1


class PlanCache:
    """Bound plans by key (seed, mode sizes, hash lengths, D, L), so that
    hash tables stay resident between requests.  A plan that a resident
    sketch or a staged input uses is pinned; when the cached table bytes
    exceed `limit_bytes`, unpinned plans go out least recently used first,
    and their bytes leave the scheduler's resident total.  `make(key)` builds
    a plan; `nbytes(plan)` gives its device bytes; `close(plan)` releases it
    (no device calls here, so the policy is testable on the host)."""

    def __init__(self, sched: Scheduler, limit_bytes: float, make, nbytes, close=lambda p: None):
        self.sched = sched
        self.limit = float(limit_bytes)
        self.make, self.nbytes, self.close = make, nbytes, close
        self.plans: collections.OrderedDict = collections.OrderedDict()
        self.pins: collections.Counter = collections.Counter()
        self.bytes = 0

    def get(self, key):
        p = self.plans.get(key)
        if p is not None:
            self.plans.move_to_end(key)
            return p
        p = self.make(key)
        nb = int(self.nbytes(p))
        self.plans[key] = p
        self.bytes += nb
        self.sched.resident_bytes += nb
        self._evict(keep=key)
        return p

    def pin(self, key):
        self.pins[key] += 1

    def unpin(self, key):
        self.pins[key] -= 1
        if self.pins[key] <= 0:
            del self.pins[key]
        self._evict(keep=None)

    def _evict(self, keep):
        for k in list(self.plans):
            if self.bytes <= self.limit:
                break
            if k == keep or self.pins.get(k, 0) > 0:
                continue
            p = self.plans.pop(k)
            nb = int(self.nbytes(p))
            self.bytes -= nb
            self.sched.resident_bytes -= nb
            self.close(p)


def _plan_key(I, J, D, seed, L=0):
    return (int(seed) & ((1 << 64) - 1), tuple(int(i) for i in I), tuple(int(j) for j in J), int(D), int(L))


class Server:
    """Device side of the serving loop."""

    def __init__(self, device=None, streams: int = 4, cap_bytes: float = 200e9, max_group: int = 256,
                 max_inflight: int = 8, plan_cache_bytes: float = 16e9):
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.sched = Scheduler(cap_bytes, max_group, max_inflight)
        self.plans = PlanCache(self.sched, plan_cache_bytes,
                               make=lambda k: Plan(k[1], k[2], k[3], k[0], L=k[4], device=self.device),
                               nbytes=lambda p: p.tables.numel(), close=lambda p: p.close())
        self.resident: dict = {}       # name -> (plan, spec, bank_u, bank_v)
        self.inputs: dict = {}         # name -> ("cp", plan, U) or ("coo", plan, idx, val)
        self.inflight: list = []       # (event, members, nbytes)
        self.rr = 0

    # ------------------------------------------------------------ resources
    def plan(self, I, J, D, seed, L=0) -> Plan:
        key = _plan_key(I, J, D, seed, L)
        p = self.plans.get(key)
        p.cache_key = key
        return p

    @staticmethod
    def _bytes(tensors):
        flat = [x for t in tensors for x in (t if isinstance(t, (list, tuple)) else [t])]
        return sum(t.numel() * t.element_size() for t in flat)

    def add_resident_sketch(self, name, plan: Plan, spec: torch.Tensor, bank_u: torch.Tensor,
                            bank_v: torch.Tensor):
        """A sketch spectrum kept on the device with a bank of (u, v) pairs
        that contraction requests refer to by index (pins its plan)."""
        self.resident[name] = (plan, spec, bank_u, bank_v)
        self.sched.resident_bytes += self._bytes((spec, bank_u, bank_v))
        if getattr(plan, "cache_key", None) is not None:
            self.plans.pin(plan.cache_key)

    def remove_resident_sketch(self, name):
        plan, spec, bank_u, bank_v = self.resident.pop(name)
        self.sched.resident_bytes -= self._bytes((spec, bank_u, bank_v))
        if getattr(plan, "cache_key", None) is not None:
            self.plans.unpin(plan.cache_key)

    def add_input(self, name, kind, plan: Plan, *tensors):
        """Pre-staged request input: kind "cp" with one argument, the list
        of N factor tensors (R x I_n); kind "coo" with (idx, val) (pins its
        plan)."""
        self.inputs[name] = (kind, plan, *tensors)
        self.sched.resident_bytes += self._bytes(tensors)
        if getattr(plan, "cache_key", None) is not None:
            self.plans.pin(plan.cache_key)

    def remove_input(self, name):
        kind, plan, *tensors = self.inputs.pop(name)
        self.sched.resident_bytes -= self._bytes(tensors)
        if getattr(plan, "cache_key", None) is not None:
            self.plans.unpin(plan.cache_key)

    def footprint(self, req: Request) -> int:
        """Device bytes a request holds while in flight (outputs, gathered
        vectors and workspace)."""
        if req.kind == "contract":
            plan, _, bu, _ = self.resident[req.key]
            I0 = plan.I[0]
            ws = int(plan.lib.fcs_workspace_bytes(plan.handle, C.OP_FREE_MODE, 0, 1))
            return I0 * 8 + (plan.I[1] + plan.I[2]) * 4 + ws
        kind, plan, *t = self.inputs[req.key]
        out = plan.D * plan.Jt * 4
        if kind == "cp":
            R = int(t[0][0].shape[0])
            return out + int(plan.lib.fcs_workspace_bytes(plan.handle, C.OP_CP, R, 0))
        return out + int(plan.lib.fcs_workspace_bytes(plan.handle, C.OP_COO, 0, 0))

    def make_request(self, rid, kind, arrival, key, index=0) -> Request:
        r = Request(rid, kind, arrival, key, index)
        r.footprint = self.footprint(r)
        if kind != "contract":
            r.sketches = self.inputs[key][1].D
        return r

    # ------------------------------------------------------------ execution
    def _launch(self, members, stream):
        head = members[0]
        with torch.cuda.stream(stream):
            if head.kind == "contract":
                plan, spec, bu, bv = self.resident[head.key]
                idx = torch.tensor([r.index for r in members], dtype=torch.int64).to(self.device,
                                                                                      non_blocking=True)
                u = bu.index_select(0, idx)
                v = bv.index_select(0, idx)
                out = plan.contract_free_mode(spec, 0, [None, u, v], stream=stream)
                for k, r in enumerate(members):
                    r.result = (out, k)
            else:
                kind, plan, *t = self.inputs[head.key]
                if kind == "cp":
                    y, _ = plan.sketch_cp(t[0], stream=stream)
                else:
                    y = plan.sketch_coo(t[0], t[1], stream=stream)
                head.result = y
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev

    def submit(self, req: Request):
        self.sched.submit(req)

    def poll(self, now: float):
        """Retire finished groups (stamping `now`), then launch what fits."""
        still = []
        for ev, members, nbytes in self.inflight:
            if ev.query():
                for r in members:
                    r.done = now
                self.sched.release(nbytes)
            else:
                still.append((ev, members, nbytes))
        self.inflight = still
        for members, nbytes in self.sched.next_groups():
            stream = self.streams[self.rr % len(self.streams)]
            self.rr += 1
            ev = self._launch(members, stream)
            self.inflight.append((ev, members, nbytes))

    def idle(self) -> bool:
        return not self.inflight and not self.sched.waiting

    def run(self, requests, clock=time.perf_counter, timeout: float = 60.0):
        """Replay requests at their arrival times (seconds from the start)
        and serve them; returns the wall time from the first arrival to the
        last completion."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = clock()
        i = 0
        while i < len(reqs) or not self.idle():
            now = clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                self.submit(reqs[i])
                i += 1
            self.poll(now)
            if now > timeout:
                raise TimeoutError("serving loop did not drain in time")
        return clock() - t0


def latency_stats(requests):
    lat = np.array([r.done - r.arrival for r in requests if r.done is not None])
    if lat.size == 0:
        return {}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "served": int(lat.size)}


def run_alone(server: Server, req: Request):
    """The same request on its own: one launch, waited for (the plain
    one-request-at-a-time path)."""
    ev = server._launch([req], server.streams[0])
    ev.synchronize()
    return req.result
