"""Continuous-batching propagation server for the symmetry-adapted HTC HEOM.

A request is one propagation: a problem (N, m, L, d, bath, eps, omega_c, g,
kappa), a tier-0 initial block, a time step, a horizon in RK4 steps and an
observable stride. The response is the observable trajectory on the host
(one row of HEOM_NOBS values every `obs_every` steps, Sec. V.D).

Device residency. Every admitted request keeps its state (16 B per unique
variable), its work vectors (32 B per variable plus a small control area),
its parameter block and its observable buffer in HBM until it completes.
Requests whose structure key (min(N, L+d+2), m, L, d) agrees share one
uploaded structure image; the unique-variable set is N-independent beyond
that key (Sec. V.C.4), so only the parameter block (pool size, g, bath,
loss) is per request. Images of keys no request uses stay cached while the
byte budget allows and are evicted least recently used first.

Continuous batching. Requests are split by size (unique variables) into
lanes; a lane is a heom_batch on its own stream whose in-flight requests
are stepped together, a chunk of RK4 steps per heom_batch_propagate call.
At a chunk boundary a lane retires completed requests (observables copied
to the host) and admits waiting ones into the freed slots and memory, so
requests that arrive while others run join without waiting for them. The
lanes' kernels run concurrently on the device; a short request advances at
its own lane's step rate rather than at that of the largest request in
flight. A chunk never runs a request past its horizon.

Admission is first come, first served against the byte budget: the first
waiting request that does not fit stops admission for all later ones (no
overtaking on memory, so large requests are not starved), while a request
whose lane has no free slot lets later requests of other lanes pass.

Each request's trajectory is computed by the same kernels in the same
order whatever else is in flight, so a result is bitwise the one the request
gets alone.

The scheduling decisions (lane choice, admission, chunk length, eviction)
are plain functions of host state and are tested without a device.
"""
from __future__ import annotations

import bisect
import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import heom

ALIGN = 256


def _round(n: int) -> int:
    return (int(n) + ALIGN - 1) // ALIGN * ALIGN


# --------------------------------------------------------------- requests

@dataclasses.dataclass
class Request:
    rid: int
    problem: object                    # workloads.Problem (or any object with its fields)
    horizon: int                       # RK4 steps
    dt: float
    obs_every: int = 100
    arrival: float = 0.0               # seconds after the start of the trace
    tier0: Optional[np.ndarray] = None # complex tier-0 block; None = all population in the photon


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    obs: np.ndarray                    # (horizon // obs_every + 1, HEOM_NOBS)
    n_var: int
    lane: int = -1
    finite: bool = True                # False if the state became NaN or infinite (heom_batch_status)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def structure_key(p) -> Tuple[int, int, int, int]:
    return (min(int(p.N), int(p.L) + int(p.d) + 2), int(p.m), int(p.L), int(p.d))


# --------------------------------------------------------------- pure scheduling rules

def lane_of(n_var: int, thresholds: Sequence[int]) -> int:
    """Lane index of a request with n_var unique variables: lane i holds
    thresholds[i-1] <= n_var < thresholds[i]."""
    return bisect.bisect_right(list(thresholds), int(n_var))


def request_bytes(n_var: int, work_bytes: int, params_bytes: int, horizon: int, obs_every: int) -> int:
    """Device bytes a request holds while in flight."""
    nobs = horizon // obs_every + 1 if obs_every > 0 else 1
    return (_round(16 * n_var) + _round(work_bytes) + _round(params_bytes)
            + _round(8 * heom.HEOM_NOBS * nobs))


def plan_admission(waiting: Sequence[Tuple[int, int, int, Optional[Tuple]]], free_slots: Dict[int, int],
                   free_bytes: int, resident: Dict[Tuple, int], evictable: Sequence[Tuple],
                   table_bytes: Dict[Tuple, int], budget: int) -> Tuple[List[int], List[Tuple]]:
    """Choose which waiting requests to admit now.

    waiting: (rid, lane, request bytes, structure key) in arrival order.
    free_slots: lane -> free slots. free_bytes: budget minus everything held.
    resident: structure keys with an uploaded image -> its bytes.
    evictable: resident keys no in-flight request uses, least recently used
    first. table_bytes: image bytes of every key that may be needed.
    Returns (admitted rids in order, keys to evict first).

    A request needing more than the whole budget is skipped here (the
    caller rejects it at submission). The first request that does not fit
    in memory, even after evicting unused images, stops admission."""
    slots = dict(free_slots)
    free = int(free_bytes)
    res = set(resident)
    ev = [k for k in evictable]
    evict: List[Tuple] = []
    admitted: List[int] = []
    for rid, lane, nbytes, key in waiting:
        if not any(v > 0 for v in slots.values()):
            break
        if slots.get(lane, 0) <= 0:
            continue
        need = nbytes + (0 if key is None or key in res else table_bytes[key])
        if need > budget:
            continue
        while need > free and ev:
            k = ev.pop(0)
            if k == key:
                continue
            evict.append(k)
            res.discard(k)
            free += resident[k]
        if need > free:
            break
        free -= need
        slots[lane] -= 1
        if key is not None and key not in res:
            res.add(key)
        if key in ev:
            ev.remove(key)              # now in use
        admitted.append(rid)
    return admitted, evict


def predicted_ms_per_step(measured_ms: Optional[float], measured_vars: int, vars_now: int) -> Optional[float]:
    """Step time of a lane's next chunk: the last measured step time, scaled
    up in proportion when the lane now holds more unique variables than it
    did then (a large request joining small ones would otherwise get a chunk
    sized for the small ones' step time, and hold back every later arrival of
    the lane for as long). Never scaled down: a shorter chunk only costs a
    little launch overhead."""
    if measured_ms is None or measured_ms <= 0:
        return None
    if measured_vars > 0 and vars_now > measured_vars:
        return measured_ms * (vars_now / measured_vars)
    return measured_ms


def hermitian_request_ok(problem, slot_matrix: Optional[np.ndarray], tol: float = 1e-12) -> bool:
    """A request may run under HEOM_HERMITIAN only if every ADO stays
    Hermitian: c_check_k = conj(c_k) for every channel (Eq.
    adjoint-preservation with real rates) and a Hermitian rho_S(0), given by
    its slot matrix (None: the photon start, which is Hermitian)."""
    cc = problem.c_check if problem.c_check is not None else [complex(z).conjugate() for z in problem.c]
    if not all(complex(b) == complex(a).conjugate() for a, b in zip(problem.c, cc)):
        return False
    if slot_matrix is None:
        return True
    R = np.asarray(slot_matrix)
    return bool(np.abs(R - R.conj().T).max() <= tol * max(1.0, float(np.abs(R).max())))


def chunk_steps(remaining: Sequence[int], ms_per_step: Optional[float], target_ms: float,
                first: int = 8, cap: int = 4096) -> int:
    """Steps of the next chunk of a lane: about target_ms of device time at
    the lane's (predicted) step time, never past the nearest horizon."""
    if not remaining:
        return 0
    lim = min(int(r) for r in remaining)
    if ms_per_step is None or ms_per_step <= 0:
        k = first
    else:
        k = int(target_ms / ms_per_step)
    return max(1, min(k, lim, cap))


# --------------------------------------------------------------- the server

@dataclasses.dataclass
class _Active:
    req: Request
    slot: int
    key: Tuple
    n_var: int
    nbytes: int
    admitted: float
    enqueued: int                       # steps launched so far
    bufs: tuple                         # (params, y, work, obs) tensors


class _Structure:
    def __init__(self, tables: "heom.Tables"):
        self.tables = tables
        info = tables.info()
        self.n_var = int(info["n_var"])
        self.table_bytes = _round(int(info["table_bytes"]))
        self.work_bytes = int(info["work_bytes_fp64"])
        self.params_bytes = int(tables.params_bytes())
        self.image = None               # device tensor while resident
        self.users = 0
        self.last_use = 0.0


class _Lane:
    def __init__(self, torch, index: int, capacity: int):
        self.index = index
        self.batch = heom.Batch(capacity)
        self.capacity = capacity
        self.stream = torch.cuda.Stream()
        self.free = list(range(capacity))[::-1]
        self.active: Dict[int, _Active] = {}
        self.inflight: collections.deque = collections.deque()   # (start event, end event, steps)
        self.ms_per_step: Optional[float] = None
        self.measured_vars = 0              # unique variables in flight when ms_per_step was measured
        self.dirty = False
        self.busy_ms = 0.0
        self.chunks = 0


class Server:
    """Continuous-batching server on one device.

    budget_bytes: HBM the server may hold (requests and table images).
    lanes: ascending unique-variable thresholds splitting requests into
    len(lanes)+1 lanes. capacity: slots per lane (an int or one per lane).
    precision: HEOM_FP64 or HEOM_FP32 (FP32 bulk with FP64 state), with
    HEOM_HERMITIAN OR-ed in when every request's ADOs are Hermitian (a
    Hermitian rho_S(0) and c_check = conj(c)); the structures then use
    compact tiles (heom_tuning.compact). One value, or one per lane (FP32
    bulk pays off on large states, whose steps are bound by memory traffic;
    small states are bound by launch latency, where FP64 steps are as fast or
    faster). The Hermitian flag must be the same in every lane.
    target_ms: device time per chunk; sets how long an arrival waits for
    its lane's next chunk boundary."""

    def __init__(self, torch, budget_bytes: int, lanes: Sequence[int] = (1 << 20,), capacity=256,
                 precision: int = heom.HEOM_FP64, target_ms: float = 25.0, clock: Callable[[], float] = None):
        self.torch = torch
        self.budget = int(budget_bytes)
        self.thresholds = list(lanes)
        caps = capacity if isinstance(capacity, (list, tuple)) else [capacity] * (len(self.thresholds) + 1)
        if len(caps) != len(self.thresholds) + 1:
            raise ValueError("one capacity per lane")
        self.lanes = [_Lane(torch, i, int(c)) for i, c in enumerate(caps)]
        precs = list(precision) if isinstance(precision, (list, tuple)) else [precision] * len(self.lanes)
        if len(precs) != len(self.lanes):
            raise ValueError("one precision per lane")
        if len({p & heom.HEOM_HERMITIAN for p in precs}) != 1:
            raise ValueError("the Hermitian flag must be the same in every lane")
        for lane, p in zip(self.lanes, precs):
            lane.precision = int(p)
        self.precision = int(precs[0])          # its Hermitian flag holds for every lane
        self.target_ms = float(target_ms)
        self.structs: Dict[Tuple, _Structure] = {}
        self.waiting: collections.deque = collections.deque()   # (request, lane, bytes, key)
        self.waiting_per_lane = [0] * len(self.lanes)
        self.results: List[Result] = []
        self.rejected: List[Tuple[int, str]] = []
        self.held_bytes = 0              # in-flight requests
        self.peak_bytes = 0              # most bytes held at once (requests + images)
        self.peak_in_flight = 0
        self.t0 = None
        self._clock = clock or time.perf_counter

    # ---- clock
    def now(self) -> float:
        return self._clock() - self.t0

    # ---- structures
    def prepare(self, problems) -> None:
        """Build host tables for the structure keys of these problems ahead of
        time (table construction happens before propagation, Sec. V.C.4)."""
        for p in problems:
            self._structure(p)

    def _structure(self, p) -> _Structure:
        key = structure_key(p)
        s = self.structs.get(key)
        if s is None:
            T = heom.Tables(p)
            if self.precision & heom.HEOM_HERMITIAN:
                T.set_tuning(compact=1)
            s = _Structure(T)
            self.structs[key] = s
        return s

    def _resident_bytes(self) -> int:
        return sum(s.table_bytes for s in self.structs.values() if s.image is not None)

    def free_bytes(self) -> int:
        return self.budget - self.held_bytes - self._resident_bytes()

    # ---- requests
    def footprint(self, req: Request) -> Tuple[int, _Structure]:
        s = self._structure(req.problem)
        return request_bytes(s.n_var, s.work_bytes, s.params_bytes, req.horizon, req.obs_every), s

    def submit(self, req: Request) -> bool:
        """Queue a request; False (and an entry in self.rejected) if it can
        never be served."""
        if req.horizon < 1 or req.obs_every < 0 or (req.obs_every > 0 and req.horizon % req.obs_every):
            self.rejected.append((req.rid, "horizon must be a positive multiple of obs_every"))
            return False
        nbytes, s = self.footprint(req)
        if self.precision & heom.HEOM_HERMITIAN:
            R = s.tables.tier0_expand(req.tier0) if req.tier0 is not None else None
            if not hermitian_request_ok(req.problem, R):
                self.rejected.append((req.rid, "HEOM_HERMITIAN needs c_check = conj(c) and a Hermitian rho_S(0)"))
                return False
        if nbytes + s.table_bytes > self.budget:
            self.rejected.append((req.rid, "footprint exceeds the byte budget"))
            return False
        lane = lane_of(s.n_var, self.thresholds)
        self.waiting.append((req, lane, nbytes, structure_key(req.problem)))
        self.waiting_per_lane[lane] += 1
        return True

    def in_flight(self) -> int:
        return sum(len(l.active) for l in self.lanes)

    # ---- lane mechanics
    def _admit(self, lane_idle: Sequence[bool]) -> None:
        free_slots = {l.index: (len(l.free) if lane_idle[l.index] else 0) for l in self.lanes}
        if not self.waiting or not any(free_slots[i] > 0 and self.waiting_per_lane[i] > 0 for i in free_slots):
            return
        waiting = ((w[0].rid, w[1], w[2], w[3]) for w in self.waiting)   # lazily: admission stops early
        resident = {k: s.table_bytes for k, s in self.structs.items() if s.image is not None}
        evictable = sorted((k for k, s in self.structs.items() if s.image is not None and s.users == 0),
                           key=lambda k: self.structs[k].last_use)
        table_bytes = {k: s.table_bytes for k, s in self.structs.items()}
        admitted, evict = plan_admission(waiting, free_slots, self.free_bytes(), resident, evictable,
                                         table_bytes, self.budget)
        for k in evict:
            self.structs[k].image = None
            self.structs[k].tables.image = None
        if not admitted:
            return
        chosen = set(admitted)
        keep = collections.deque()
        byid = {}
        for w in self.waiting:
            if w[0].rid in chosen:
                byid[w[0].rid] = w
            else:
                keep.append(w)
        self.waiting = keep
        for rid in admitted:
            self._start(*byid[rid])

    def _start(self, req: Request, lane_idx: int, nbytes: int, key: Tuple) -> None:
        torch = self.torch
        s = self.structs[key]
        lane = self.lanes[lane_idx]
        st = lane.stream
        with torch.cuda.stream(st):
            if s.image is None:
                img = torch.empty(s.table_bytes, dtype=torch.uint8, device="cuda")
                s.tables.upload(img, st)
                s.image = img
            s.users += 1
            s.last_use = self.now()
            params = torch.empty(_round(s.params_bytes), dtype=torch.uint8, device="cuda")
            s.tables.upload_params(req.problem, params, st)
            y = torch.empty(s.n_var, dtype=torch.complex128, device="cuda")
            tier0 = req.tier0 if req.tier0 is not None else s.tables.tier0_pure(1.0, 0.0, [0.0] * int(req.problem.d))
            s.tables.init_state(tier0, y, st)
            work = torch.empty(_round(s.work_bytes), dtype=torch.uint8, device="cuda")
            nobs = req.horizon // req.obs_every + 1 if req.obs_every > 0 else 1
            obs = torch.zeros(nobs * heom.HEOM_NOBS, dtype=torch.float64, device="cuda")
        slot = lane.free.pop()
        lane.batch.set_slot(slot, s.tables, y, work, req.dt, params=params,
                            obs=obs if req.obs_every > 0 else None, obs_every=req.obs_every)
        lane.active[slot] = _Active(req, slot, key, s.n_var, nbytes, self.now(), 0, (params, y, work, obs))
        lane.dirty = True
        self.held_bytes += nbytes
        self.waiting_per_lane[lane_idx] -= 1
        self.peak_bytes = max(self.peak_bytes, self.held_bytes + self._resident_bytes())
        self.peak_in_flight = max(self.peak_in_flight, self.in_flight())

    def _retire(self, lane: _Lane) -> None:
        """Lane idle: hand back every request that reached its horizon."""
        done = [a for a in lane.active.values() if a.enqueued >= a.req.horizon]
        if not done:
            return
        # slots whose state became NaN or infinite since the lane's last commit
        flags = lane.batch.status(lane.stream) if not lane.dirty else None
        for a in done:
            obs = a.bufs[3].cpu().numpy().reshape(-1, heom.HEOM_NOBS)
            fin = bool(np.isfinite(obs).all()) and (flags is None or flags[a.slot] == 0)
            self.results.append(Result(a.req.rid, a.req.arrival, a.admitted, self.now(), obs, a.n_var, lane.index,
                                       finite=fin))
            lane.batch.clear_slot(a.slot)
            lane.free.append(a.slot)
            del lane.active[a.slot]
            s = self.structs[a.key]
            s.users -= 1
            s.last_use = self.now()
            self.held_bytes -= a.nbytes
            lane.dirty = True

    def _launch(self, lane: _Lane) -> None:
        torch = self.torch
        if lane.dirty:
            lane.batch.commit(torch, lane.stream)
            lane.dirty = False
        rem = [a.req.horizon - a.enqueued for a in lane.active.values()]
        nv = sum(a.n_var for a in lane.active.values())
        k = chunk_steps(rem, predicted_ms_per_step(lane.ms_per_step, lane.measured_vars, nv), self.target_ms)
        if k <= 0:
            return
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(lane.stream)
        lane.batch.propagate(k, lane.precision, lane.stream)
        e1.record(lane.stream)
        for a in lane.active.values():
            a.enqueued += k
        lane.inflight.append((e0, e1, k, nv))

    def _boundary_pending(self, lane: _Lane) -> bool:
        """True when the lane's slot set changes at the end of what is queued:
        a request reaches its horizon, or a waiting request could join."""
        if any(a.enqueued >= a.req.horizon for a in lane.active.values()):
            return True
        return bool(lane.free) and self.waiting_per_lane[lane.index] > 0

    def poll(self) -> bool:
        """One pass of the event loop; returns True if anything happened."""
        progressed = False
        idle = []
        for lane in self.lanes:
            while lane.inflight and lane.inflight[0][1].query():
                e0, e1, k, nv = lane.inflight.popleft()
                ms = e0.elapsed_time(e1)
                lane.busy_ms += ms
                lane.chunks += 1
                lane.ms_per_step = ms / k
                lane.measured_vars = nv
                progressed = True
            idle.append(not lane.inflight)
        for lane in self.lanes:
            if idle[lane.index]:
                n0 = len(self.results)
                self._retire(lane)
                progressed |= len(self.results) != n0
        n0 = self.in_flight()
        self._admit(idle)
        progressed |= self.in_flight() != n0
        for lane in self.lanes:
            if not lane.active:
                continue
            if not lane.inflight:
                self._launch(lane)
                progressed = True
            elif len(lane.inflight) < 2 and not self._boundary_pending(lane):
                self._launch(lane)       # keep the lane's queue two chunks deep
                progressed = True
        return progressed

    def run(self, requests: Sequence[Request], window: Optional[float] = None,
            deadline: Optional[float] = None) -> Dict:
        """Replay a trace: each request is submitted at its arrival time
        (seconds from the start). Only arrivals up to `window` seconds are
        submitted (all when None). The run ends when every submitted request
        has completed or, if given, at `deadline` seconds; what is then
        still waiting or in flight is reported as outstanding. Returns
        summary statistics; per-request results are in self.results."""
        reqs = [r for r in sorted(requests, key=lambda r: r.arrival) if window is None or r.arrival <= window]
        self.t0 = self._clock()
        i = 0
        submitted = []
        while True:
            now = self.now()
            while i < len(reqs) and reqs[i].arrival <= now:
                if self.submit(reqs[i]):
                    submitted.append((reqs[i].rid, reqs[i].arrival))
                i += 1
            more = i < len(reqs)
            busy = self.in_flight() > 0 or bool(self.waiting)
            if not more and not busy:
                break
            if deadline is not None and now > deadline:
                break
            if not self.poll():
                if not busy and more:
                    time.sleep(max(0.0, min(reqs[i].arrival - now, 0.01)))
                else:
                    time.sleep(0.0002)
        for lane in self.lanes:
            lane.stream.synchronize()
        elapsed = self.now()
        out = summarize(self.results, submitted, elapsed, outstanding=self.in_flight() + len(self.waiting),
                        busy_ms=[l.busy_ms for l in self.lanes])
        out.update(peak_bytes=self.peak_bytes, peak_in_flight=self.peak_in_flight, rejected=len(self.rejected),
                   chunks=[l.chunks for l in self.lanes], nonfinite=sum(1 for r in self.results if not r.finite))
        return out


# --------------------------------------------------------------- plain baseline

class Fifo:
    """The plain per-instance FP64 (or FP32-bulk) propagator, one request at a
    time in arrival order: tables of the request's structure key with its own
    parameters (heom_set_params + heom_upload), then heom_propagate in chunks
    of `chunk` steps (a multiple of obs_every) so that a stop time can end it."""

    def __init__(self, torch, precision: int = heom.HEOM_FP64, chunk: int = 2000,
                 clock: Callable[[], float] = None):
        self.torch = torch
        self.precision = precision
        self.chunk = int(chunk)
        self.structs: Dict[Tuple, "heom.Tables"] = {}
        self.results: List[Result] = []
        self._clock = clock or time.perf_counter
        self.t0 = None

    def now(self) -> float:
        return self._clock() - self.t0

    def prepare(self, problems) -> None:
        for p in problems:
            self._tables(p)

    def _tables(self, p) -> "heom.Tables":
        key = structure_key(p)
        T = self.structs.get(key)
        if T is None:
            T = heom.Tables(p)
            if self.precision & heom.HEOM_HERMITIAN:
                T.set_tuning(compact=1)
            self.structs[key] = T
        return T

    def solve(self, req: Request, deadline: Optional[float] = None) -> Optional[np.ndarray]:
        """One request start to finish; None if the deadline passed first."""
        torch = self.torch
        s = torch.cuda.current_stream()
        T = self._tables(req.problem)
        T.set_params(req.problem)
        info = T.info()
        img = torch.empty(_round(info["table_bytes"]), dtype=torch.uint8, device="cuda")
        T.upload(img, s)
        y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
        tier0 = req.tier0 if req.tier0 is not None else T.tier0_pure(1.0, 0.0, [0.0] * int(req.problem.d))
        T.init_state(tier0, y, s)
        work = torch.empty(_round(info["work_bytes_fp64"]), dtype=torch.uint8, device="cuda")
        every = req.obs_every
        nobs = req.horizon // every + 1 if every > 0 else 1
        obs = torch.zeros(nobs * heom.HEOM_NOBS, dtype=torch.float64, device="cuda")
        step = max(self.chunk - self.chunk % every, every) if every > 0 else self.chunk
        done = 0
        while done < req.horizon:
            k = min(step, req.horizon - done)
            view = obs[(done // every) * heom.HEOM_NOBS:] if every > 0 else None
            T.propagate(y, work, req.dt, k, every, view, self.precision, s)
            done += k
            if deadline is not None and done < req.horizon:
                torch.cuda.synchronize()
                if self.now() > deadline:
                    return None
        return obs.cpu().numpy().reshape(-1, heom.HEOM_NOBS)

    def run(self, requests: Sequence[Request], window: Optional[float] = None,
            deadline: Optional[float] = None) -> Dict:
        """The same trace rules as Server.run."""
        reqs = [r for r in sorted(requests, key=lambda r: r.arrival) if window is None or r.arrival <= window]
        self.t0 = self._clock()
        completed = 0
        for j, r in enumerate(reqs):
            now = self.now()
            if deadline is not None and max(now, r.arrival) > deadline:
                break
            if r.arrival > now:
                time.sleep(r.arrival - now)
            start = self.now()
            obs = self.solve(r, deadline)
            if obs is None:
                break
            T = self.structs[structure_key(r.problem)]
            self.results.append(Result(r.rid, r.arrival, start, self.now(), obs, int(T.info()["n_var"])))
            completed += 1
        self.torch.cuda.synchronize()
        elapsed = self.now()
        submitted = [(r.rid, r.arrival) for r in reqs if r.arrival <= elapsed]
        return summarize(self.results, submitted, elapsed, outstanding=len(submitted) - completed)


# --------------------------------------------------------------- statistics

def summarize(results: Sequence[Result], submitted, elapsed: float, outstanding: int = 0,
              busy_ms=None) -> Dict:
    """Throughput and latency of a run. `submitted`: (rid, arrival) of every
    request admitted to the queue (or their count). Percentiles are given
    over the completed requests and, as a lower bound that does not favour
    a policy that finishes only its short requests, over all submitted ones
    with each unfinished request counted as waiting until the end of the run."""
    lat = np.array([r.latency for r in results]) if results else np.zeros(0)
    if isinstance(submitted, int):
        n_sub, cens = submitted, np.zeros(0)
    else:
        done = {r.rid for r in results}
        n_sub = len(submitted)
        cens = np.array([elapsed - a for rid, a in submitted if rid not in done])
    allv = np.concatenate([lat, cens])
    out = {
        "submitted": int(n_sub),
        "completed": len(results),
        "outstanding": int(outstanding),
        "elapsed_s": float(elapsed),
        "solves_per_s": len(results) / elapsed if elapsed > 0 else 0.0,
        "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
        "mean_latency_s": float(lat.mean()) if lat.size else None,
        "p50_latency_all_lower_bound_s": float(np.percentile(allv, 50)) if allv.size else None,
        "p99_latency_all_lower_bound_s": float(np.percentile(allv, 99)) if allv.size else None,
    }
    if busy_ms is not None:
        out["lane_busy_ms"] = [float(b) for b in busy_ms]
    return out


def make_requests(problems, arrivals: Sequence[float], dt: float = 0.02, obs_every: int = 100) -> List[Request]:
    """Requests from problems carrying a `horizon` attribute (RK4 steps),
    rounded up to a multiple of obs_every, at the given arrival times."""
    out = []
    for i, (p, t) in enumerate(zip(problems, arrivals)):
        h = int(p.horizon)
        h = ((h + obs_every - 1) // obs_every) * obs_every
        out.append(Request(i, p, h, dt, obs_every, float(t)))
    return out
