"""Continuous-batching server for CBS forward and adjoint solves on one GPU.

Requests (mixed grid sizes, forward or adjoint = forward + adjoint solve +
permittivity gradient) arrive over time.  The server keeps plans, fields and
FFT scratch resident in reusable slots, admits waiting requests in arrival
order whenever a slot and HBM budget are free (footprint admission), and
advances every active solve in small quanta on its own HIP stream, so solves
of different sizes overlap on the device.  A solve's iteration count is decided
by its own device-side stopping rule, independent of quanta, and every
reduction is fixed-order, so a request's result is bit-identical alone and in
the mix.  All arithmetic runs in libcbs; this module only schedules.

A request the library rejects (an invalid medium: gain, a non-finite value,
material in the absorbing layer) or whose solve diverges (non-finite residual)
fails alone: its result carries the library's negative status, no fields or
gradient, and the other requests are served as if it had not been there.

Scheduling.  Admission is in arrival order while a slot and HBM are free.
Active solves advance in quanta of about 4 ms of device work, each on its own
stream.  A request whose solve has run for longer than `exclusive_after_s`
since admission is given the device alone: no new request is admitted and the
other active solves get no further quanta until it completes (their queued
quanta drain), and it advances in quanta `exclusive_scale` times longer with one
more in flight.  One large solve saturates HBM by itself, so sharing the device
with it only stretches it; short requests keep overlapping freely.  This keeps
the latency of the few long solves near their one-at-a-time service time while
the many short ones are served concurrently.

Latency is arrival -> result complete in device memory.
"""

from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np
import torch

from . import libcbs as L
from .scenes import ServedRequest
from .solver import Plan


@dataclasses.dataclass
class ServedResult:
    rid: int
    kind: str
    shape: tuple
    status: int
    iterations: tuple            # (forward, adjoint)
    arrival: float
    admitted: float
    finished: float
    E: torch.Tensor | None = None
    E_adj: torch.Tensor | None = None
    grad: torch.Tensor | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class _Slot:
    """A resident plan with its fields, on its own stream."""

    def __init__(self, key, device, stream):
        shape, pitch, pml, lam, nbg = key
        self.key = key
        self.stream = stream
        with torch.cuda.stream(stream):
            self.plan = Plan(shape, pitch, lam, nbg, pml, device=device, stream=stream)
            self.E = self.plan.new_field()
            self.Ea = self.plan.new_field()
            nx, ny, nz = shape
            self.eps = torch.empty((nz, ny, nx), dtype=torch.float32, device=device)
        # pinned staging buffer: a request's permittivity is uploaded without a
        # pageable (blocking) copy
        self.eps_host = torch.empty((nz, ny, nx), dtype=torch.float32, pin_memory=True)
        self.nbytes = slot_bytes(shape)
        self.last_used = 0.0

    def upload(self, eps_r: np.ndarray):
        """Stage eps_r in pinned memory and copy it on the slot's stream (the
        previous use of the staging buffer completed: set_permittivity
        synchronises the stream)."""
        self.eps_host.numpy()[...] = eps_r
        with torch.cuda.stream(self.stream):
            self.eps.copy_(self.eps_host, non_blocking=True)

    def close(self):
        self.plan.close()


def slot_bytes(shape) -> int:
    """HBM footprint of one slot: workspace + E + E_adj + eps_r."""
    nx, ny, nz = shape
    n = nx * ny * nz
    return L.cbs_plan_workspace_bytes(nx, ny, nz) + 2 * 24 * n + 4 * n


def quantum_for(shape, target_ms: float = 4.0) -> int:
    """Iterations per quantum so that one quantum is about target_ms of work
    (248 B/voxel-iteration at ~5 TB/s plus ~25 us of launches)."""
    nx, ny, nz = shape
    it_ms = nx * ny * nz * 248 / 5e12 * 1e3 + 0.025
    return int(min(200, max(2, round(target_ms / it_ms))))


class _Job:
    def __init__(self, req: ServedRequest, slot: _Slot, admitted: float):
        self.req = req
        self.slot = slot
        self.admitted = admitted
        self.phase = 0        # 0 forward, 1 adjoint
        self.iters = [0, 0]
        self.status = L.CBS_OK
        self.quantum = quantum_for(req.scene.shape)


class Server:
    """One-GPU continuous-batching CBS server.

    max_active   slots that may run concurrently (each on its own stream)
    budget_bytes HBM the server may hold for slots (default 85% of free)
    inflight     quanta kept queued per active solve
    """

    def __init__(self, device=None, max_active: int = 4, budget_bytes: int | None = None,
                 tol: float = 1e-4, max_iter: int = 20000, inflight: int = 2,
                 target_ms: float = 4.0, exclusive_after_s: float | None = 0.25,
                 exclusive_scale: int = 4):
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget_bytes = int(0.85 * free)
        self.budget = budget_bytes
        self.max_active = max_active
        self.tol = tol
        self.max_iter = max_iter
        self.inflight = inflight
        self.target_ms = target_ms
        self.exclusive_after_s = exclusive_after_s
        self.exclusive_scale = int(exclusive_scale)
        self.idle = collections.defaultdict(list)   # key -> [_Slot]
        self.used = 0
        self.refused = 0

    # -- slots -----------------------------------------------------------------
    @staticmethod
    def key_of(sc):
        return (tuple(sc.shape), float(sc.pitch), tuple(sc.pml), float(sc.lambda0), float(sc.n_bg))

    def _acquire(self, sc, now) -> _Slot | None:
        key = self.key_of(sc)
        if self.idle[key]:
            return self.idle[key].pop()
        need = slot_bytes(sc.shape)
        if need > self.budget:
            raise ValueError(f"request footprint {need} B exceeds the server budget {self.budget} B")
        # evict least-recently-used idle slots until the new one fits
        while self.used + need > self.budget:
            cands = [(s.last_used, k, i) for k, lst in self.idle.items() for i, s in enumerate(lst)]
            if not cands:
                return None
            _, k, i = min(cands)
            s = self.idle[k].pop(i)
            self.used -= s.nbytes
            s.close()
            del s
        slot = _Slot(key, self.device, torch.cuda.Stream(self.device))
        self.used += slot.nbytes
        return slot

    def _release(self, slot: _Slot, now):
        slot.last_used = now
        self.idle[slot.key].append(slot)

    def close(self):
        for lst in self.idle.values():
            for s in lst:
                s.close()
        self.idle.clear()
        self.used = 0

    # -- job phases ------------------------------------------------------------
    def _start(self, job: _Job):
        s = job.slot
        sc = job.req.scene
        s.upload(sc.eps_r)
        s.plan.set_permittivity(s.eps)
        s.plan.begin(s.E, tol=self.tol, max_iter=self.max_iter)
        for _ in range(self.inflight):
            s.plan.advance(job.quantum)

    def _next_phase(self, job: _Job) -> bool:
        """Called when the current solve stopped; True when the job is complete."""
        s = job.slot
        try:
            st = s.plan.end()
        except L.CbsError as e:
            if e.code != L.CBS_E_DIVERGED:
                raise
            job.status = e.code       # the plan has left the solve and is reusable
            return True
        job.iters[job.phase] = st.iterations
        if st.status not in (L.CBS_OK,):
            job.status = st.status
        if job.req.kind == "adjoint" and job.phase == 0:
            job.phase = 1
            s.plan.begin(s.Ea, adjoint=True, E_fwd=s.E, r0=job.req.scene.r0, tol=self.tol,
                         max_iter=self.max_iter)
            for _ in range(self.inflight):
                s.plan.advance(job.quantum)
            return False
        return True

    def _finish(self, job: _Job, t0: float, keep: bool) -> ServedResult:
        s = job.slot
        sc = job.req.scene
        grad = None
        failed = job.status < 0
        if job.req.kind == "adjoint" and not failed:
            lo, hi = sc.design_box
            grad = s.plan.gradient(s.E, s.Ea, lo, hi, scale=2.0)
        s.stream.synchronize()
        fin = time.perf_counter() - t0
        res = ServedResult(job.req.rid, job.req.kind, tuple(sc.shape), job.status,
                           tuple(job.iters), job.req.arrival, job.admitted, fin)
        if keep and not failed:
            with torch.cuda.stream(s.stream):   # ordered before the slot's next use
                res.E = s.E.clone()
                if job.req.kind == "adjoint":
                    res.E_adj = s.Ea.clone()
                    res.grad = grad.clone()
            s.stream.synchronize()
        return res

    # -- the loop --------------------------------------------------------------
    def run(self, requests, keep_fields: bool = False, realtime: bool = True, progress=None):
        """Serve `requests` (ServedRequest, arrival times in seconds from the
        start).  realtime=False admits every request at t = 0 (offline batch).
        Returns results in completion order."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = collections.deque(reqs)
        waiting = collections.deque()
        active: list[_Job] = []
        results = []
        t0 = time.perf_counter()
        while pending or waiting or active:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                waiting.append(pending.popleft())
            # the oldest active solve, once long-running, has the device alone
            excl = None
            if active and self.exclusive_after_s is not None \
                    and now - active[0].admitted > self.exclusive_after_s:
                excl = active[0]
            while excl is None and waiting and len(active) < self.max_active:
                slot = self._acquire(waiting[0].scene, now)
                if slot is None:
                    self.refused += 1
                    break
                job = _Job(waiting.popleft(), slot, time.perf_counter() - t0)
                try:
                    self._start(job)
                except L.CbsError as e:
                    if e.code != L.CBS_E_INVALID:
                        raise
                    job.status = e.code
                    results.append(self._finish(job, t0, keep_fields))
                    if progress is not None:
                        progress(results[-1], len(results))
                    self._release(slot, time.perf_counter() - t0)
                    continue
                active.append(job)
            if not active:
                if pending:
                    time.sleep(max(0.0, min(0.005, pending[0].arrival - now)))
                continue
            progressed = False
            for job in list(active):
                done, outstanding = job.slot.plan.poll()
                if done:
                    progressed = True
                    if self._next_phase(job):
                        results.append(self._finish(job, t0, keep_fields))
                        if progress is not None:
                            progress(results[-1], len(results))
                        active.remove(job)
                        self._release(job.slot, time.perf_counter() - t0)
                elif job is excl and outstanding < self.inflight + 1:
                    # alone on the device: longer quanta, one more in flight, so
                    # the host's polling never leaves it idle
                    job.slot.plan.advance(self.exclusive_scale * job.quantum)
                    progressed = True
                elif excl is None and outstanding < self.inflight:
                    job.slot.plan.advance(job.quantum)
                    progressed = True
            if not progressed:
                time.sleep(20e-6)
        return results

    def run_sequential(self, requests, keep_fields: bool = False, progress=None):
        """The same requests one at a time with plain blocking solves, each
        started when it has arrived and the previous one has finished."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        results = []
        t0 = time.perf_counter()
        for r in reqs:
            now = time.perf_counter() - t0
            if r.arrival > now:
                time.sleep(r.arrival - now)
            adm = time.perf_counter() - t0
            slot = self._acquire(r.scene, adm)
            if slot is None:
                raise RuntimeError("no memory for a sequential slot")
            p = slot.plan
            slot.upload(r.scene.eps_r)
            its = (0, 0)
            grad = None
            try:
                p.set_permittivity(slot.eps)
                _, s1 = p.solve(slot.E, tol=self.tol, max_iter=self.max_iter, check_every=20)
                its = (s1.iterations, 0)
                status = s1.status
                if r.kind == "adjoint":
                    _, s2 = p.adjoint(E_fwd=slot.E, r0=r.scene.r0, E_adj=slot.Ea, tol=self.tol,
                                      max_iter=self.max_iter, check_every=20)
                    lo, hi = r.scene.design_box
                    grad = p.gradient(slot.E, slot.Ea, lo, hi, scale=2.0)
                    its = (s1.iterations, s2.iterations)
                    status = status or s2.status
            except L.CbsError as e:
                if e.code not in (L.CBS_E_INVALID, L.CBS_E_DIVERGED):
                    raise
                status = e.code
            slot.stream.synchronize()
            fin = time.perf_counter() - t0
            res = ServedResult(r.rid, r.kind, tuple(r.scene.shape), status, its, r.arrival, adm, fin)
            if keep_fields and status >= 0:
                with torch.cuda.stream(slot.stream):
                    res.E = slot.E.clone()
                    if r.kind == "adjoint":
                        res.E_adj = slot.Ea.clone()
                        res.grad = grad.clone()
                slot.stream.synchronize()
            results.append(res)
            self._release(slot, fin)
            if progress is not None:
                progress(res, len(results))
        return results


def fifo_one_at_a_time(requests, service: dict) -> list:
    """Results of serving `requests` one at a time in arrival order, from each
    request's measured service time (service[rid], from a back-to-back
    run_sequential pass): each starts at max(its arrival, the previous finish).
    Solves are deterministic (fixed-order reductions, device-side stopping
    rule), so a request's service time does not depend on when it runs."""
    out = []
    t = 0.0
    for r in sorted(requests, key=lambda r: r.arrival):
        sv = service[r.rid]
        start = max(r.arrival, t)
        t = start + sv.seconds
        out.append(ServedResult(r.rid, r.kind, tuple(r.scene.shape), sv.status, sv.iterations,
                                r.arrival, start, t))
    return out


@dataclasses.dataclass
class ServiceTime:
    seconds: float
    status: int
    iterations: tuple


def service_times(results) -> dict:
    """rid -> service time of a back-to-back run_sequential pass."""
    return {r.rid: ServiceTime(r.finished - r.admitted, r.status, r.iterations) for r in results}


def summarize(results, wall_s: float | None = None) -> dict:
    """p50/p99 latency, throughput and aggregate voxel-iterations per second."""
    lat = np.array([r.latency for r in results])
    if wall_s is None:
        wall_s = max(r.finished for r in results) - min(r.arrival for r in results)
    vi = sum(int(np.prod(r.shape)) * sum(r.iterations) for r in results)
    return {
        "requests": len(results),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()),
        "throughput_solves_per_s": len(results) / wall_s,
        "gvoxel_iter_per_s": vi / wall_s / 1e9,
        "wall_s": wall_s,
        "not_ok": sum(1 for r in results if r.status != L.CBS_OK),
    }
