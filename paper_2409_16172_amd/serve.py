"""Continuous-batching solve server on one GPU.

Requests (a medium, a frequency and a right-hand side each) arrive over time.
A request is admitted as soon as its device footprint (preconditioner plan plus
Krylov workspace) fits in the HBM budget and an active slot is free; admission
builds its plan (FP64 set-up on the host, upload) and starts a resumable solve
on a stream of its own.  The loop then advances every active solve by a few
Arnoldi steps at a time without waiting on the device, so the work of different
requests overlaps on the GPU; a finished request retires and frees its slot and
memory for the queue.  Latency is measured from arrival to the solution.
All GPU work runs in the HIP library; this module only schedules it.
"""
from __future__ import annotations

import heapq
import time
from dataclasses import dataclass, field

import numpy as np

from . import binding, inputs


@dataclass
class Request:
    rid: int
    arrival: float            # seconds from the start of the stream
    workload: inputs.Workload
    k_nodes: int = 0
    footprint: int = 0
    # filled by the server
    admitted: float = 0.0
    finished: float = 0.0
    info: list = field(default_factory=list)
    x: object = None


def _pooled_workload(base, n_lambda, seed):
    """A request on a pooled medium: its own frequency (n_lambda wavelengths), damping
    a = 0.05 omega and Gaussian source at a seeded position; the medium (c, layer)
    is shared with the other requests drawn from the same pool entry."""
    shape = base.shape
    omega = inputs.omega_for_wavelengths(n_lambda)
    width = base.info["layer_cells"]
    ctr = inputs.random_source_centres(shape, 1, width, 2.0, seed)[0]
    f = inputs.gaussian_source(shape, 2.0, ctr)[None]
    info = dict(base.info)
    info.update({"n_lambda": n_lambda, "source": ctr, "pool_seed": base.info.get("seed")})
    return inputs.Workload(base.name, shape, base.length, omega, base.c, np.full(shape, 0.05 * omega), base.zeta, f,
                           base.m_real, base.m_layer, a_floor=0.05 * omega, precision=base.precision, info=info)


def stream_requests(n_requests, rate_per_s, seed=20240920, grids=((256, 256), (512, 512), (1024, 1024)),
                    precision="mixed", n_lambda=(20.0, 150.0), restart=30, pool=None):
    """Seeded request stream: Poisson arrivals; grid drawn from `grids`; wavelengths
    across the domain drawn uniformly and clamped to at most N/4 (4 points per
    wavelength); media and source from the random-field recipes (2-D: correlation 20
    cells, layer max(8, N/32) cells; 3-D: correlation 12 cells scaled, sphere).
    pool: None, a new medium per request; an integer P, P media per grid generated
    once and drawn from by the requests (each still with its own frequency and
    source), which keeps the host-side generation of long streams short."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    media = {}
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        shape = tuple(grids[rng.integers(len(grids))])
        n = shape[0]
        nl = min(rng.uniform(*n_lambda), n / 4.0)
        wseed = int(rng.integers(1 << 30))
        if pool:
            slot = (shape, int(rng.integers(pool)))
            if slot not in media:
                mseed = int(np.random.default_rng([seed, n, len(shape), slot[1]]).integers(1 << 30))
                media[slot] = _fresh_workload(shape, nl, mseed, precision)
            w = _pooled_workload(media[slot], nl, wseed)
        else:
            w = _fresh_workload(shape, nl, wseed, precision)
        r = Request(rid, t, w)
        r.k_nodes = w.m_real + w.m_layer
        r.footprint = binding.workspace_bytes(w.shape, precision, r.k_nodes, 1, restart)
        reqs.append(r)
    return reqs


def _fresh_workload(shape, nl, wseed, precision):
    n = shape[0]
    if len(shape) == 2:
        return inputs.workload("2d_1024_grf", n=n, n_lambda=nl, width=max(8, n // 32), seed=wseed,
                               m_real=24 if n >= 2048 else 16, precision=precision)
    w = inputs.workload("3d_256_grf", n=n, n_lambda=nl, nrhs=1, seed=wseed)
    w.precision = precision
    return w


def retimed(requests, rate_per_s=None, seed=20240921):
    """Fresh copies of `requests` (same problems, no results) with new arrival times:
    Poisson arrivals at rate_per_s, or all at time 0 when rate_per_s is None (a closed
    loop that measures capacity)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in requests:
        if rate_per_s is not None:
            t += rng.exponential(1.0 / rate_per_s)
        c = Request(r.rid, t, r.workload, r.k_nodes, r.footprint)
        out.append(c)
    return out


class Server:
    """keep_x: keep each request's solution tensor on the GPU (False: only its info,
    so that long streams do not hold every solution).
    grouped: the active solves are spread over `streams` streams and advance together,
    the Arnoldi steps of those on one stream that the grouped kernels take running as
    one launch per pass over all of them (uneven grids and media in the same launches);
    otherwise each active solve runs its own launches on a stream of its own."""

    def __init__(self, hbm_budget_bytes, max_active=8, steps_per_turn=2, restart=30, rtol=1e-8,
                 max_cycles=200, keep_x=True, grouped=False, streams=4):
        self.budget = int(hbm_budget_bytes)
        self.max_active = int(max_active)
        self.steps = int(steps_per_turn)
        self.restart, self.rtol, self.max_cycles = restart, rtol, max_cycles
        self.keep_x = bool(keep_x)
        self.grouped = bool(grouped)
        self.n_streams = max(1, int(streams))
        self._streams = []
        self._admitted = 0
        self.in_use = 0
        self.peak_in_use = 0
        self.deferred_rids = set()   # requests held back by the HBM budget while a slot was free
        self.active = []
        self.done = []

    def _admit(self, r, now, dev, torch):
        w = r.workload
        if self.grouped:
            if not self._streams:
                self._streams = [torch.cuda.Stream(device=dev) for _ in range(self.n_streams)]   # default priority
            # the stream with the fewest active solves (ties: round robin)
            load = [sum(1 for it in self.active if it[5] is st) for st in self._streams]
            k0 = self._admitted % self.n_streams
            k = min(range(self.n_streams), key=lambda q: (load[q], (q - k0) % self.n_streams))
            stream = self._streams[k]
            self._admitted += 1
        else:
            stream = torch.cuda.Stream(device=dev)          # default priority
        plan = binding.plan_from_workload(w, max_nrhs=1)
        solver = binding.Solver(plan, 1, restart=self.restart, max_cycles=self.max_cycles, rtol=self.rtol)
        with torch.cuda.stream(stream):
            f = torch.from_numpy(w.f[:1]).to(dev, non_blocking=False)
        stream.synchronize()
        x = solver.start(f, stream=stream)
        r.admitted = now
        self.in_use += r.footprint
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        self.active.append((r, plan, solver, f, x, stream))

    def _progress(self, item, t0, finished=None):
        """Advance one active solve by a few steps (or take the grouped advance's
        verdict `finished`); on completion collect its result and release its plan
        and workspace.  Returns True when it has finished."""
        r, plan, solver, f, x, stream = item
        if finished is None:
            finished = solver.advance(self.steps)
        if not finished:
            return False
        x, info = solver.result()
        r.finished = time.perf_counter() - t0
        r.info = info
        r.x = x if self.keep_x else None
        solver.close()
        plan.close()
        return True

    def run(self, requests, dev=None, time_scale=1.0):
        """Serve `requests` (sorted by arrival); returns the finished requests."""
        torch = None
        if dev is not False:
            import torch
            dev = dev or torch.device("cuda:0")
        queue = []
        pending = sorted(requests, key=lambda r: r.arrival)
        t0 = time.perf_counter()
        i = 0
        while i < len(pending) or queue or self.active:
            now = time.perf_counter() - t0
            while i < len(pending) and pending[i].arrival * time_scale <= now:
                heapq.heappush(queue, (pending[i].arrival, pending[i].rid, pending[i]))
                i += 1
            # admission: first come first served while slots and memory allow
            while queue and len(self.active) < self.max_active:
                r = queue[0][2]
                if self.in_use + r.footprint > self.budget and self.active:
                    self.deferred_rids.add(r.rid)
                    break
                heapq.heappop(queue)
                self._admit(r, time.perf_counter() - t0, dev, torch)
            # progress every active solve without waiting on the device
            flags = [None] * len(self.active)
            if self.grouped and self.active:
                flags = binding.advance_group([it[2] for it in self.active], self.steps)
            still = []
            for item, fl in zip(self.active, flags):
                if (self._progress(item, t0) if fl is None else self._progress(item, t0, fl)):
                    self.in_use -= item[0].footprint
                    self.done.append(item[0])
                else:
                    still.append(item)
            self.active = still
            if not self.active and not queue and i < len(pending):
                # idle until the next arrival
                time.sleep(max(0.0, pending[i].arrival * time_scale - (time.perf_counter() - t0)))
        return self.done


def latency_stats(done, time_scale=1.0):
    lat = np.array([r.finished - r.arrival * time_scale for r in done])
    span = max(r.finished for r in done) - min(r.arrival * time_scale for r in done)
    return {"requests": len(done), "solves_per_s": len(done) / span,
            "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
            "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
            "converged": int(sum(r.info[0].status == 0 for r in done))}
