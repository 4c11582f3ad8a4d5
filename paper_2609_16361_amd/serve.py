"""Continuous-batching solve server over one lbm_batch.

Requests (an initial state, a step count, a storage type) arrive over time.  The
serving loop admits requests that have arrived (in the order below) as long as
their populations fit in the HBM budget (the batch arena) and the active-cell cap
allows; it then advances the whole batch by one graph-captured chunk of steps
(every admitted instance overlaps with the others on the device), retires the
instances that have made their steps, reads their conserved fields back and frees
their memory for the next arrivals.  A result is exactly what the same request
gives alone: the batch updates each instance with the same arithmetic as a single
context, and an instance freezes when it reaches its own step count.

Admission order is largest work (cells x steps) first among the arrived requests,
except that a request waiting longer than max_wait_s (2 s by default) goes first
in arrival order; this starts the long solves early and fills the gaps with short
ones.  order="fifo" admits strictly in arrival order.

A request whose state stops being finite (the scheme has diverged) is retired as
failed at the next divergence check (every 200 steps by default), rather than
occupying the device until its step count.  A request the library refuses at
admission (an initial state with non-positive density or pressure, or one larger
than the whole budget) is rejected: it never runs and is counted apart from the
failures.  The sequential baseline applies the same divergence check and the
same rejection.

The loop runs on the wall clock (arrival times are seconds after start); latency
is completion minus arrival.  A stand-in backend with the same methods as
binding.Batch can replace the GPU (the CPU tests use one).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

EINVAL, ENOMEM = -1, -2  # lbm_status LBM_EINVAL, LBM_ENOMEM


@dataclass
class Outcome:
    rid: int
    kind: str
    storage: int
    cells: int
    steps: int
    arrival: float
    admitted: float = math.nan
    completed: float = math.nan
    ok: bool = False
    result: object = None       # whatever the result handler returned
    rejected: str = ""          # why admission refused it ("" = admitted)

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


@dataclass
class ServeStats:
    outcomes: list = field(default_factory=list)
    wall_s: float = 0.0
    chunks: int = 0
    max_active: int = 0
    peak_bytes: int = 0
    stopped: int = 0            # failed requests retired early by the divergence check
    # one entry per chunk: (start, end, resident instances, resident cells); the
    # instances that reached their step count earlier in the chunk are included
    timeline: list = field(default_factory=list)

    def summary(self) -> dict:
        done = [o for o in self.outcomes if o.ok]
        rejected = [o for o in self.outcomes if o.rejected]
        lat = np.array([o.latency for o in done]) if done else np.array([math.nan])
        first = min(o.arrival for o in self.outcomes) if self.outcomes else 0.0
        last = max((o.completed for o in done), default=first)
        span = max(last - first, 1e-9)
        lups = sum(o.cells * o.steps for o in done)
        return {"requests": len(self.outcomes), "completed": len(done),
                "failed": len(self.outcomes) - len(done) - len(rejected),
                "rejected": len(rejected),
                "rejected_by_kind": {k: sum(1 for o in rejected if o.kind == k)
                                     for k in sorted({o.kind for o in rejected})},
                "solves_per_s": len(done) / span, "span_s": span,
                "glups": lups / span / 1e9,
                "latency_p50_s": float(np.percentile(lat, 50)),
                "latency_p99_s": float(np.percentile(lat, 99)),
                "latency_mean_s": float(np.mean(lat)),
                "stopped_diverged": self.stopped,
                "resident_cells_mean": (sum((b - a) * c for a, b, _, c in self.timeline) /
                                        max(sum(b - a for a, b, _, _ in self.timeline), 1e-12)
                                        if self.timeline else 0.0),
                "chunks": self.chunks, "max_active": self.max_active,
                "peak_arena_bytes": self.peak_bytes, "wall_s": self.wall_s}


def state_bytes(params: dict, storage: int) -> int:
    """Device bytes of one instance -- mirrors lbm_state_bytes without a device
    call: 35 arrays, each starting on a 256-byte boundary, whose x-rows are padded
    to whole 128-byte lines when that adds at most a sixteenth of the row."""
    nx, ny, nz = int(params["nx"]), int(params["ny"]), int(params["nz"])
    el = 2 if storage else 4
    px = nx
    if ny * nz > 1:
        line = 128 // el
        pr = (nx + line - 1) // line * line
        px = pr if 16 * (pr - nx) <= nx and pr * ny * nz <= 2 ** 31 - 1 - 65535 else nx
    align = 256 // el
    s = (px * ny * nz + int(params.get("layout_pad", 0)) + align - 1) // align * align
    return 35 * el * s


class Server:
    """backend: object with add(params, Q, steps, storage) -> id, run(n), query(id)
    -> (done, finished), moments(id) -> Q, remove(id), and optionally nonfinite()
    -> ids of instances whose state is no longer finite.

    With stop_diverged (and a backend that has nonfinite()), a divergence check
    follows every chunk that completes check_steps steps (rounded up to whole
    chunks), and a request whose state has stopped being finite is retired at once
    as failed instead of running to its step count; its result handler is not
    called (it has no result), failure_handler(request) is."""

    def __init__(self, backend, arena_bytes: int, max_active_cells: int | None = None,
                 chunk_steps: int = 50, result_handler=None, clock=time.perf_counter,
                 sync=None, max_instances: int = 4096, storage_override: int | None = None,
                 order: str = "largest", max_wait_s: float | None = 2.0, stop_diverged: bool = True,
                 check_steps: int = 200, failure_handler=None, fp16_kinds=None, fp16_max_steps=None,
                 solo_factory=None, solo_min_bytes: int | None = None):
        self.b = backend
        # Requests whose state takes solo_min_bytes or more run in a context of their
        # own, made by solo_factory(request, storage) (an object with init(Q),
        # step(n, diag_every), diagnostics(), moments() and close(), on the stream
        # the batch uses), stepped one chunk at a time after each batch chunk; the
        # rest share the batch.  The single-context kernels move such states faster
        # than the batch kernel does (whole-row tiles, a launch shape chosen for the
        # grid), and the results are those of the same request run alone.  A solo
        # state is allocated by the factory, outside the batch's arena, and counts
        # against the same byte budget and cell cap: the device must hold the arena
        # and the solo states together (the benchmark's cell cap of 8 Mi cells keeps
        # them below 1.2 GB beside its 200 GB arena).
        self.solo_factory = solo_factory
        self.solo_min = solo_min_bytes if solo_factory is not None else None
        self.stop_diverged = bool(stop_diverged)
        self.check_steps = int(check_steps)
        self.arena_bytes = int(arena_bytes)
        self.max_cells = max_active_cells
        self.chunk = int(chunk_steps)
        self.handle = result_handler or (lambda req, Q: bool(np.isfinite(Q).all()))
        self.clock = clock
        self.sync = sync or (lambda: None)
        self.max_instances = max_instances
        # None: each request's own storage; else every request in this storage
        self.storage_override = storage_override
        # None: FP16 wherever requested; else a request of a kind outside this set
        # runs in FP32 (kinds whose stated accuracy FP16 storage does not reach)
        self.fp16_kinds = None if fp16_kinds is None else set(fp16_kinds)
        # None: any length; else a request of more steps runs in FP32 (stochastic
        # rounding's error grows about as the square root of the step count)
        self.fp16_max_steps = fp16_max_steps
        # "fifo": admit arrived requests in arrival order, the first that does not
        # fit blocks the rest; "largest": among the arrived requests, largest work
        # (cells x steps) first, skipping those that do not fit yet, except that
        # requests waiting longer than max_wait_s go first in arrival order.  The
        # first overdue request that does not fit holds a reservation: all
        # instances advance one step per step, so the chunk at which enough of
        # the running ones have finished for it to fit (its shadow) is known
        # exactly, and a later request is admitted meanwhile only if it finishes
        # by then or fits beside it in what is left at that chunk (backfilling).
        # So neither a stream of large requests nor one of small ones can hold a
        # request back without bound, and the device is not left half empty
        # while the overdue request waits.
        if order not in ("fifo", "largest"):
            raise ValueError(f"order must be 'fifo' or 'largest', not {order!r}")
        self.order = order
        self.max_wait = max_wait_s
        self.check = getattr(backend, "nonfinite", None) if stop_diverged else None
        # the check synchronises and reads 5 of the 35 arrays (about 45 us on the
        # 64-request serving mix): once per chunk cost 1-2% of its throughput
        self.check_chunks = max(1, -(-int(check_steps) // self.chunk))
        self.on_failure = failure_handler

    def storage_of(self, r) -> int:
        """The storage a request runs in."""
        if self.storage_override is not None:
            return self.storage_override
        if r.storage and self.fp16_kinds is not None and r.kind not in self.fp16_kinds:
            return 0
        if r.storage and self.fp16_max_steps is not None and r.steps > self.fp16_max_steps:
            return 0
        return r.storage

    def _chunks(self, steps: int) -> int:
        """Chunks until an instance with `steps` steps left retires."""
        return -(-max(int(steps), 0) // self.chunk)

    def _reserve(self, r, nb, active, used_bytes, used_cells, steps_run, fragmented=False):
        """Reservation for request r that does not fit now: the chunk at which it
        will (running instances retire in order of their remaining steps) and the
        bytes, cells and instance slots left beside it then."""
        rem = sorted((self._chunks(q.steps - (steps_run - s0)), b, q.case.cells) for q, b, s0 in active.values())
        fb = fc = fn = 0
        at = rem[0][0] if rem else 0
        for ch, b, c in rem:  # at least one retirement: r does not fit (or find room) now
            fb, fc, fn = fb + b, fc + c, fn + 1
            at = ch
            left = len(active) - fn
            if (used_bytes - fb + nb <= self.arena_bytes and left < self.max_instances and
                    (self.max_cells is None or left == 0 or used_cells - fc + r.case.cells <= self.max_cells)):
                break
        extra_b = self.arena_bytes - (used_bytes - fb) - nb
        extra_c = None if self.max_cells is None else self.max_cells - (used_cells - fc) - r.case.cells
        extra_n = self.max_instances - (len(active) - fn) - 1
        if fragmented:  # the byte count fits but no free run does: no room beside it
            extra_b = extra_n = 0
            extra_c = None if self.max_cells is None else 0
        return {"at": at, "bytes": extra_b, "cells": extra_c, "n": extra_n}

    def _backfills(self, hold, r, nb) -> bool:
        """Whether request r may start now without delaying the held request: it
        finishes by the held request's chunk, or fits in what is left beside it
        (which it then takes)."""
        if self._chunks(r.steps) <= hold["at"]:
            return True
        if nb <= hold["bytes"] and hold["n"] >= 1 and (hold["cells"] is None or r.case.cells <= hold["cells"]):
            hold["bytes"] -= nb
            hold["n"] -= 1
            if hold["cells"] is not None:
                hold["cells"] -= r.case.cells
            return True
        return False

    @staticmethod
    def _reject(o: Outcome, now: float, why: str) -> None:
        o.ok = False
        o.completed = now
        o.rejected = why or "rejected"

    def serve(self, requests) -> ServeStats:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        stg = {r.rid: self.storage_of(r) for r in reqs}
        out = {r.rid: Outcome(r.rid, r.kind, stg[r.rid], r.case.cells, r.steps, r.arrival) for r in reqs}
        nbytes = {r.rid: state_bytes(r.case.params, stg[r.rid]) for r in reqs}
        ncells = {r.rid: r.case.cells for r in reqs}
        work = {r.rid: ncells[r.rid] * r.steps for r in reqs}
        # request id -> request, in arrival order (ids, not request equality, on the
        # hot path: comparing requests compares their arrays)
        pending = {r.rid: r for r in reqs}
        active = {}                 # instance id -> (request, bytes, steps run when admitted)
        solos = {}                  # id ("solo", request id) -> [context, steps done]
        used_bytes = 0
        used_cells = 0
        steps_run = 0               # steps every resident instance has been offered so far
        st = ServeStats()
        t0 = self.clock()
        while pending or active:
            now = self.clock() - t0
            # admission: arrived requests while memory and the cell cap allow
            arrived = []
            for r in pending.values():
                if r.arrival > now:
                    break
                arrived.append(r)
            overdue = set()
            if self.order == "largest":
                late = [r for r in arrived if self.max_wait is not None and now - r.arrival > self.max_wait]
                overdue = {r.rid for r in late}
                rest = sorted((r for r in arrived if r.rid not in overdue), key=lambda r: -work[r.rid])
                arrived = late + rest
            hold = None  # reservation of the first overdue request that does not fit
            for r in arrived:
                nb = nbytes[r.rid]
                if nb > self.arena_bytes:
                    self._reject(out[r.rid], now, "larger than the HBM budget")
                    del pending[r.rid]
                    continue
                fits = used_bytes + nb <= self.arena_bytes and len(active) < self.max_instances and not (
                    self.max_cells is not None and active and used_cells + ncells[r.rid] > self.max_cells)
                if fits and hold is not None and not self._backfills(hold, r, nb):
                    continue
                if fits:
                    try:
                        if self.solo_min is not None and nb >= self.solo_min:
                            iid = ("solo", r.rid)
                            ctx = self.solo_factory(r, stg[r.rid])
                            try:
                                ctx.init(r.case.Q0)
                            except BaseException:
                                ctx.close()
                                raise
                            solos[iid] = [ctx, 0]
                        else:
                            iid = self.b.add(r.case.params, r.case.Q0, r.steps, storage=stg[r.rid])
                    except RuntimeError as e:
                        status = getattr(e, "status", None)
                        if status == EINVAL:
                            # the library refuses the request itself (e.g. an initial
                            # state with non-positive density or pressure)
                            self._reject(out[r.rid], self.clock() - t0, str(e))
                            del pending[r.rid]
                            continue
                        # no free run of that size yet (fragmentation): wait for retirements
                        if status != ENOMEM or not active:
                            raise
                        fits = False
                        if hold is None and r.rid in overdue:
                            hold = self._reserve(r, nb, active, used_bytes, used_cells, steps_run,
                                                 fragmented=True)
                        continue
                if not fits:
                    if self.order == "fifo":
                        break
                    if hold is None and r.rid in overdue:
                        hold = self._reserve(r, nb, active, used_bytes, used_cells, steps_run)
                    continue
                del pending[r.rid]
                active[iid] = (r, nb, steps_run)
                used_bytes += nb
                used_cells += ncells[r.rid]
                out[r.rid].admitted = self.clock() - t0
            st.max_active = max(st.max_active, len(active))
            st.peak_bytes = max(st.peak_bytes, used_bytes)
            if not active:
                # idle until the next arrival
                wait = next(iter(pending.values())).arrival - (self.clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
                continue
            # one chunk (a graph replay) for everything on the device; an instance that
            # reaches its step count inside the chunk stays frozen there
            t_start = self.clock() - t0
            if len(active) > len(solos):
                self.b.run(self.chunk)
            for iid, ent in solos.items():
                k = min(self.chunk, active[iid][0].steps - ent[1])
                if k > 0:
                    # the sequential baseline's divergence check: a diagnostic
                    # record on every step that is a multiple of check_steps
                    ent[0].step(k, self.check_steps if self.stop_diverged else 0)
                    ent[1] += k
            steps_run += self.chunk
            st.chunks += 1
            self.sync()
            tnow = self.clock() - t0
            st.timeline.append((t_start, tnow, len(active), used_cells))
            for iid in list(solos):
                ctx, done = solos[iid]
                r, nb, _ = active[iid]
                diverged = False
                if self.stop_diverged:
                    recs, _ = ctx.diagnostics()
                    diverged = any(rec["nonfinite"] > 0 for rec in recs)
                if not diverged and done < r.steps:
                    continue
                del active[iid], solos[iid]
                o = out[r.rid]
                o.completed = tnow
                if diverged:
                    o.ok = False
                    st.stopped += 1
                else:
                    res = self.handle(r, ctx.moments())
                    o.ok = bool(res) if isinstance(res, (bool, np.bool_)) else True
                    o.result = res
                ctx.close()
                used_bytes -= nb
                used_cells -= ncells[r.rid]
                if diverged and self.on_failure is not None:
                    self.on_failure(r)
            for iid in [i for i in active if i not in solos and self.b.query(i)[1]]:
                r, nb, _ = active.pop(iid)
                Q = self.b.moments(iid)
                o = out[r.rid]
                o.completed = tnow
                res = self.handle(r, Q)
                o.ok = bool(res) if isinstance(res, (bool, np.bool_)) else True
                o.result = res
                self.b.remove(iid)
                used_bytes -= nb
                used_cells -= ncells[r.rid]
            if self.check is not None and len(active) > len(solos) and st.chunks % self.check_chunks == 0:
                for iid in self.check():
                    if iid not in active:
                        continue
                    r, nb, _ = active.pop(iid)
                    o = out[r.rid]
                    o.completed = tnow
                    o.ok = False
                    self.b.remove(iid)
                    used_bytes -= nb
                    used_cells -= ncells[r.rid]
                    st.stopped += 1
                    if self.on_failure is not None:
                        self.on_failure(r)
        st.wall_s = self.clock() - t0
        st.outcomes = [out[r.rid] for r in reqs]
        return st


def serve_sequential(requests, solver_factory, result_handler=None, clock=time.perf_counter,
                     sync=None, stop_diverged: bool = True, check_steps: int = 200,
                     failure_handler=None) -> ServeStats:
    """Baseline: the same requests one at a time in arrival order, each in its own
    single context made by solver_factory(params) (plain FP32).  With stop_diverged
    a request steps in pieces of check_steps, each carrying the fused diagnostic
    reduction on its first step, and one whose non-finite count is positive stops
    there as failed (the batched server's check, at the same interval).  A request
    the library refuses at initialisation (LBM_EINVAL) is rejected, as in the
    server."""
    handle = result_handler or (lambda req, Q: bool(np.isfinite(Q).all()))
    sync = sync or (lambda: None)
    reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
    st = ServeStats()
    t0 = clock()
    for r in reqs:
        now = clock() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        o = Outcome(r.rid, r.kind, 0, r.case.cells, r.steps, r.arrival)
        st.outcomes.append(o)
        st.max_active = 1
        o.admitted = clock() - t0
        with solver_factory(r.case.params) as s:
            try:
                s.init(r.case.Q0)
            except RuntimeError as e:
                if getattr(e, "status", None) != EINVAL:
                    raise
                Server._reject(o, clock() - t0, str(e))
                continue
            diverged = False
            if stop_diverged:
                done = 0
                while done < r.steps and not diverged:
                    k = min(int(check_steps), r.steps - done)
                    s.step(k, int(check_steps))
                    done += k
                    recs, _ = s.diagnostics()
                    diverged = any(rec["nonfinite"] > 0 for rec in recs)
            else:
                s.step(r.steps)
            sync()
            Q = None if diverged else s.moments()
        o.completed = clock() - t0
        if diverged:
            st.stopped += 1
            if failure_handler is not None:
                failure_handler(r)
            continue
        res = handle(r, Q)
        o.ok = bool(res) if isinstance(res, (bool, np.bool_)) else True
        o.result = res
    st.wall_s = clock() - t0
    return st
