"""Continuous-batching solve server for mixed (d, n, p) Poisson solves.

Requests (right-hand side already in device memory) arrive over time.  The
server keeps one resident plan per problem shape (tables on the device) with
a resident PCG state of several slots (iffd_pcg_state_*), admits a request
into a free slot of its shape as soon as the HBM budget allows, advances every
shape's active slots by a few PCG iterations per round on that shape's own
stream (so different shapes overlap on the device and same-shape solves share
one launch per kernel; a round is one replay of a HIP graph captured when the
shape's entry is created), and hands a solution back as soon as its slot
converges.  A slot's arithmetic does not depend on the other slots, so a
request gives the same bits alone and in the mix.

Admission by footprint: a shape's entry costs its plan tables plus its state
(fixed part + per-slot part, both queried from the library); a request also
holds its result buffer (8 N bytes) while in flight.  An entry with no active
slot may be evicted (least recently used) to make room for another shape.  A
request that cannot fit even alone is rejected.

The measurement driver (Poisson arrivals, QPS sweep, latency percentiles)
is bench.py --serve.
"""

from __future__ import annotations

import collections
import math
import time

from . import PcgState, Plan


class _Entry:
    def __init__(self, key, slots, tune, device, k, graphs):
        import torch
        d, n, p = key
        self.key = key
        self.plan = Plan(d, n, p, method="fft", precision="f32", max_rhs=slots, device=device)
        if tune:
            self.plan.tune(reps=5)
        self.state = PcgState(self.plan, slots)
        self.stream = torch.cuda.Stream(device=self.plan.device)
        self.slots = slots
        self.free = list(range(slots))[::-1]
        self.busy = {}                      # slot -> request
        self.last_used = 0.0
        # asynchronous status: device records -> pinned host copy -> event
        self.dstat = torch.empty((slots, 4), dtype=torch.float64, device=self.plan.device)
        self.hstat = torch.empty((slots, 4), dtype=torch.float64, pin_memory=True)
        self.ev = torch.cuda.Event()
        self.inflight = False
        self.watch = ()                     # slots that were busy at the last launch
        self.bytes = self.plan.tables.numel() + self.state.buf.numel()
        # k PCG iterations over every slot, captured once as a HIP graph (the
        # kernels read the per-slot active flags on the device, so the same
        # graph serves any mix of busy and free slots); one launch per round
        self.k = k
        self.graph = None
        if graphs:
            g = torch.cuda.CUDAGraph()
            cap = torch.cuda.Stream(device=self.plan.device)
            cap.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(cap):
                with torch.cuda.graph(g, stream=cap):
                    self.state.iterate(k)
            torch.cuda.current_stream().wait_stream(cap)
            self.graph = g

    def iterate(self):
        import torch
        if self.graph is not None:
            with torch.cuda.stream(self.stream):
                self.graph.replay()
        else:
            self.state.iterate(self.k, stream=self.stream)


class Request:
    __slots__ = ("rid", "arrival", "d", "n", "p", "f", "u", "t_admit", "t_done", "status",
                 "iterations", "relres", "key")

    def __init__(self, rid, arrival, d, n, p, f):
        self.rid, self.arrival, self.d, self.n, self.p, self.f = rid, arrival, d, n, p, f
        self.key = (d, n, p)
        self.u = None
        self.t_admit = self.t_done = None
        self.status = None
        self.iterations = 0
        self.relres = math.nan


class SolveServer:
    """hbm_budget: bytes the server may hold (plans, states, result buffers).
    slots: PCG slots per shape.  iters_per_round: PCG iterations enqueued per
    shape between two polls.  graphs: replay each shape's round from a HIP
    graph (else launch its kernels one by one)."""

    def __init__(self, hbm_budget: int, slots: int = 8, iters_per_round: int = 2,
                 rtol: float = 1e-8, maxit: int = 200, tune: bool = False, device="cuda",
                 graphs: bool = True):
        self.budget = int(hbm_budget)
        self.slots = slots
        self.k = iters_per_round
        self.rtol, self.maxit = rtol, maxit
        self.tune = tune
        self.device = device
        self.graphs = graphs
        self.entries = collections.OrderedDict()   # key -> _Entry (LRU order)
        self.used = 0
        self.peak = 0
        self.rejected = []
        self.launches = 0        # iterate launches (one shape each)
        self.busy_slots_at_launch = 0   # sum over launches of the busy slots
        self.inflight_at_launch = 0      # sum over launches of the shapes in flight

    # ---- footprint --------------------------------------------------------------
    _sizes = {}

    @classmethod
    def entry_bytes(cls, key, slots):
        """Device bytes of a shape's entry (plan tables + PCG state) and N,
        from the library's size queries (host only)."""
        if (key, slots) in cls._sizes:
            return cls._sizes[(key, slots)]
        import ctypes
        from . import _Info, _Opts, lib, METHOD_FFT, PREC_F32
        h = ctypes.c_void_p()
        if lib.iffd_plan_create(ctypes.byref(h), key[0], key[1], key[2],
                                ctypes.byref(_Opts(METHOD_FFT, PREC_F32, slots))) != 0:
            cls._sizes[(key, slots)] = (None, None)
            return None, None
        info = _Info()
        lib.iffd_plan_query(h, ctypes.byref(info))
        lib.iffd_plan_destroy(h)
        need = info.table_bytes + info.state_bytes_fixed + slots * info.state_bytes_per_slot
        cls._sizes[(key, slots)] = (need, info.N)
        return need, info.N

    def _entry_for(self, key, now):
        e = self.entries.get(key)
        if e is not None:
            self.entries.move_to_end(key)
            return e
        need, N = self.entry_bytes(key, self.slots)
        if need is None:
            return None
        need += 8 * N          # the entry is only worth creating with room for one request
        # evict idle shapes (least recently used first) until the entry fits,
        # and none at all when evicting every idle shape would not make room
        idle = [k for k, old in self.entries.items() if not old.busy and not old.inflight]
        if self.used - sum(self.entries[k].bytes for k in idle) + need > self.budget:
            return None
        for k in idle:
            if self.used + need <= self.budget:
                break
            self.used -= self.entries[k].bytes
            del self.entries[k]
        e = _Entry(key, self.slots, self.tune, self.device, self.k, self.graphs)
        self.entries[key] = e
        self.used += e.bytes
        self.peak = max(self.peak, self.used)
        e.last_used = now
        return e

    def fits_alone(self, req):
        need, N = self.entry_bytes(req.key, self.slots)
        return need is not None and need + 8 * N <= self.budget

    def _admit(self, req, now):
        import torch
        e = self._entry_for(req.key, now)
        if e is None or not e.free:
            return False
        nbytes = 8 * e.plan.N
        if self.used + nbytes > self.budget:
            return False
        slot = e.free.pop()
        req.u = torch.empty(e.plan.shape, dtype=torch.float64, device=e.plan.device)
        e.stream.wait_stream(torch.cuda.current_stream())   # f and u are ready
        e.state.begin([slot], req.f, rtol=self.rtol, maxit=self.maxit, stream=e.stream)
        self.used += nbytes
        self.peak = max(self.peak, self.used)
        e.busy[slot] = req
        req.t_admit = now
        return True

    # ---- the loop ----------------------------------------------------------------
    def _launch(self, e):
        """Enqueue k iterations of every busy slot of a shape and an
        asynchronous copy of its slot records; never waits."""
        import torch
        e.iterate()
        e.state.status_async(e.dstat, stream=e.stream)
        with torch.cuda.stream(e.stream):
            e.hstat.copy_(e.dstat, non_blocking=True)
        e.ev.record(e.stream)
        e.watch = tuple(e.busy)
        e.inflight = True
        self.launches += 1
        self.busy_slots_at_launch += len(e.busy)
        self.inflight_at_launch += sum(1 for x in self.entries.values() if x.inflight)

    def _complete(self, e, t0, clock, done):
        """The shape's last launch has finished: hand back converged slots."""
        e.inflight = False
        st = e.hstat.numpy()
        fin = [s for s in e.watch if s in e.busy and st[s, 0] == 0.0]
        reqs = []
        for s in fin:
            r = e.busy.pop(s)
            e.state.take(s, out=r.u, stream=e.stream)
            r.status = int(st[s, 1])
            r.iterations = int(st[s, 2])
            r.relres = float(st[s, 3])
            e.free.append(s)
            reqs.append(r)
        if reqs:
            e.stream.synchronize()          # the copies out are done
            tnow = clock() - t0
            for r in reqs:
                r.t_done = tnow
                self.used -= 8 * r.u.numel()          # result handed back
                done.append(r)
        e.last_used = clock() - t0

    def run(self, requests, clock=time.perf_counter):
        """Serve `requests` (arrival in seconds from the start).  Each shape
        advances on its own stream as soon as its previous launch finished;
        new requests join free slots between launches.  Returns the requests
        (finished or rejected) with t_admit / t_done / status filled in."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = []
        t0 = clock()
        done = []
        while pending or queue or any(e.busy or e.inflight for e in self.entries.values()):
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                if not self.fits_alone(r):
                    r.status = "rejected"
                    self.rejected.append(r)
                    done.append(r)
                else:
                    queue.append(r)
            # admit in arrival order; a request that does not fit waits
            if queue:
                queue = [r for r in queue if not self._admit(r, now)]
            for e in list(self.entries.values()):
                if e.busy and not e.inflight:
                    self._launch(e)
            progressed = False
            for e in list(self.entries.values()):
                if e.inflight and e.ev.query():
                    self._complete(e, t0, clock, done)
                    progressed = True
            if not progressed:
                time.sleep(0.00005)
        return done
