"""Continuous-batching service for space-homogeneous relaxation problems.

A request is one cell's distribution f0 on an N x N velocity grid, a
collision kernel and a number of time steps of d f/dt = Q(f)/eps (section
3.4; explicit Euler by default). Requests of different N and kernels run side
by side on one GPU:

  * residency: each (N, kernel) group keeps its live cells contiguous in one
    device buffer (its pool of f slots and their status flags; one plan per
    group); f stays on the device between steps;
  * admission by HBM footprint: the budget is charged with the device bytes
    the pools really hold (their capacity, as the caching allocator rounds
    it), including the moment a pool grows, when the old and the new buffer
    are both alive. A request is admitted when its group has a free slot, or
    when the pool can grow within the budget (pools of idle groups are
    released first); otherwise it waits in a FIFO queue and is admitted as
    soon as slots or memory free up;
  * scheduling: every tick advances every live request by one step in ONE
    batched launch over all groups (qcoll_step_multi), then retires finished
    requests (copy to pinned host memory, compaction of the pool) and admits
    waiting ones; the host work of tick k + 1 overlaps the device work of
    tick k (flags and results are read one tick later);
  * faults: a cell whose update became non-finite is flagged by the kernel
    and evicted without affecting the others;
  * small groups: a group with few live cells runs in the transform split form
    (qcoll_plan_set_split: a cell's transforms shared by several wavefronts or
    workgroups), so a tick over a few large-grid requests fills more of the GPU.
    The split factor follows the group's size, and it changes the order of a
    step's FP64 gain sum, so a request's result may then differ from that of a
    lone run in the last FP32 bits; Server(split=False) keeps every result
    independent of what ran beside it, bitwise.

Latency is completion time minus arrival time on the host monotonic clock.
All device work is done by the HIP library through the binding.
"""

from __future__ import annotations

import collections
import ctypes
import dataclasses
import time

import numpy as np

from . import qcoll


@dataclasses.dataclass
class Request:
    rid: int
    N: int
    kernel: str
    steps: int
    f0: np.ndarray           # float32 [N, N]
    arrival: float = 0.0     # seconds on the service clock


@dataclasses.dataclass
class Result:
    rid: int
    f: np.ndarray | None
    arrival: float
    admitted: float
    done: float
    failed: bool = False

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def _alloc_bytes(nbytes: int) -> int:
    """Bytes the caching allocator hands out for a request of nbytes (blocks
    are multiples of 512 bytes)."""
    return -(-int(nbytes) // 512) * 512


class _Group:
    """Live requests of one (N, kernel): f slots [cap][N][N] float32 and their
    status flags [cap] int32 in one device buffer."""

    def __init__(self, plan: qcoll.Plan, N: int, device):
        self.plan, self.N, self.device = plan, N, device
        self.tile = plan.tile()[0]
        self.fx16 = plan.precision == "fx16"
        self.split = 1
        self.cap = 0
        self.buf = None
        self.pool = None
        self.status = None
        self.live: list[int] = []          # request id of slot i
        self.left: list[int] = []          # steps remaining for slot i

    def set_split_for(self, cells: int) -> None:
        """Split factor for a step over `cells` cells, from measured step times
        of lone groups: a tile-64 cell (one workgroup unsplit) runs as 8 parts
        up to 8 cells, 4 up to 48 and 2 up to 112 (beyond that the chip is
        full enough unsplit); a 32x32 FX16 cell (one wavefront unsplit) runs as
        a workgroup of four wavefronts up to 640 cells."""
        if self.tile == 64:
            s = 8 if cells <= 8 else (4 if cells <= 48 else (2 if cells <= 112 else 1))
        elif self.tile == 32 and self.fx16:
            s = 4 if cells <= 640 else 1
        else:
            s = 1
        if s != self.split:
            self.plan.set_split(s)
            self.split = s

    @staticmethod
    def footprint(N: int, cap: int) -> int:
        return _alloc_bytes(cap * (4 * N * N + 4)) if cap > 0 else 0

    @property
    def bytes(self) -> int:
        return self.footprint(self.N, self.cap)

    def resize(self, cap: int):
        """Move the live slots into a buffer of `cap` slots (cap >= live); cap 0
        releases the buffer."""
        import torch
        assert cap >= len(self.live)
        if cap == 0:
            self.buf = self.pool = self.status = None
            self.cap = 0
            return
        nn = self.N * self.N
        buf = torch.empty(cap * nn + cap, dtype=torch.float32, device=self.device)
        pool = buf[:cap * nn].view(cap, self.N, self.N)
        if self.live:
            pool[:len(self.live)].copy_(self.pool[:len(self.live)])
        self.buf, self.pool, self.cap = buf, pool, cap
        self.status = buf[cap * nn:].view(torch.int32)


class Server:
    """Continuous-batching scheduler over qcoll_step_multi."""

    def __init__(self, L: float = 8.0, M: int = 8, precision: str = "fx16", dt: float = 0.01,
                 eps: float = 1.0, scheme: str = "explicit", budget_bytes: int = 256 << 20,
                 max_slots: int = 1 << 16, device=None, split: bool = True):
        import torch
        self.L, self.M, self.precision = L, M, precision
        self.split = split                 # transform split for groups with few live cells
        self.dt, self.eps, self.scheme = dt, eps, scheme
        self.budget = int(budget_bytes)
        self.max_slots = max_slots
        self.device = device or torch.device("cuda:0")
        self.groups: dict[tuple[int, str], _Group] = {}
        self.queue: collections.deque[Request] = collections.deque()
        self.results: dict[int, Result] = {}
        self.bytes_charged = 0             # device bytes of all pools
        self.peak_bytes = 0                # largest footprint, growth transients included
        self.waited: set[int] = set()      # requests that were queued behind a full budget or pool
        self.ticks = 0
        self.cell_steps = 0
        self._pending = None               # the previous tick, completed by the next tick or flush()
        self._admit_time: dict[int, float] = {}
        self._flags = [None, None]         # pinned status buffers of alternate ticks
        self._events = [None, None]        # and their completion events
        self._scheme = qcoll._SCHEMES[scheme]

    # ----------------------------------------------------------- admission
    def _group(self, N: int, kernel: str) -> _Group:
        key = (N, kernel)
        if key not in self.groups:
            plan = qcoll.Plan(2, N, self.L, kernel, self.M, precision=self.precision)
            self.groups[key] = _Group(plan, N, self.device)
        return self.groups[key]

    def submit(self, req: Request) -> None:
        need = _Group.footprint(req.N, 1)
        if need > self.budget:
            raise ValueError(f"request {req.rid} needs {need} B, more than the whole budget")
        self.queue.append(req)

    def _grow(self, g: _Group, need: int) -> bool:
        """Give g room for `need` slots within the budget: double its capacity
        if that fits (old and new buffer are alive together while the live
        slots move), else as many slots as fit; release idle pools first when
        even `need` does not fit."""
        if g.cap >= need:
            return True
        for attempt in range(2):
            room = self.budget - self.bytes_charged   # the old pool stays charged during the move
            cap = max(need, 2 * g.cap, 8)
            while cap > need and _Group.footprint(g.N, cap) > room:
                cap = max(need, cap * 3 // 4 if cap * 3 // 4 < cap else cap - 1)
            if _Group.footprint(g.N, cap) <= room:
                old = g.bytes
                self.peak_bytes = max(self.peak_bytes, self.bytes_charged + _Group.footprint(g.N, cap))
                g.resize(cap)
                self.bytes_charged += g.bytes - old
                return True
            if attempt == 0:   # release the pools of groups without live requests
                idle = [h for h in self.groups.values() if h is not g and not h.live and h.cap > 0]
                if not idle:
                    return False
                for h in idle:
                    self.bytes_charged -= h.bytes
                    h.resize(0)
        return False

    def _try_admit(self, now: float) -> None:
        import torch
        while self.queue:
            req = self.queue[0]
            g = self._group(req.N, req.kernel)
            if len(g.live) >= self.max_slots or not self._grow(g, len(g.live) + 1):
                self.waited.update(r.rid for r in self.queue)
                return  # FIFO: the head waits for slots or memory to free up
            self.queue.popleft()
            g.pool[len(g.live)].copy_(torch.from_numpy(np.ascontiguousarray(req.f0, dtype=np.float32)))
            g.live.append(req.rid)
            g.left.append(req.steps)
            self.peak_bytes = max(self.peak_bytes, self.bytes_charged)
            self._admit_time[req.rid] = now
            self.results[req.rid] = Result(req.rid, None, req.arrival, now, float("nan"))

    # ---------------------------------------------------------------- tick
    def _compact(self, g: _Group, gone: list[int]) -> None:
        """Free slots `gone` of group g: move the last live slots into the holes
        (device copies, ordered on the stream after everything queued so far)."""
        for i in sorted(gone, reverse=True):
            last = len(g.live) - 1
            if i != last:
                g.pool[i].copy_(g.pool[last])
                g.live[i], g.left[i] = g.live[last], g.left[last]
            g.live.pop()
            g.left.pop()

    def tick(self, clock) -> int:
        """One batched step of every live request. The step's status flags and
        the results of the requests it finishes are copied to pinned host
        memory asynchronously and handed out by the next tick (or flush()), so
        the host prepares tick k + 1 while the device runs tick k. Returns the
        number of requests retired by the previous tick."""
        import torch
        groups = [g for g in self.groups.values() if g.live]
        new = None
        if groups:
            if self.split:
                for g in groups:
                    g.set_split_for(len(g.live))
            stream = torch.cuda.current_stream()
            # the batched step through the C ABI (the pools are this server's own
            # contiguous device buffers: the binding's per-tensor checks are skipped)
            n = len(groups)
            counts = [len(g.live) for g in groups]
            total = sum(counts)
            PtrArr = ctypes.c_void_p * n
            qcoll._check(qcoll.LIB.qcoll_step_multi(
                PtrArr(*[g.plan._h.value for g in groups]), n, PtrArr(*[g.pool.data_ptr() for g in groups]),
                (ctypes.c_int64 * n)(*counts), self.dt, self.eps, self._scheme,
                PtrArr(*[g.status.data_ptr() for g in groups]), ctypes.c_void_p(stream.cuda_stream)),
                "qcoll_step_multi")
            self.ticks += 1
            self.cell_steps += total
            # status flags straight into pinned host memory (no device temporary);
            # alternate ticks use alternate buffers (the previous tick's is read
            # by flush() after this tick's copies are queued)
            b = self.ticks & 1
            if self._flags[b] is None or self._flags[b].numel() < total:
                self._flags[b] = torch.empty(max(total, 256) * 2, dtype=torch.int32, pin_memory=True)
            flags = self._flags[b][:total]
            k = 0
            for g, c in zip(groups, counts):
                flags[k:k + c].copy_(g.status[:c], non_blocking=True)
                k += c
            slots = [(g, list(g.live)) for g in groups]   # request of each slot in this step
            finished = []
            for g in groups:
                for i in range(len(g.live)):
                    g.left[i] -= 1
                done = [i for i in range(len(g.live)) if g.left[i] <= 0]
                if not done:
                    continue
                host = torch.empty((len(done), g.N, g.N), dtype=torch.float32, pin_memory=True)
                for j, i in enumerate(done):
                    host[j].copy_(g.pool[i], non_blocking=True)
                    finished.append((g.live[i], host, j))
                self._compact(g, done)
            if self._events[b] is None:
                self._events[b] = torch.cuda.Event()
            ev = self._events[b]
            ev.record(stream)
            new = (ev, flags, slots, finished)
        retired = self.flush(clock)
        self._pending = new
        return retired

    def flush(self, clock) -> int:
        """Complete the previous tick: wait for it, hand out the results of the
        requests it finished and evict live requests that its status flags mark
        non-finite (a non-finite cell stays non-finite, so a request that
        finished since is flagged again by its own last step). Returns the number
        of requests retired."""
        p, self._pending = self._pending, None
        if p is None:
            return 0
        ev, flags, slots, finished = p
        ev.synchronize()
        now = clock()
        fl = flags.numpy()
        bad, k = set(), 0
        if fl.any():   # (the common case has no flagged cell)
            for g, rids in slots:
                bad.update(rid for i, rid in enumerate(rids) if fl[k + i] != 0)
                k += len(rids)
        for rid, host, j in finished:
            r = self.results[rid]
            r.failed = rid in bad
            r.f = None if r.failed else host[j].numpy().copy()
            r.done = now
        retired = len(finished)
        for g, rids in (slots if bad else ()):
            gone = [g.live.index(rid) for rid in rids if rid in bad and rid in g.live]
            for i in gone:
                r = self.results[g.live[i]]
                r.failed, r.f, r.done = True, None, now
            if gone:
                self._compact(g, gone)
                retired += len(gone)
        return retired

    # ----------------------------------------------------------------- run
    def run(self, requests: list[Request], realtime: bool = True, poll: float = 2e-4) -> dict:
        """Serve requests arriving at their `arrival` times (open loop). With
        realtime=False the clock is virtual and advances by the measured tick
        time (deterministic admission order for tests)."""
        import torch
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        t0 = time.monotonic()
        vclock = [0.0]
        clock = (lambda: time.monotonic() - t0) if realtime else (lambda: vclock[0])
        i = 0
        pending = len(reqs)
        while pending:
            now = clock()
            while i < len(reqs) and reqs[i].arrival <= now:
                self.submit(reqs[i])
                i += 1
            self._try_admit(now)
            if any(g.live for g in self.groups.values()) or self._pending is not None:
                ts = time.monotonic()
                pending -= self.tick(clock if realtime else (lambda: vclock[0]))
                if not realtime:
                    vclock[0] += time.monotonic() - ts
            elif i < len(reqs):
                if realtime:
                    time.sleep(min(poll, max(0.0, reqs[i].arrival - clock())))
                else:
                    vclock[0] = max(vclock[0], reqs[i].arrival)
            elif self.queue:
                raise RuntimeError("queued requests cannot be admitted")
        torch.cuda.synchronize()
        return self.stats(clock())

    def stats(self, wall: float) -> dict:
        lat = np.array([r.latency for r in self.results.values() if not r.failed])
        ok = len(lat)
        return {
            "requests": len(self.results),
            "failed": sum(r.failed for r in self.results.values()),
            "p50_latency_s": float(np.percentile(lat, 50)) if ok else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if ok else None,
            "throughput_req_s": ok / wall if wall > 0 else None,
            "cell_steps_s": self.cell_steps / wall if wall > 0 else None,
            "ticks": self.ticks,
            "peak_bytes": self.peak_bytes,
            "budget_bytes": self.budget,
            "waited": len(self.waited),
            "wall_s": wall,
        }

    def close(self):
        for g in self.groups.values():
            g.plan.close()


def poisson_requests(n: int, rate: float, seed: int, L: float = 8.0, sizes=(16, 24, 32, 48, 64),
                     kernels=("maxwell", "hard_sphere"), steps=(50, 400)) -> list[Request]:
    """Open-loop Poisson arrivals with N, kernel and step count drawn uniformly;
    f0 is a two-Maxwellian mixture (the same generator as the batch workloads)."""
    import workloads as wl
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    out = []
    for k in range(n):
        N = int(rng.choice(sizes))
        kern = str(rng.choice(kernels))
        st = int(rng.integers(steps[0], steps[1] + 1))
        f0 = wl.mixture_cells(2, N, L, 1, seed * 100003 + k)[0].astype(np.float32)
        out.append(Request(k, N, kern, st, f0, float(t[k])))
    return out
