"""Continuous-batching server for factored FIO solves.

Requests (a right-hand-side block for one factor key: dimension, n, phase, eps)
arrive over time.  Factors of every key stay resident on the GPU.  The scheduler
keeps one queue per key; whenever a key has no batch on the device, all its
queued requests (up to ``max_batch_rhs`` columns) are merged into one batch and
started on a free stream, if the batch's buffers fit the HBM budget.  Batches of
different keys run concurrently on different streams, so requests that arrive
while others are on the GPU are admitted as soon as their key's slot and the
memory free up.  Every request's latency (arrival to result in host memory) is
recorded.

The scheduler talks to an executor with three calls (``footprint``, ``start``,
``poll``); ``GpuExecutor`` runs batches through the C ABI (``fio_solve``), and
``MockExecutor`` completes them after a modelled duration so the scheduling,
admission and accounting logic can be tested on a CPU.
"""
from __future__ import annotations

import collections
import dataclasses
import heapq
import time

import numpy as np


@dataclasses.dataclass
class ServeRequest:
    rid: int
    key: tuple            # (d, n, phase, eps)
    arrival: float        # seconds, on the server clock
    u: np.ndarray         # (N, nrhs) complex128
    result: np.ndarray | None = None
    start: float | None = None
    done: float | None = None
    error: str | None = None   # set when the request was cancelled or its batch failed

    @property
    def nrhs(self) -> int:
        return self.u.shape[1]

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclasses.dataclass
class Batch:
    key: tuple
    requests: list
    nrhs: int
    bytes: int
    handle: object = None


class Scheduler:
    """Continuous batching with HBM-footprint admission over an executor."""

    def __init__(self, executor, hbm_budget: int, max_batch_rhs: int = 256,
                 max_inflight: int = 8):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_batch_rhs = max_batch_rhs
        # never more batches in flight than the executor can run side by side
        self.max_inflight = min(max_inflight, getattr(executor, "max_concurrent", max_inflight))
        self.queues = collections.defaultdict(collections.deque)
        self.running = {}           # key -> Batch
        self.resident = 0           # bytes of resident factors and workspaces
        self.inflight_bytes = 0
        self.finished = []
        self.batches_started = 0
        self.groups_started = 0      # multi-instance launches of several batches
        self.peak_inflight = 0
        self.rejected_keys = []
        self.failed = []             # requests whose batch the executor could not run
        self.cancelled = []          # requests withdrawn by cancel()
        self._cancel_ids = set()     # cancelled while their batch runs

    # ---------------------------------------------------------------- keys
    def register(self, key) -> bool:
        """Make a key's factors resident if they fit the budget (else refuse it)."""
        need = self.ex.resident_bytes(key)
        if self.resident + need > self.budget:
            self.rejected_keys.append(key)
            return False
        self.ex.load(key)
        self.resident += need
        return True

    # ---------------------------------------------------------------- loop
    def check(self, req: ServeRequest):
        """A request wider than max_batch_rhs columns could never be batched (the
        executor's buffers and graphs stop there): it is refused, as is an empty one."""
        if req.nrhs > self.max_batch_rhs:
            raise ValueError("request %s has %d right-hand sides, more than max_batch_rhs = %d"
                             % (req.rid, req.nrhs, self.max_batch_rhs))
        if req.nrhs < 1:
            raise ValueError("request %s has no right-hand side" % (req.rid,))

    def submit(self, req: ServeRequest):
        self.check(req)
        self.queues[req.key].append(req)

    def cancel(self, rid) -> bool:
        """Withdraw a request.  A queued one leaves its queue at once; one whose batch
        already runs is dropped when the batch completes (the other requests of the
        batch are unaffected).  Returns False if the request is unknown or done."""
        for q in self.queues.values():
            for r in q:
                if r.rid == rid:
                    q.remove(r)
                    self._withdraw(r, "cancelled")
                    return True
        for b in self.running.values():
            if any(r.rid == rid for r in b.requests):
                self._cancel_ids.add(rid)
                return True
        return False

    def _withdraw(self, r, why):
        r.error = why
        r.done = self.ex.clock()
        (self.cancelled if why == "cancelled" else self.failed).append(r)

    def _fail_batch(self, b, exc):
        """The executor raised for batch b: its requests fail with the error and its
        memory is released; the loop goes on with the other keys."""
        for r in b.requests:
            self._cancel_ids.discard(r.rid)
            self._withdraw(r, "%s: %s" % (type(exc).__name__, exc))
        self.inflight_bytes -= b.bytes

    def _form_batch(self, key):
        """The key's queued requests in arrival order, up to the executor's column cap
        for the key (``batch_cap``, a bound on one batch's device time, so that a large
        key's batches do not hold the device, and the requests behind them, for long)
        and ``max_batch_rhs``; the first request is always taken."""
        q = self.queues[key]
        cap = self.max_batch_rhs
        if hasattr(self.ex, "batch_cap"):
            cap = min(cap, self.ex.batch_cap(key))
        first = q.popleft()
        reqs, cols = [first], first.nrhs
        while q and cols + q[0].nrhs <= cap:
            r = q.popleft()
            reqs.append(r)
            cols += r.nrhs
        return Batch(key, reqs, cols, self.ex.footprint(key, cols))

    def step(self, now: float):
        """Start every admissible batch, oldest waiting request first, then collect
        the finished ones.  Batches admitted in the same step go to the executor
        together (``start_group``) when it can run them as one multi-instance solve."""
        ready = [k for k, q in self.queues.items() if q and k not in self.running]
        ready.sort(key=lambda k: self.queues[k][0].arrival)
        admitted = []
        for key in ready:
            if len(self.running) + len(admitted) >= self.max_inflight:
                break
            b = self._form_batch(key)
            if self.resident + self.inflight_bytes + b.bytes > self.budget:
                for r in reversed(b.requests):  # not admitted: back to the queue head
                    self.queues[key].appendleft(r)
                continue
            for r in b.requests:
                r.start = now
            self.inflight_bytes += b.bytes
            admitted.append(b)
        if admitted:
            if len(admitted) > 1 and hasattr(self.ex, "start_group"):
                try:
                    handles = self.ex.start_group(admitted, now)
                    self.groups_started += 1
                except Exception as exc:  # noqa: BLE001 - the group's batches fail, the loop goes on
                    for b in admitted:
                        self._fail_batch(b, exc)
                    admitted, handles = [], []
            else:
                handles = []
                for b in list(admitted):
                    try:
                        handles.append(self.ex.start(b, now))
                    except Exception as exc:  # noqa: BLE001 - the batch fails, the loop goes on
                        self._fail_batch(b, exc)
                        admitted.remove(b)
            for b, h in zip(admitted, handles):
                b.handle = h
                self.running[b.key] = b
                self.batches_started += 1
            self.peak_inflight = max(self.peak_inflight, len(self.running))
        for key, b in list(self.running.items()):
            try:
                res = self.ex.poll(b.handle, now)
            except Exception as exc:  # noqa: BLE001
                del self.running[key]
                self._fail_batch(b, exc)
                continue
            if res is None:
                continue
            t = self.ex.clock()
            c0 = 0
            for r in b.requests:
                if r.rid in self._cancel_ids:  # withdrawn while running: result dropped
                    self._cancel_ids.discard(r.rid)
                    self._withdraw(r, "cancelled")
                else:
                    r.result = res[:, c0:c0 + r.nrhs]
                    r.done = t
                    self.finished.append(r)
                c0 += r.nrhs
            del self.running[key]
            self.inflight_bytes -= b.bytes

    def idle(self) -> bool:
        return not self.running and not any(self.queues.values())

    def run(self, requests, time_scale: float = 1.0, timeout: float = 600.0):
        """Replay requests at their arrival times (seconds * time_scale) until all finish."""
        pending = sorted(requests, key=lambda r: r.arrival)
        for r in pending:  # refuse a bad request before anything starts
            self.check(r)
        t0 = self.ex.clock()
        i = 0
        while True:
            now = self.ex.clock() - t0
            while i < len(pending) and pending[i].arrival * time_scale <= now:
                r = pending[i]
                r.arrival = t0 + r.arrival * time_scale
                self.submit(r)
                i += 1
            self.step(self.ex.clock())
            if i == len(pending) and self.idle():
                break
            if now > timeout:
                raise TimeoutError("serving run exceeded %.0f s" % timeout)
            self.ex.wait()
        return self.finished


def latency_stats(finished) -> dict:
    lat = np.array([r.latency for r in finished])
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "count": int(lat.size)}


def throughput(finished) -> float:
    """RHS * N per second over the span from the first arrival to the last completion."""
    t0 = min(r.arrival for r in finished)
    t1 = max(r.done for r in finished)
    work = sum(r.nrhs * r.u.shape[0] for r in finished)
    return work / max(t1 - t0, 1e-9)


# ====================================================================== executors
class MockExecutor:
    """CPU stand-in: a batch takes ``cost(key, nrhs)`` seconds of modelled time and
    returns ``transform(key, u)``; clock and waiting are virtual."""

    def __init__(self, cost, transform=None, factor_bytes=None, ws_bytes_per_rhs=None, fail_starts=(),
                 batch_caps=None):
        self.cost = cost
        if batch_caps is not None:  # per-key column caps, as GpuExecutor.batch_cap
            self.batch_cap = lambda key: batch_caps.get(key, 1 << 30)
        self.transform = transform or (lambda key, u: u.copy())
        self.factor_bytes = factor_bytes or (lambda key: 0)
        self.ws_bytes_per_rhs = ws_bytes_per_rhs or (lambda key: 0)
        self.fail_starts = set(fail_starts)  # 0-based start() calls that raise (out of memory)
        self.starts = 0
        self.t = 0.0
        self.events = []
        self.loaded = []

    def clock(self):
        return self.t

    def wait(self):
        self.t += 1e-4

    def resident_bytes(self, key):
        return self.factor_bytes(key)

    def load(self, key):
        self.loaded.append(key)

    def footprint(self, key, nrhs):
        return self.ws_bytes_per_rhs(key) * nrhs

    def start(self, batch, now):
        k = self.starts
        self.starts += 1
        if k in self.fail_starts:
            raise MemoryError("device allocation failed (modelled, start call %d)" % k)
        u = np.concatenate([r.u for r in batch.requests], axis=1)
        return (self.t + self.cost(batch.key, batch.nrhs), self.transform(batch.key, u))

    def poll(self, handle, now):
        t_done, res = handle
        return res if self.t >= t_done else None


class GpuExecutor:
    """Runs batches through the C ABI on a pool of HIP streams (default priority).

    Loading a key sizes its plan's workspace for ``max_batch_rhs`` columns and
    allocates pinned host staging for it, so nothing is allocated inside the
    library while serving.  A batch copies its right-hand sides to the device,
    runs ``fio_solve`` (complex64 applies + ``refine`` FP64 refinement steps),
    copies the result back and records an event.

    With ``use_graphs`` the solve of each key is captured once per batch-size
    bucket (a HIP graph of all its kernel launches, on static device buffers) and
    replayed; a batch is padded up to its bucket.  Columns are independent, so
    padding does not change the results.

    With ``trim`` every plan keeps only the device images the refined complex64 solve
    uses (``fio_plan_trim``), about half the factor memory, so more keys fit the HBM
    budget.

    With ``use_multi``, batches of different keys admitted together run as one
    multi-instance solve (``fio_solve_multi``: one launch per factor level for all
    of them, on one stream); with graphs, each group (its keys and buckets) is
    captured once and replayed.
    """

    BUCKETS = (16, 32, 64, 128, 256, 512, 1024)

    MULTI_MAX = 8  # instances per multi-instance solve (fio.h)

    def __init__(self, plans: dict, max_batch_rhs: int = 256, refine: int = 1, nstreams: int = 8,
                 use_graphs: bool = False, use_multi: bool = False, trim: bool = False, autotune: bool = True):
        import torch
        from . import fio as F
        self.torch, self.F = torch, F
        self.plans = plans            # key -> Plan
        self.max_batch_rhs = max_batch_rhs
        self.refine = refine
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.max_concurrent = nstreams  # one batch per stream
        self.busy = {}
        if trim:  # keep only what the refined complex64 solve uses: more keys fit in HBM
            for p in plans.values():
                F.fio_plan_trim(p, F.FIO_KEEP_REFINE_C64)
        self.stats = {k: F.fio_plan_stats(p) for k, p in plans.items()}
        self.autotune = autotune      # tune each key's kernels at its bucket widths on load
        self.use_graphs = use_graphs
        self.graphs = {}              # (key, bucket) -> (graph, U, X)
        self.stage = {}               # key -> (pinned u, pinned x)
        self.use_multi = use_multi
        self.group_graphs = {}        # ((key, bucket), ...) -> graph of the multi-instance solve
        self.group_seen = {}          # group signature -> times started

    def clock(self):
        return time.perf_counter()

    def wait(self):
        time.sleep(5e-5)

    def _N(self, key):
        return self.stats[key]["n"] ** self.stats[key]["d"]

    def _bucket(self, nrhs):
        for b in self.BUCKETS:
            if nrhs <= b:
                return b
        return nrhs

    def resident_bytes(self, key):
        s = self.stats[key]
        static = 0
        if self.use_graphs:
            static = sum(2 * self._N(key) * b * 16 for b in self.BUCKETS if b <= self._bucket(self.max_batch_rhs))
        return s["device_bytes"] + s["workspace_bytes"] * self._bucket(self.max_batch_rhs) + static

    def _solve(self, key, U, X, B, stream):
        F = self.F
        F.fio_solve(self.plans[key], F.FIO_SOLVE_REFINE, F.FIO_C64, U, X, B, self._N(key), tol=0.0,
                    maxit=self.refine, stream=stream, want_info=False)

    def load(self, key):
        torch = self.torch
        N = self._N(key)
        top = self._bucket(self.max_batch_rhs)
        U = torch.zeros((top, N), dtype=torch.complex128, device="cuda")
        X = torch.zeros_like(U)
        self._solve(key, U, X, top, torch.cuda.current_stream())  # sizes the plan's workspace
        torch.cuda.synchronize()
        if self.autotune and self.use_graphs:
            # kernel choices per batch width (the library looks them up by exact width):
            # with graphs batches run at the bucket widths, up to the key's cap; tuned for
            # the complex64 applies and the complex128 residual before any graph captures
            # the choices (eager batches run at their own widths, so they are not tuned)
            F = self.F
            cap = min(top, self.batch_cap(key))
            st = torch.cuda.current_stream()
            for b in self.BUCKETS:
                if b > cap:
                    break
                F.fio_autotune(self.plans[key], F.FIO_C64, b, 2, st)
                if self.refine > 0:
                    F.fio_autotune(self.plans[key], F.FIO_C128, b, 2, st)
            torch.cuda.synchronize()
        self.stage[key] = (torch.empty((top, N), dtype=torch.complex128).pin_memory(),
                           torch.empty((top, N), dtype=torch.complex128).pin_memory())
        if self.use_graphs:
            s = self.streams[0]
            for b in self.BUCKETS:
                if b > top:
                    break
                Ub = torch.zeros((b, N), dtype=torch.complex128, device="cuda")
                Xb = torch.zeros_like(Ub)
                with torch.cuda.stream(s):
                    self._solve(key, Ub, Xb, b, s)  # eager warm-up on the capture stream
                s.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=s):
                    self._solve(key, Ub, Xb, b, s)
                self.graphs[(key, b)] = (g, Ub, Xb)
            torch.cuda.synchronize()

    def footprint(self, key, nrhs):
        if self.use_graphs:
            return 0  # static per-bucket buffers are counted as resident
        return 2 * self._N(key) * nrhs * 16

    def _stream(self):
        used = set(id(s) for s in self.busy.values())
        for s in self.streams:
            if id(s) not in used:
                return s
        raise RuntimeError("every stream is busy: the scheduler started more batches than streams")

    def start(self, batch, now):
        torch = self.torch
        key = batch.key
        N = self._N(key)
        B = batch.nrhs
        s = self._stream()
        hu, hx = self.stage[key]
        c0 = 0
        for r in batch.requests:
            hu[c0:c0 + r.nrhs].copy_(torch.from_numpy(np.ascontiguousarray(r.u.T)))
            c0 += r.nrhs
        with torch.cuda.stream(s):
            if self.use_graphs:
                g, U, X = self.graphs[(key, self._bucket(B))]
                U[:B].copy_(hu[:B], non_blocking=True)
                g.replay()
                hx[:B].copy_(X[:B], non_blocking=True)
                keep = None
            else:
                U = torch.empty((B, N), dtype=torch.complex128, device="cuda")
                X = torch.empty_like(U)
                U.copy_(hu[:B], non_blocking=True)
                self._solve(key, U, X, B, s)
                hx[:B].copy_(X, non_blocking=True)
                keep = (U, X)
            ev = torch.cuda.Event()
            ev.record(s)
        self.busy[id(batch)] = s
        return (batch, ev, B, keep)

    def _multi(self, members, s):
        """fio_solve_multi over members [(key, U, X, columns)] on stream s."""
        F = self.F
        F.fio_solve_multi([self.plans[k] for k, _, _, _ in members], F.FIO_SOLVE_REFINE, F.FIO_C64,
                          [U for _, U, _, _ in members], [X for _, _, X, _ in members],
                          [b for _, _, _, b in members], [self._N(k) for k, _, _, _ in members],
                          maxit=self.refine, stream=s)

    GROUP_SPREAD = 4.0  # batches of one group differ in estimated work by at most this factor
    GROUP_CAPTURE_AFTER = 3  # a group (keys and column buckets) is captured on its third start

    def _work(self, batch):
        """Estimated work of a batch: butterfly nonzeros times padded columns."""
        return float(self.stats[batch.key]["bf_nnz"]) * self._bucket(batch.nrhs)

    BATCH_TARGET_MS = 24.0   # device time one batch may take, estimated
    EST_TFLOPS = 110.0       # rate of the estimate (the batched applies run at 100-130)

    def batch_cap(self, key):
        """Columns per batch of this key: the largest bucket whose estimated solve
        time stays within BATCH_TARGET_MS (a direct complex64 apply of Kd^* and Gd, and
        per refinement step a complex128 Kd at half the rate and another complex64
        apply: 8 flop per butterfly nonzero and column each, Gd neglected), at least
        the smallest bucket.  Only the largest keys are capped (2D n = 256: 64 columns,
        about 20 ms)."""
        per_col = 8.0 * self.stats[key]["bf_nnz"] * (2 + 2 * self.refine) / (self.EST_TFLOPS * 1e12) * 1e3
        cap = self.BUCKETS[0]
        for b in self.BUCKETS:
            if b <= self.max_batch_rhs and b * per_col <= self.BATCH_TARGET_MS:
                cap = b
        return cap

    def _groups(self, batches):
        """Index groups of batches of similar work (a small solve grouped with a large
        one would wait for it), at most MULTI_MAX each, keys in a fixed order."""
        order = sorted(range(len(batches)), key=lambda i: self._work(batches[i]))
        groups, cur = [], []
        for i in order:
            if cur and (len(cur) == self.MULTI_MAX or
                        self._work(batches[i]) > self.GROUP_SPREAD * self._work(batches[cur[0]])):
                groups.append(cur)
                cur = []
            cur.append(i)
        if cur:
            groups.append(cur)
        return [sorted(g, key=lambda i: batches[i].key) for g in groups]

    def start_group(self, batches, now):
        """Several batches of different keys as multi-instance solves (groups of
        similar work, up to MULTI_MAX, one stream each; a batch left alone runs its
        own solve); returns one handle per batch."""
        if not self.use_multi:
            return [self.start(b, now) for b in batches]
        torch = self.torch
        handles = [None] * len(batches)
        for idx in self._groups(batches):
            if len(idx) == 1:
                handles[idx[0]] = self.start(batches[idx[0]], now)
                continue
            s = self._stream()
            members, keep = [], []
            for i in idx:
                b = batches[i]
                hu = self.stage[b.key][0]
                c0 = 0
                for r in b.requests:
                    hu[c0:c0 + r.nrhs].copy_(torch.from_numpy(np.ascontiguousarray(r.u.T)))
                    c0 += r.nrhs
            with torch.cuda.stream(s):
                for i in idx:
                    b = batches[i]
                    if self.use_graphs:
                        _, U, X = self.graphs[(b.key, self._bucket(b.nrhs))]
                        members.append((b.key, U, X, self._bucket(b.nrhs)))
                    else:
                        U = torch.empty((b.nrhs, self._N(b.key)), dtype=torch.complex128, device="cuda")
                        X = torch.empty_like(U)
                        members.append((b.key, U, X, b.nrhs))
                        keep.append((U, X))
                    U[:b.nrhs].copy_(self.stage[b.key][0][:b.nrhs], non_blocking=True)
                sig = tuple((k, cols) for k, _, _, cols in members)
                g = self.group_graphs.get(sig)
                seen = self.group_seen.get(sig, 0) + 1
                self.group_seen[sig] = seen
                if g is None and self.use_graphs and seen >= self.GROUP_CAPTURE_AFTER:
                    # a recurring group: capture it once (a capture waits for the whole
                    # device, so rare groups run eagerly instead)
                    s.synchronize()
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g, stream=s):
                        self._multi(members, s)
                    self.group_graphs[sig] = g
                if g is not None:
                    g.replay()
                else:
                    self._multi(members, s)
                for i, (_, _, X, _) in zip(idx, members):
                    b = batches[i]
                    self.stage[b.key][1][:b.nrhs].copy_(X[:b.nrhs], non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(s)
            for i in idx:
                self.busy[id(batches[i])] = s
                handles[i] = (batches[i], ev, batches[i].nrhs, keep)
        return handles

    def poll(self, handle, now):
        batch, ev, B, keep = handle
        if not ev.query():
            return None
        self.busy.pop(id(batch), None)
        return self.stage[batch.key][1][:B].numpy().T.copy()
