"""Continuous-batching request loop for FRAM solves on one GPU.

Requests (graph pairs) arrive over time.  A pool of worker slots serves them:
each slot is a context with its own HIP stream and workspace, so the kernels
of every request in flight overlap on the device.  A request is admitted the
moment a slot is free and its device workspace fits the HBM budget that is
still free; it is never held back for other requests.

* requests whose matrix is one tile (2 <= n <= ``group_n``, 256) are taken by
  the group slot in batches: every such request waiting (up to
  ``group_max``) is solved in one fram_solve_many call, whose lockstep group
  runs all of them with one launch per kernel per outer iteration;
* other requests with n <= ``small_n`` are taken by the small slots, and by a
  large slot that finds no large request waiting;
* larger requests are taken by the large slots only, so a burst of large
  requests cannot hold up the small ones.

A slot request runs exactly the single-pair solve (fram_solve_ex), with
tile ``slot_tile`` (256 by default: the solve's SDSN grid then occupies few
compute units -- 16 workgroups at n = 1000 against 256 with the automatic
64-tiles, which fill the device for one solve alone --, so that many
requests in flight share the device; measured on the 200 req/s stream of
n in [30, 2000]: 200 solves/s with p99 0.37 s, against 130 solves/s and a
growing backlog with automatic tiles), and a grouped one the lockstep group,
whose result equals, bit for bit, the single-pair solve with the request's
one-tile edge as tile: either way a request's result is the same whether it
ran alone or in the mix.  Latency is measured
from a request's arrival to the moment its result is back on the host.  The
loop is plain Python around native calls (ctypes releases the GIL during each
call, so the slots run concurrently).

HBM budget.  A context keeps its workspace between calls (it only grows), so
the budget charges every slot for the memory its context holds, not only for
the request it runs: before a solve the slot's charge is raised to the
workspace the request needs (if the budget has room; otherwise the slot
releases its own workspace and waits for the full amount), and while any
slot waits for memory, idle slots release theirs (fram_trim).  The memory all
contexts hold therefore never exceeds the budget.

A request whose solve raises is completed with the error recorded
(``Request.error``); its slot keeps serving.
"""
from __future__ import annotations

import dataclasses
import threading
import time
from collections import deque

import numpy as np

from .fram import Context, fram_workspace_bytes, PRECISIONS


@dataclasses.dataclass
class Request:
    rid: int
    A: np.ndarray
    B: np.ndarray
    arrival: float            # seconds since the trace start
    done: float = -1.0        # completion time, same clock
    perm: np.ndarray | None = None
    objective: float = float("nan")
    stats: dict | None = None
    worker: str = ""
    error: str = ""

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def latency_ms(self) -> float:
        return 1e3 * (self.done - self.arrival)


class Budget:
    """HBM admission: a counting semaphore over bytes, with a count of the
    slots waiting for memory (idle slots release theirs while it is > 0)."""

    def __init__(self, total: int):
        self.total = int(total)
        self.free = int(total)
        self.waiting = 0
        self.cv = threading.Condition()

    def try_acquire(self, nbytes: int) -> bool:
        with self.cv:
            if self.free >= nbytes:
                self.free -= nbytes
                return True
            return False

    def acquire(self, nbytes: int, stop: threading.Event) -> bool:
        """Blocks until nbytes are free; nbytes above the total are admitted
        alone (the whole budget is taken)."""
        nbytes = min(int(nbytes), self.total)
        with self.cv:
            self.waiting += 1
            try:
                while self.free < nbytes and not stop.is_set():
                    self.cv.wait(0.01)
                if stop.is_set():
                    return False
                self.free -= nbytes
                return True
            finally:
                self.waiting -= 1

    def release(self, nbytes: int):
        with self.cv:
            self.free += int(nbytes)
            self.cv.notify_all()


class Server:
    def __init__(self, hbm_budget_bytes: int = 64 << 30, large_workers: int = 8,
                 small_workers: int = 2, small_n: int = 512, prec: str = "bf16",
                 theta: float = 2.0, iters: int = 100, tol: float = 1e-6,
                 stall_iters: int = 3, device: int = 0, context_factory=None,
                 group_n: int = 256, group_max: int = 64, slot_tile: int = 256):
        if large_workers < 1 or small_workers < 0:
            raise ValueError("need at least one large slot and no negative slot count")
        if not 0 <= group_n <= 256 or group_max < 1:
            raise ValueError("group_n must be in [0, 256] (0: no group slot), group_max >= 1")
        self.small_n = small_n
        self.group_n, self.group_max = group_n, group_max
        if slot_tile not in (0, 64, 128, 256):
            raise ValueError("slot_tile must be 0 (automatic), 64, 128 or 256")
        self.slot_tile = slot_tile
        self.opts = dict(prec=prec, stall_iters=stall_iters)
        self.theta, self.iters, self.tol = theta, iters, tol
        self.budget = Budget(hbm_budget_bytes)
        self.q_group: deque[Request] = deque()
        self.q_small: deque[Request] = deque()
        self.q_large: deque[Request] = deque()
        self.cv = threading.Condition()
        self.stop = threading.Event()
        self.completed: list[Request] = []
        self.t0 = 0.0
        make = context_factory or Context
        self.slots = [(f"small{i}", make(device), False) for i in range(small_workers)]
        self.slots += [(f"large{i}", make(device), True) for i in range(large_workers)]
        self.threads = [threading.Thread(target=self._slot_loop, args=(name, c, large),
                                         daemon=True) for name, c, large in self.slots]
        if group_n > 0:
            gc = make(device)
            self.slots.append(("group0", gc, False))
            self.threads.append(threading.Thread(target=self._group_loop, args=("group0", gc),
                                                 daemon=True))

    # ------------------------------------------------------------- clock
    def now(self) -> float:
        return time.perf_counter() - self.t0

    # ------------------------------------------------------------- bytes
    def _bytes(self, n: int) -> int:
        p = PRECISIONS[self.opts["prec"]]
        try:
            return fram_workspace_bytes(n, p)
        except (ImportError, OSError):
            np_ = (n + 31) // 32 * 32
            es = 4 if p == 0 else 2
            return 16 * n * n + 4 * np_ * np_ * (3 * es + 12)

    # ------------------------------------------------------------- API
    def start(self):
        self.t0 = time.perf_counter()
        for t in self.threads:
            t.start()

    def _grouped(self, n: int) -> bool:
        return 2 <= n <= self.group_n

    @staticmethod
    def _edge(n: int) -> int:
        return 64 if n <= 64 else (128 if n <= 128 else 256)

    def submit(self, req: Request):
        with self.cv:
            if self._grouped(req.n):
                self.q_group.append(req)
            else:
                (self.q_small if req.n <= self.small_n else self.q_large).append(req)
            self.cv.notify_all()

    def shutdown(self):
        self.stop.set()
        with self.cv:
            self.cv.notify_all()
        for t in self.threads:
            t.join()
        for _, c, _ in self.slots:
            c.close()

    # ------------------------------------------------------------- slots
    def _finish(self, req: Request, perm, obj, st, worker: str):
        req.perm, req.objective, req.stats, req.worker = perm, obj, st, worker
        req.done = self.now()
        with self.cv:
            self.completed.append(req)
            self.cv.notify_all()

    def _take(self, large: bool, slot: dict) -> Request | None:
        """Next request for a slot (oldest first), or None once stopped and
        drained.  While waiting, an idle slot gives its workspace back if
        another slot is waiting for memory."""
        with self.cv:
            while True:
                if large and self.q_large:
                    return self.q_large.popleft()
                if self.q_small:
                    return self.q_small.popleft()
                if self.stop.is_set():
                    return None
                if self.budget.waiting and slot["held"] > self.FIXED:
                    self.cv.release()
                    try:
                        self._trim(slot)
                    finally:
                        self.cv.acquire()
                    continue
                self.cv.wait(0.01)

    # Device memory a context holds besides its workspace (small fixed
    # buffers), charged to every slot from its first solve on.
    FIXED = 1 << 20

    def _trim(self, slot: dict):
        """Release the slot's workspace and its charge (down to FIXED)."""
        trim = getattr(slot["ctx"], "trim", None)
        if trim is not None:
            trim()
        if slot["held"] > self.FIXED:
            self.budget.release(slot["held"] - self.FIXED)
            slot["held"] = self.FIXED

    def _reserve(self, slot: dict, need: int) -> bool:
        """Raise the slot's charge to cover `need` bytes of workspace."""
        want = need + self.FIXED
        extra = want - slot["held"]
        if extra <= 0:
            return True
        if self.budget.try_acquire(extra):
            slot["held"] = want
            return True
        # Not enough room: give back this slot's own workspace, then wait for
        # the whole amount (idle slots release theirs meanwhile).
        self._trim(slot)
        if slot["held"]:
            self.budget.release(slot["held"])
            slot["held"] = 0
        if not self.budget.acquire(want, self.stop):
            return False
        slot["held"] = want
        return True

    def _slot_loop(self, name: str, ctx, large: bool):
        slot = {"ctx": ctx, "held": 0}
        try:
            while True:
                req = self._take(large, slot)
                if req is None:
                    return
                try:
                    need = self._bytes(req.n)
                except Exception as e:  # noqa: BLE001 - recorded on the request
                    req.error = f"{type(e).__name__}: {e}"
                    self._finish(req, None, float("nan"), None, name)
                    continue
                if need + self.FIXED > self.budget.total:
                    req.error = "FramError: workspace exceeds the HBM budget"
                    self._finish(req, None, float("nan"), None, name)
                    continue
                if not self._reserve(slot, need):
                    return
                try:
                    kw = dict(self.opts)
                    if self.slot_tile:
                        kw["tile"] = self.slot_tile
                    perm, obj, st = ctx.solve(req.A, req.B, theta=self.theta, iters=self.iters,
                                              tol=self.tol, sdsn_mode="auto", **kw)
                except Exception as e:  # noqa: BLE001 - recorded on the request
                    req.error = f"{type(e).__name__}: {e}"
                    perm, obj, st = None, float("nan"), None
                self._finish(req, perm, obj, st, name)
        finally:
            if slot["held"]:
                self.budget.release(slot["held"])

    def _take_group(self, slot: dict) -> list[Request] | None:
        """Every grouped request waiting (oldest first, up to group_max), or
        None once stopped and drained."""
        with self.cv:
            while True:
                if self.q_group:
                    batch = []
                    while self.q_group and len(batch) < self.group_max:
                        batch.append(self.q_group.popleft())
                    return batch
                if self.stop.is_set():
                    return None
                if self.budget.waiting and slot["held"] > self.FIXED:
                    self.cv.release()
                    try:
                        self._trim(slot)
                    finally:
                        self.cv.acquire()
                    continue
                self.cv.wait(0.01)

    def _group_loop(self, name: str, ctx):
        slot = {"ctx": ctx, "held": 0}
        try:
            while True:
                batch = self._take_group(slot)
                if batch is None:
                    return
                try:
                    # A grouped pair's workspace is at most that of its edge.
                    need = sum(self._bytes(self._edge(r.n)) for r in batch)
                except Exception as e:  # noqa: BLE001 - recorded on the requests
                    for r in batch:
                        r.error = f"{type(e).__name__}: {e}"
                        self._finish(r, None, float("nan"), None, name)
                    continue
                need = min(need, self.budget.total - self.FIXED)
                if not self._reserve(slot, need):
                    return
                try:
                    perms, objs, sts = ctx.solve_many([r.A for r in batch], [r.B for r in batch],
                                                      theta=self.theta, iters=self.iters,
                                                      tol=self.tol, **self.opts)
                except Exception:  # noqa: BLE001 - one request spoils the call
                    # The call stops at its first failing pair: solve the
                    # batch one by one (each with its edge as tile, which is
                    # what the group computes), so only the failing requests
                    # carry an error.
                    for r in batch:
                        try:
                            p_, o_, st = ctx.solve(r.A, r.B, theta=self.theta, iters=self.iters,
                                                   tol=self.tol, tile=self._edge(r.n),
                                                   **self.opts)
                        except Exception as e:  # noqa: BLE001 - recorded on the request
                            r.error = f"{type(e).__name__}: {e}"
                            p_, o_, st = None, float("nan"), None
                        self._finish(r, p_, o_, st, name)
                    continue
                for r, p_, o_, st in zip(batch, perms, objs, sts):
                    self._finish(r, p_, o_, st, name)
        finally:
            if slot["held"]:
                self.budget.release(slot["held"])

    # ------------------------------------------------------------- trace replay
    def replay(self, requests: list[Request], timeout_s: float = 600.0) -> list[Request]:
        """Submit each request at its arrival time; wait for all results."""
        self.start()
        for r in sorted(requests, key=lambda r: r.arrival):
            delay = r.arrival - self.now()
            if delay > 0:
                time.sleep(delay)
            self.submit(r)
        deadline = time.perf_counter() + timeout_s
        with self.cv:
            while len(self.completed) < len(requests) and time.perf_counter() < deadline:
                self.cv.wait(0.05)
        self.shutdown()
        return list(self.completed)

    def resident_bytes(self) -> int:
        """Device memory all slot contexts hold (fram_resident_bytes)."""
        return sum(int(getattr(c, "resident_bytes", lambda: 0)()) for _, c, _ in self.slots)


def summarize(done: list[Request], warmup_s: float, duration_s: float,
              offered: int | None = None) -> dict:
    """p50 / p99 latency and throughput over the requests arriving after
    warm-up that completed without error; failed requests are counted apart,
    and `offered` (requests submitted after warm-up) shows any left unfinished."""
    after = [r for r in done if r.arrival >= warmup_s and r.done >= 0]
    meas = [r for r in after if not r.error]
    lat = np.array([r.latency_ms for r in meas]) if meas else np.array([np.nan])
    last = max((r.done for r in meas), default=warmup_s)
    return dict(
        requests=len(meas),
        failed=len(after) - len(meas),
        errors=sorted({r.error for r in after if r.error})[:5],
        unfinished=(offered - len(after)) if offered is not None else 0,
        p50_ms=float(np.percentile(lat, 50)),
        p99_ms=float(np.percentile(lat, 99)),
        mean_ms=float(np.mean(lat)),
        solves_per_s=len(meas) / max(1e-9, last - warmup_s),
        offered_per_s=len(meas) / duration_s,
        by_small_slots=sum(1 for r in meas if r.worker.startswith("small")),
        by_group=sum(1 for r in meas if r.worker.startswith("group")),
    )
