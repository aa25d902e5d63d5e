"""A CPU model of workgroups sharing the compute units, for grids whose
workgroups wait for each other (the on-chip SDSN projection keeps the iterate
in registers and meets at a grid-wide barrier every pass, Algorithm 2).

Such a grid makes progress only when all of its workgroups are resident at
once.  The model is a discrete-event simulation: a device with C slots (one
workgroup of the on-chip grid per compute unit), kernels submitted on
several streams, and a dispatcher that hands free slots to waiting
workgroups in submission order, interleaving the kernels of different
streams as the hardware queues do.  A resident workgroup of a barrier grid
holds its slot while it waits.

What it shows:

* two barrier grids that each need the whole device, launched from two
  streams (two contexts solving at once: the server's slots, fram_solve_many's
  workers), can each get part of the device; every slot is then held by a
  waiting workgroup and nothing can run again -- a deadlock, which without a
  bound on the wait hangs the device (with a bound, every workgroup times out);
* a barrier grid next to a kernel that holds a slot for a long time (one
  workgroup of the assignment) only waits, it does not deadlock;
* the launch protocol of the library -- a compute-unit budget over the
  on-chip launches of the process (a launch that would not fit beside the
  launches that may still run waits for the oldest of them), a roll call at
  kernel start with a bounded wait, and a fallback to the streaming passes
  when the roll call fails -- completes in every scenario, lets small grids
  run side by side, and takes the fallback only when a long kernel of another
  stream holds slots past the roll-call bound.
"""
from __future__ import annotations

import heapq
from dataclasses import dataclass, field

import pytest


@dataclass
class Kernel:
    name: str
    grid: int                 # workgroups
    barrier: bool             # workgroups wait for the whole grid
    work: float               # time a workgroup runs once the grid can proceed
    after: list = field(default_factory=list)   # kernels that must complete first
    roll_call: float | None = None   # bounded wait for all workgroups (barrier grids)
    wait_bound: float | None = None  # bound on a barrier wait without roll call
    # results
    started: int = 0
    done: int = 0
    finished_at: float | None = None
    outcome: str = ""          # "ok", "fallback", "timeout"


def simulate(slots: int, kernels: list[Kernel], horizon: float = 1e6) -> dict:
    """Event simulation; returns {'deadlock': bool, 'time': t}."""
    free = slots
    t = 0.0
    ev: list = []   # (time, seq, kind, kernel index)
    seq = 0
    waiting: dict[int, int] = {}   # barrier kernel -> resident workgroups waiting
    first_arrival: dict[int, float] = {}
    aborted: set[int] = set()

    def ready(k: Kernel) -> bool:
        return all(d.finished_at is not None for d in k.after)

    def push(tt, kind, i):
        nonlocal seq
        heapq.heappush(ev, (tt, seq, kind, i))
        seq += 1

    def dispatch():
        nonlocal free
        progressed = True
        while progressed and free > 0:
            progressed = False
            # round-robin over the kernels that are ready and have workgroups left
            for i, k in enumerate(kernels):
                if free == 0:
                    break
                if k.finished_at is not None or k.started >= k.grid or not ready(k):
                    continue
                if i in aborted:
                    continue
                k.started += 1
                free -= 1
                progressed = True
                if not k.barrier:
                    push(t + k.work, "end", i)
                else:
                    waiting[i] = waiting.get(i, 0) + 1
                    if i not in first_arrival:
                        first_arrival[i] = t
                        bound = k.roll_call if k.roll_call is not None else k.wait_bound
                        if bound is not None:
                            push(t + bound, "bound", i)
                    if waiting[i] == k.grid:
                        # every workgroup resident: the grid runs to the end
                        push(t + k.work, "gridend", i)

    dispatch()
    while ev:
        t, _, kind, i = heapq.heappop(ev)
        if t > horizon:
            break
        k = kernels[i]
        if kind == "end":
            k.done += 1
            free += 1
            if k.done == k.grid:
                k.finished_at = t
                k.outcome = "ok"
        elif kind == "gridend":
            if k.finished_at is None:
                free += waiting.pop(i, 0)
                k.done = k.grid
                k.finished_at = t
                k.outcome = "ok"
        elif kind == "bound":
            if k.finished_at is None and waiting.get(i, 0) < k.grid:
                # the bounded wait ends: resident workgroups leave, the rest
                # exit at once when they start (they see the abort flag)
                free += waiting.pop(i, 0)
                aborted.add(i)
                k.finished_at = t
                k.outcome = "fallback" if k.roll_call is not None else "timeout"
        dispatch()
    unfinished = [k for k in kernels if k.finished_at is None]
    return {"deadlock": bool(unfinished), "time": t, "unfinished": [k.name for k in unfinished]}


C = 256  # compute units of the device; one on-chip workgroup each


def test_one_barrier_grid_alone_completes():
    k = Kernel("sdsn", C, True, 50.0)
    r = simulate(C, [k])
    assert not r["deadlock"] and k.outcome == "ok"


def test_two_concurrent_barrier_grids_deadlock_without_a_bound():
    a = Kernel("sdsn-a", C, True, 50.0)
    b = Kernel("sdsn-b", C, True, 50.0)
    r = simulate(C, [a, b])
    assert r["deadlock"] and set(r["unfinished"]) == {"sdsn-a", "sdsn-b"}
    assert a.started + b.started == C  # every slot held by a waiting workgroup


def test_eight_server_slots_deadlock_without_a_bound():
    ks = [Kernel(f"slot{i}", C, True, 50.0) for i in range(8)]
    r = simulate(C, ks)
    assert r["deadlock"]


def test_bounded_waits_turn_the_deadlock_into_timeouts():
    a = Kernel("sdsn-a", C, True, 50.0, wait_bound=1e6 / 1e3)
    b = Kernel("sdsn-b", C, True, 50.0, wait_bound=1e6 / 1e3)
    r = simulate(C, [a, b])
    # the first bound to expire frees its slots and lets the other grid finish
    assert not r["deadlock"] and "timeout" in (a.outcome, b.outcome)


def test_a_long_kernel_of_another_stream_only_delays_a_barrier_grid():
    lap = Kernel("lap", 1, False, 50_000.0)  # one workgroup for ~50 ms
    k = Kernel("sdsn", C, True, 50.0)
    r = simulate(C, [lap, k])
    assert not r["deadlock"] and k.outcome == "ok" and k.finished_at >= 50_000.0


def serialized(kernels: list[Kernel], slots: int = C) -> list[Kernel]:
    """The library's launch protocol for on-chip grids, in submission order:
    the launches that may still run are counted (here: every earlier one not
    already waited for, since nothing has completed at submission), and while
    they and the new grid together need more slots than the device has, the
    new launch waits for the oldest of them."""
    live: list[Kernel] = []
    for k in kernels:
        if not k.barrier:
            continue
        used = sum(x.grid for x in live)
        while live and used + k.grid > slots:
            k.after.append(live[0])
            used -= live[0].grid
            live.pop(0)
        live.append(k)
    return kernels


@pytest.mark.parametrize("streams", [2, 3, 8, 32])
def test_library_protocol_completes_for_any_number_of_streams(streams):
    ks = serialized([Kernel(f"slot{i}", C, True, 50.0, roll_call=20_000.0)
                     for i in range(streams)])
    r = simulate(C, ks)
    assert not r["deadlock"]
    assert all(k.outcome == "ok" for k in ks)


def test_library_protocol_with_other_kernels_in_flight():
    # Streaming passes and assignments of other contexts in between: barrier
    # grids still complete; one whose roll call overlaps a long assignment
    # past the bound falls back to the streaming passes (which always run).
    plain = [Kernel(f"pass{i}", 64, False, 20.0) for i in range(20)]
    lap = Kernel("lap", 1, False, 50_000.0)
    on = serialized([Kernel(f"sdsn{i}", C, True, 50.0, roll_call=20_000.0) for i in range(4)])
    ks = plain[:10] + [lap] + on + plain[10:]
    r = simulate(C, ks)
    assert not r["deadlock"]
    assert {k.outcome for k in on} <= {"ok", "fallback"}
    assert any(k.outcome == "fallback" for k in on)
    assert all(k.outcome == "ok" for k in plain + [lap])


def test_small_grids_run_side_by_side_under_the_budget():
    # 16 projections of 16 workgroups each (small pairs solved concurrently):
    # all fit together, so none waits for another and all finish at once.
    ks = serialized([Kernel(f"small{i}", 16, True, 50.0, roll_call=20_000.0) for i in range(16)])
    r = simulate(C, ks)
    assert not r["deadlock"] and all(k.outcome == "ok" for k in ks)
    assert all(not k.after for k in ks) and max(k.finished_at for k in ks) == 50.0


def test_budget_with_mixed_grid_sizes_completes_without_fallback():
    sizes = [16, 256, 64, 100, 256, 25, 128, 200]
    ks = serialized([Kernel(f"g{i}", g, True, 50.0, roll_call=20_000.0)
                     for i, g in enumerate(sizes)])
    r = simulate(C, ks)
    assert not r["deadlock"] and all(k.outcome == "ok" for k in ks)
    # a whole-device grid never overlaps another on-chip grid
    for k in ks:
        if k.grid == C:
            assert k.after
