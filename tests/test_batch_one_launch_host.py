"""Host emulation of the one-launch batch (batch.hip, k_batch_one) on the
library's own work-item order (fdwt_batch_schedule, computed on the host):

  * the schedule lists every tile of every pass of every job once, with the
    dependency count of the pass before, and every item of pass k - 1 of a
    job comes before every item of pass k of that job (tickets are taken in
    this order);
  * an event-driven simulation of the protocol (a ticket counter handing out
    chunks of items, per-job pass counters, waits until a job's previous pass
    is complete) with more workgroups than resident slots, random item times
    and random arrival of non-resident workgroups: every run completes, and
    whenever a workgroup waits, every item it waits for is done or held by a
    resident workgroup (no wait precedes its producer's residency);
  * the same simulator finds the deadlock of a fixed-stride order (item i to
    workgroup i mod G) once fewer than G workgroups are resident, the flaw of
    an earlier one-launch design.
"""
import heapq

import numpy as np
import pytest

from paper_0808_0487_amd import fdwt

KBLOGE, KBMAXPASS = 13, 3


def plan_passes(m):
    """Passes (d0, r, wdig) of a job in the one-launch batch (batch.hip,
    batch_plan_one): m < 13 one pass; otherwise a contiguous first pass of 13
    digits, then the other m - 13 digits split evenly into strided passes of
    at most 9 digits over rows of 2^(13 - r) elements."""
    if m < KBLOGE:
        return [(0, m, 0)]
    rem = m - KBLOGE
    nstr = (rem + 8) // 9
    out, d = [(0, KBLOGE, 0)], KBLOGE
    for i in range(nstr):
        r = (rem - (d - KBLOGE) + (nstr - i) - 1) // (nstr - i)
        out.append((d, r, KBLOGE - r))
        d += r
    return out


def plan_tiles(m):
    return [2 ** m >> (r + w) for d0, r, w in plan_passes(m)]


@pytest.mark.parametrize("m", range(1, 27))
def test_one_launch_plan_covers_the_digits_in_2_13_tiles(m):
    done = 0
    for d0, r, w in plan_passes(m):
        assert d0 == done and w <= d0 and r >= 1
        if m >= KBLOGE:
            assert r + w == KBLOGE and (d0 == 0 or w >= 4)
        done += r
    assert done == m and len(plan_passes(m)) <= KBMAXPASS


def ragged(n, lo, hi, seed):
    return np.random.default_rng(seed).integers(lo, hi + 1, n).astype(np.int32)


@pytest.mark.parametrize("ms", [ragged(512, 12, 22, 4), ragged(40, 1, 26, 5), np.array([7], np.int32),
                                np.array([26, 1, 13, 14, 23], np.int32)])
def test_schedule_lists_each_tile_once_in_dependency_order(ms):
    job, ps, tile, need, chunk = fdwt.batch_schedule(ms)
    assert chunk >= 1
    seen = {}
    for i, (j, k, t) in enumerate(zip(job, ps, tile)):
        assert (j, k, t) not in seen
        seen[(j, k, t)] = i
    for j, m in enumerate(ms):
        nt = plan_tiles(int(m))
        assert len(nt) <= KBMAXPASS
        for k, n in enumerate(nt):
            idx = [seen[(j, k, t)] for t in range(n)]
            if k > 0:
                prev = [seen[(j, k - 1, t)] for t in range(nt[k - 1])]
                assert max(prev) < min(idx)
                assert np.all(need[idx] == nt[k - 1])
            else:
                assert np.all(need[idx] == 0)
    assert len(seen) == sum(sum(plan_tiles(int(m))) for m in ms)


def simulate(job, ps, need, order, G, R, seed, chunk):
    """Event-driven run of G workgroups, at most R resident at once (the rest
    start as resident ones exit).  order: 'ticket' (the kernel's protocol:
    chunks of `chunk` items from a shared counter) or 'stride' (workgroup b
    runs items b, b + G, ...).  Returns (completed, violations)."""
    rng = np.random.default_rng(seed)
    n = len(job)
    done = {}
    holder = np.full(n, -1)          # workgroup holding item i (ticket taken, not finished)
    finished = np.zeros(n, bool)
    resident = set()
    pending = list(range(G))         # not yet started
    queue = {b: [] for b in range(G)}
    state = {}                       # b -> ('run', item) | ('wait', item) | ('exit',)
    ticket = [0]
    ev, now = [], 0.0
    violations = 0

    def refill(b):
        if order == "ticket":
            if ticket[0] >= n:
                return False
            first = ticket[0]
            ticket[0] += chunk
            queue[b] = list(range(first, min(first + chunk, n)))
        else:
            queue[b] = list(range(b, n, G)) if not queue[b] and state.get(b) is None else []
        for i in queue[b]:
            holder[i] = b
        return bool(queue[b])

    def ready(i):
        return ps[i] == 0 or done.get((job[i], ps[i] - 1), 0) >= need[i]

    todo = []                        # workgroups to advance (iteratively)

    def advance(b):
        nonlocal violations
        while True:
            if not queue[b] and not refill(b):
                state[b] = ("exit",)
                resident.discard(b)
                if pending:
                    nb = pending.pop(0)
                    resident.add(nb)
                    state[nb] = None
                    todo.append(nb)
                return
            i = queue[b][0]
            if ready(i):
                state[b] = ("run", i)
                heapq.heappush(ev, (now + rng.exponential(1.0), b))
                return
            # a wait: every item of the job's previous pass must be done or
            # held by a resident workgroup
            prev = np.nonzero((job == job[i]) & (ps == ps[i] - 1))[0]
            for d in prev:
                if not finished[d] and holder[d] not in resident:
                    violations += 1
                    break
            state[b] = ("wait", i)
            return

    def drain():
        while todo:
            advance(todo.pop())

    first = pending[:R]
    pending = pending[R:]
    for b in first:
        resident.add(b)
        state[b] = None
        todo.append(b)
    drain()
    while ev:
        now, b = heapq.heappop(ev)
        _, i = state[b]
        queue[b].pop(0)
        finished[i] = True
        key = (job[i], ps[i])
        done[key] = done.get(key, 0) + 1
        todo.append(b)
        drain()
        for w in list(resident):
            if state.get(w) and state[w][0] == "wait" and ready(state[w][1]):
                todo.append(w)
        drain()
    return bool(finished.all()), violations


@pytest.mark.parametrize("seed", range(6))
def test_ticket_protocol_always_completes(seed):
    g = np.random.default_rng(100 + seed)
    ms = ragged(int(g.integers(3, 40)), 1, 19, 200 + seed)
    job, ps, tile, need, chunk = fdwt.batch_schedule(ms)
    G = int(g.integers(2, 64))
    R = int(g.integers(1, G + 1))
    ok, bad = simulate(job, ps, need, "ticket", G, R, seed, chunk)
    assert ok and bad == 0, (G, R)


def test_ticket_protocol_at_the_benchmark_shape():
    """512 jobs of 2^12..2^22 points, 1024 workgroups of which 300 resident."""
    ms = ragged(512, 12, 22, 4)
    job, ps, tile, need, chunk = fdwt.batch_schedule(ms)
    ok, bad = simulate(job, ps, need, "ticket", 1024, 300, 1, chunk)
    assert ok and bad == 0


def test_fixed_stride_order_deadlocks_when_not_all_resident():
    ms = np.array([16, 16, 15], np.int32)
    job, ps, tile, need, chunk = fdwt.batch_schedule(ms)
    G = 16
    ok_all, _ = simulate(job, ps, need, "stride", G, G, 0, chunk)
    ok_few, bad = simulate(job, ps, need, "stride", G, 4, 0, chunk)
    assert ok_all            # every workgroup resident: the stride order works
    assert not ok_few        # four resident: a wait on an item nobody runs
    assert bad > 0
