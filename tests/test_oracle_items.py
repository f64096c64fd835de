"""Pin the oracle's memory transfers and host synchronisation (paper Section 3
"Streams and events": launches and memory transfers pass through the stream
queues; the host synchronises through cudaStreamSynchronize,
cudaEventSynchronize and cudaDeviceSynchronize).

A job given as items is its host program: launches and copies (device items,
each in a stream), host reads and writes, and host waits.  Pins, each
independent of the oracle's closure and summaries:

* Figure 1's host program (copy in, two launches, copy out, device
  synchronisation) leaves the paper's printed output in host memory, and its
  asynchronous variants race exactly where worked out by hand below;
* hand-derived tuples and final memory on small jobs;
* which items may run in parallel, against an enumeration of every execution
  order the host program admits;
* the tuples, against a pairwise scan of the items' accesses (kernel access
  records and copy / host word ranges);
* race-free jobs: every admitted order leaves the same final memory as the
  host program's order;
* a job of launches only gives the same result as items as without.
"""
import itertools
import os
import random

import numpy as np
import pytest

from oracle import oracle as O
from paper_1211_6193_amd import ir
from paper_1211_6193_amd import workloads as W
from paper_1211_6193_amd.workloads import (Job, LaunchSpec, copy_item, host_read, host_wait, host_write,
                                           launch_item)

NONE = 0xFFFFFFFF
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig1_paper_run.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        out[k.strip()] = [int(x) for x in v.split()]
    return out


def _cross(res):
    return sorted(t for t in res.race_tuples() if t[2] == 2)


# Figure 1's host program on one memory: host[0, 18) holds the inputs (the
# host array), dev_in = [18, 36) and dev_out = [36, 38) are the two device
# allocations.
HOST, DIN, DOUT = 0, 18, 36


def fig1_items_job(d2h_stream=0, d2h_sync=True, wait=True, variant="BASE"):
    p = W.sum_program(variant)
    launches = [LaunchSpec(p, (2, 1, 1), (9, 1, 1), 36, (DIN, DOUT)),
                LaunchSpec(p, (1, 1, 1), (2, 1, 1), 8, (DOUT, DOUT))]
    mem = np.zeros(38, np.int32)
    mem[HOST:HOST + 18] = W.PAPER_INPUT
    items = [copy_item(DIN, HOST, 18, sync=True),          # cudaMemcpy host -> dev_in
             launch_item(0), launch_item(1),               # sum<<<2,9,36>>>(in,out); sum<<<1,2,8>>>(out,out)
             copy_item(HOST, DOUT, 1, stream=d2h_stream, sync=d2h_sync)]   # dev_out[0] -> host[0]
    if wait:
        items.append(host_wait())                          # cudaDeviceSynchronize
    items.append(host_read(HOST, 1))                       # the host prints host[0]
    return Job(launches, mem, allocs=[(DIN, 18), (DOUT, 2)], items=items)


def test_figure1_host_program_prints_the_papers_output():
    g = _golden()
    res = O.run_job(fig1_items_job())
    assert res.race_tuples() == [] and res.fault_tuples() == []
    assert int(res.memory[HOST]) == g["OUTPUT"][0]
    assert res.launches_completed == 6
    assert res.records == O.run_job(W.fig1_job()).records      # copies and host steps make no records


def test_figure1_asynchronous_copy_out_races():
    # the copy out is asynchronous in stream 1: nothing orders it after either
    # launch (the copy in is synchronous, so it is ordered before).  Both write
    # dev_out[0] -- block 0's thread 0 (global id 0) in the first launch
    # (item 1), thread 0 in the second (item 2) -- and the copy (item 3) reads
    # that word as its thread 0: (3, global, scope 2, 1 and 2, -, 36, 0, 0).
    # The device synchronisation (item 4) orders the host read (item 5).
    res = O.run_job(fig1_items_job(d2h_stream=1, d2h_sync=False))
    assert _cross(res) == [(3, 1, 2, 1, NONE, DOUT, 0, 0), (3, 1, 2, 2, NONE, DOUT, 0, 0)]
    assert int(res.memory[HOST]) == _golden()["OUTPUT"][0]    # the host program's order still runs
    # same stream as the launches, still asynchronous: ordered behind them
    assert _cross(O.run_job(fig1_items_job(d2h_stream=0, d2h_sync=False))) == []


def test_host_reads_before_the_copy_out_finishes():
    # no synchronisation between the asynchronous copy out (item 3, writes
    # host[0] as thread 0) and the host's read of host[0] (item 4, thread 0)
    res = O.run_job(fig1_items_job(d2h_stream=0, d2h_sync=False, wait=False))
    assert _cross(res) == [(4, 1, 2, 3, NONE, HOST, 0, 0)]
    # a synchronous copy out needs no wait
    assert _cross(O.run_job(fig1_items_job(d2h_stream=0, d2h_sync=True, wait=False))) == []


def _writer(value, n):
    """Thread g (global id) stores value + g to word g; one block of n threads."""
    a = ir.Asm()
    a.SREG(0, "TID").ADDI(4, 0, value).STG(0, 0, 4).EXIT()
    return LaunchSpec(np.array(a.assemble(), dtype=np.uint64), (1, 1, 1), (n, 1, 1), 0, ())


def test_copy_and_host_write_values():
    # host writes 7 to words 8..11, copies them to 0..3 in stream 2, waits for
    # the copy (item 1), writes 9 to words 10..13, reads 0..3
    items = [host_write(8, 4, 7), copy_item(0, 8, 4, stream=2), host_wait(1), host_write(10, 4, 9),
             host_read(0, 4)]
    res = O.run_job(Job([], np.arange(16, dtype=np.int32), items=items))
    assert res.race_tuples() == []
    assert res.memory.tolist() == [7, 7, 7, 7, 4, 5, 6, 7, 7, 7, 9, 9, 9, 9, 14, 15]
    assert res.launches_completed == 5 and res.records == 0


def test_host_write_while_a_copy_reads_the_host_buffer():
    # copy (item 0, stream 1) reads words 8..11 as threads 0..3; the host then
    # overwrites words 10..11 (item 1, threads 0..1) with no wait in between:
    # the later item is the host write, w = its smallest thread on each word,
    # o = the copy's thread of that word
    items = [copy_item(0, 8, 4, stream=1), host_write(10, 2, 5)]
    res = O.run_job(Job([], np.arange(16, dtype=np.int32), items=items))
    assert _cross(res) == [(1, 1, 2, 0, NONE, 10, 0, 2), (1, 1, 2, 0, NONE, 11, 1, 3)]
    assert res.memory[0:4].tolist() == [8, 9, 10, 11]     # the copy ran first (host program order)
    # waiting for the stream (its last item) or the device orders them
    for w in (host_wait(0), host_wait()):
        assert _cross(O.run_job(Job([], np.arange(16, dtype=np.int32), items=[items[0], w, items[1]]))) == []


def test_kernel_and_copy_in_two_streams_with_and_without_event():
    # launch (item 0, stream 0) writes words 0..3 (thread g -> word g);
    # copy (item 1, stream 1) reads words 2..5 into 8..11 (thread k: word 2 + k)
    items = [launch_item(0, stream=0), copy_item(8, 2, 4, stream=1)]
    mk = lambda deps: Job([_writer(100, 4)], np.zeros(16, np.int32), items=items, deps=deps)
    res = O.run_job(mk([]))
    assert _cross(res) == [(1, 1, 2, 0, NONE, 2, 0, 2), (1, 1, 2, 0, NONE, 3, 1, 3)]
    assert res.memory[8:12].tolist() == [102, 103, 0, 0]
    assert _cross(O.run_job(mk([(0, 1)]))) == []            # event recorded behind 0, waited ahead of 1


def test_wait_for_one_item_does_not_order_another_stream():
    # items 0 (stream 0) and 1 (stream 1) write word 0 (copies from 4 and 5);
    # the host waits for item 0 only, then reads word 0: races with item 1,
    # and items 0 and 1 race with each other
    items = [copy_item(0, 4, 1, stream=0), copy_item(0, 5, 1, stream=1), host_wait(0), host_read(0, 1)]
    res = O.run_job(Job([], np.arange(8, dtype=np.int32), items=items))
    assert _cross(res) == [(1, 1, 2, 0, NONE, 0, 0, 0), (3, 1, 2, 1, NONE, 0, 0, 0)]
    assert int(res.memory[0]) == 5


def test_deadlocked_launch_ends_the_job():
    a = ir.Asm()
    a.SREG(0, "TID").BNZ(0, "E").BAR()
    a.label("E").EXIT()
    dead = LaunchSpec(np.array(a.assemble(), dtype=np.uint64), (1, 1, 1), (2, 1, 1), 0, ())
    items = [host_write(0, 1, 3), launch_item(0), copy_item(1, 0, 1)]
    res = O.run_job(Job([dead], np.zeros(4, np.int32), items=items))
    assert res.launches_completed == 1
    assert [f[1] for f in res.fault_tuples()] == [O.F_DEADLOCK]
    assert res.memory.tolist() == [3, 0, 0, 0]                # the copy never ran


@pytest.mark.parametrize("items,deps", [
    ([copy_item(0, 2, 4)], []),                  # overlapping ranges
    ([copy_item(14, 0, 4)], []),                 # past the memory
    ([host_read(15, 2)], []),
    ([copy_item(0, 8, 1), host_write(1, 1, 0)], [(0, 1)]),   # a dependency to a host item
    ([copy_item(0, 8, 1), host_wait(1)], []),    # a wait for a later item (itself)
    ([host_write(0, 1, 0), host_wait(0)], []),   # a wait for a host item
    ([launch_item(1)], []),                      # no launch 1
    ([W.Item("memset")], []),
])
def test_bad_items_rejected(items, deps):
    with pytest.raises(ValueError):
        O.run_job(Job([_writer(1, 2)], np.zeros(16, np.int32), items=items, deps=deps))


def test_launches_only_same_as_without_items():
    rng = random.Random(5)
    for _ in range(30):
        job = _random_launch_job(rng)
        as_items = Job(job.launches, job.memory, deps=job.deps,
                       items=[launch_item(i, s) for i, s in enumerate(job.streams)])
        a, b = O.run_job(job), O.run_job(as_items)
        assert a.race_tuples() == b.race_tuples() and a.fault_tuples() == b.fault_tuples()
        assert np.array_equal(a.memory, b.memory) and a.records == b.records


# ---- brute-force pins over random small item jobs ----------------------------

DEVICE = ("launch", "copy")


def _orders(items, deps):
    """Every order of the items the host program admits: each stream keeps its
    order, every dependency holds, a host step or a synchronous copy comes
    before everything issued after it, and a host wait comes after what it
    waits for."""
    n = len(items)
    cons = set(deps)
    for i in range(n):
        for j in range(i + 1, n):
            a, b = items[i], items[j]
            if a.kind in DEVICE and b.kind in DEVICE and a.stream == b.stream:
                cons.add((i, j))
            if a.kind not in DEVICE or (a.kind == "copy" and a.sync):
                cons.add((i, j))
            if b.kind == "host_wait" and a.kind in DEVICE and (b.wait is None or b.wait == i):
                cons.add((i, j))
    out = []
    for p in itertools.permutations(range(n)):
        pos = {x: k for k, x in enumerate(p)}
        if all(pos[a] < pos[b] for a, b in cons):
            out.append(p)
    return out


def _accesses(job, res, j):
    """(word, thread, is_write) of item j's global accesses."""
    it = job.items[j]
    if it.kind == "launch":
        nt = job.launches[it.launch].n_threads
        return [(int(r["addr"]), int(r["block"]) * nt + int(r["tid"]), int(r["kind"]))
                for r in res.record_log if r["launch"] == j and r["space"] == 1]
    if it.kind == "copy":
        return [(it.src + k, k, 0) for k in range(it.words)] + [(it.dst + k, k, 1) for k in range(it.words)]
    if it.kind in ("host_read", "host_write"):
        return [(it.dst + k, k, int(it.kind == "host_write")) for k in range(it.words)]
    return []


def _pairwise(job, res):
    orders = _orders(job.items, job.deps)
    out = set()
    n = len(job.items)
    for i in range(n):
        for j in range(i + 1, n):
            if not any(o.index(j) < o.index(i) for o in orders):
                continue                    # i always runs before j
            ai, aj = _accesses(job, res, i), _accesses(job, res, j)
            for x in sorted({a[0] for a in ai} & {a[0] for a in aj}):
                pairs = [(b, c) for b in aj if b[0] == x for c in ai if c[0] == x if b[2] or c[2]]
                if pairs:
                    out.add((j, 1, 2, i, NONE, x, min(b[1] for b, _ in pairs), min(c[1] for _, c in pairs)))
    return sorted(out)


def _random_kernel(rng):
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0)
    for _ in range(rng.randint(1, 3)):
        base, off = rng.choice([(15, rng.randint(0, 7)), (3, rng.randint(0, 5))])
        if rng.random() < 0.5:
            a.LDG(5, base, off)
        else:
            a.ADDI(6, 3, rng.randint(1, 50)).STG(base, off, 6)
    a.EXIT()
    return LaunchSpec(np.array(a.assemble(), dtype=np.uint64), (rng.randint(1, 2), 1, 1),
                      (rng.randint(1, 3), 1, 1), 0, ())


def _random_launch_job(rng):
    n = rng.randint(2, 4)
    specs = [_random_kernel(rng) for _ in range(n)]
    streams = [rng.randint(0, 2) for _ in range(n)]
    deps = sorted({tuple(sorted(rng.sample(range(n), 2))) for _ in range(rng.randint(0, 2))})
    return Job(specs, np.arange(16, dtype=np.int32) * 7 + 1, streams=streams, deps=deps)


def _random_item(rng, i, items, n_launches):
    r = rng.random()
    if r < 0.3:
        return launch_item(rng.randrange(n_launches), rng.randint(0, 1))
    if r < 0.55:
        w = rng.randint(1, 3)
        src = rng.randint(0, 12 - w)
        dst = rng.choice([x for x in range(0, 13 - w) if x + w <= src or src + w <= x])
        return copy_item(dst, src, w, stream=rng.randint(0, 1), sync=rng.random() < 0.2)
    if r < 0.7:
        return host_read(rng.randint(0, 10), rng.randint(1, 2))
    if r < 0.85:
        return host_write(rng.randint(0, 10), rng.randint(1, 2), rng.randint(-9, 9))
    dev = [k for k in range(i) if items[k].kind in DEVICE]
    return host_wait(rng.choice(dev) if dev and rng.random() < 0.6 else None)


def _random_item_job(rng):
    n_l = rng.randint(1, 2)
    specs = [_random_kernel(rng) for _ in range(n_l)]
    items = []
    for i in range(rng.randint(2, 5)):
        items.append(_random_item(rng, i, items, n_l))
    dev = [k for k, it in enumerate(items) if it.kind in DEVICE]
    deps = []
    if len(dev) >= 2 and rng.random() < 0.5:
        deps = [tuple(sorted(rng.sample(dev, 2)))]
    return Job(specs, np.arange(16, dtype=np.int32) * 5 + 3, deps=deps, items=items)


@pytest.mark.parametrize("seed", range(80))
def test_random_item_jobs_against_pairwise_accesses(seed):
    rng = random.Random(1000 + seed)
    job = _random_item_job(rng)
    res = O.run_job(job, keep_records=True)
    assert res.launches_completed == len(job.items)
    assert _cross(res) == _pairwise(job, res)


def test_race_free_item_jobs_are_order_independent():
    rng = random.Random(77)
    checked = 0
    for _ in range(400):
        job = _random_item_job(rng)
        res = O.run_job(job)
        if len(res.races) or len(res.faults):
            continue
        orders = _orders(job.items, job.deps)
        checked += len(orders) > 1
        for order in orders:
            serial = [job.items[k] for k in order if job.items[k].kind != "host_wait"]
            serial = [W.Item(it.kind, launch=it.launch, dst=it.dst, src=it.src, words=it.words, value=it.value)
                      for it in serial]
            got = O.run_job(Job(job.launches, job.memory, items=serial)).memory
            assert np.array_equal(got, res.memory), order
    assert checked >= 40
