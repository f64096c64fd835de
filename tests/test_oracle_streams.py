"""Pin the oracle's streams and events (paper Section 3 "Streams and events").

Launches in one stream run one after another; launches of different streams
may run in parallel unless an event (a dependency before -> after) orders
them.  A global word touched by two launches that may run in parallel, and
written by at least one of them, is a race between the launches (scope 2).

Pins, each independent of the oracle's closure and summaries:

* hand-derived tuples on small jobs (values worked out below);
* which launches may run in parallel, against an enumeration of every
  execution order the streams and events admit (two launches may run in
  parallel exactly when some admitted order runs them either way round);
* the tuples, against a pairwise scan of the two launches' access records
  (every record of one launch against every record of the other);
* race-free jobs: every admitted order of the launches leaves the same final
  memory as the submission order.
"""
import itertools
import random

import numpy as np
import pytest

from oracle import oracle as O
from paper_1211_6193_amd import ir
from paper_1211_6193_amd.workloads import Job, LaunchSpec

NONE = 0xFFFFFFFF


def _spec(a, nb, nt):
    return LaunchSpec(np.array(a.assemble(), dtype=np.uint64), (nb, 1, 1), (nt, 1, 1), 0, ())


def _writer(value):
    """Thread g (global id) stores value + g to word g."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0)
    a.ADDI(4, 3, value).STG(3, 0, 4).EXIT()
    return a


def _reader_of(base):
    """Thread g loads word base - g and stores it to word 8 + g."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0)
    a.MOVI(4, base).SUB(4, 4, 3).LDG(5, 4, 0).STG(3, 8, 5).EXIT()
    return a


def _cross(res):
    return sorted(t for t in res.race_tuples() if t[2] == 2)


def _job(specs, streams=None, deps=(), words=16):
    return Job(list(specs), np.arange(words, dtype=np.int32) * 3, streams=streams, deps=list(deps))


def test_two_streams_hand_tuples():
    # L0: 4 threads write words 0..3.  L1: 2 blocks of 1 thread, gtid g reads
    # word 3 - g and writes word 8 + g.  Words 3 and 2 are written by L0
    # (threads 3 and 2) and read by L1 (gtids 0 and 1): two races, reported on
    # launch 1 against launch 0, w_tid from L1 and o_tid from L0.
    specs = [_spec(_writer(100), 1, 4), _spec(_reader_of(3), 2, 1)]
    res = O.run_job(_job(specs, streams=[0, 1]))
    assert _cross(res) == [(1, 1, 2, 0, NONE, 2, 1, 2), (1, 1, 2, 0, NONE, 3, 0, 3)]
    # the job still runs in submission order: L1 read what L0 wrote
    assert list(res.memory[8:10]) == [103, 102]
    assert res.launches_completed == 2


def test_same_stream_or_event_orders_the_launches():
    specs = [_spec(_writer(100), 1, 4), _spec(_reader_of(3), 2, 1)]
    for job in (_job(specs), _job(specs, streams=[5, 5]), _job(specs, streams=[0, 1], deps=[(0, 1)])):
        res = O.run_job(job)
        assert _cross(res) == []
        assert list(res.memory[8:10]) == [103, 102]


def test_write_write_and_read_read():
    # Three streams.  L0 writes words 0..1 (gtids 0, 1); L1 writes words 0..2
    # (gtids 0..2): write-write races on words 0 and 1, each side's smallest
    # conflicting thread being the one that writes the word.  L2 reads words 3
    # and 2 (gtids 0, 1) and writes words 8, 9: word 2 is written by L1
    # (gtid 2) and read by L2 (gtid 1); no other launch touches words 3, 8, 9.
    specs = [_spec(_writer(10), 1, 2), _spec(_writer(20), 1, 3), _spec(_reader_of(3), 1, 2)]
    res = O.run_job(_job(specs, streams=[0, 1, 2]))
    assert _cross(res) == [(1, 1, 2, 0, NONE, 0, 0, 0), (1, 1, 2, 0, NONE, 1, 1, 1),
                           (2, 1, 2, 1, NONE, 2, 1, 2)]


def test_min_thread_when_only_one_side_writes():
    # L0: 2 blocks x 2 threads all read word 0, and gtid g writes word 4 + g.
    # L1: 1 block x 3 threads, thread t writes word t * 2 (words 0, 2, 4).
    # Word 0: L1 writes it (tid 0), L0 reads it with every thread: the
    # smallest conflicting L0 thread is gtid 0.  Word 4: L0 writes it (gtid 0)
    # and L1 writes it (tid 2).
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0)
    a.LDG(5, 15, 0).STG(3, 4, 5).EXIT()
    b = ir.Asm()
    b.SREG(0, "TID").ADD(3, 0, 0).STG(3, 0, 0).EXIT()
    res = O.run_job(_job([_spec(a, 2, 2), _spec(b, 1, 3)], streams=[0, 1]))
    assert _cross(res) == [(1, 1, 2, 0, NONE, 0, 0, 0), (1, 1, 2, 0, NONE, 4, 2, 0)]


def test_transitive_order():
    # L0 (s0), L1 (s1), L2 (s0), every launch writing words 0..1.
    w = _spec(_writer(1), 1, 2)
    # L1 waits for L0 and L2 comes after L0 in s0: L1 and L2 may overlap
    res = O.run_job(_job([w, w, w], streams=[0, 1, 0], deps=[(0, 1)]))
    assert sorted({(r[0], r[3]) for r in _cross(res)}) == [(2, 1)]
    # ... unless L2 also waits for L1: then 0 -> 1 -> 2, no races
    res = O.run_job(_job([w, w, w], streams=[0, 1, 0], deps=[(0, 1), (1, 2)]))
    assert _cross(res) == []
    # chain through a third stream: 0 -> 1 (event), 1 -> 2 (event), all streams differ
    res = O.run_job(_job([w, w, w], streams=[0, 1, 2], deps=[(0, 1), (1, 2)]))
    assert _cross(res) == []


def test_deadlocked_launch_ends_the_job():
    # L1 deadlocks (thread 0 exits, thread 1 waits); L2 (another stream) never runs
    d = ir.Asm()
    d.SREG(0, "TID").STG(0, 0, 0).BZ(0, "E").BAR().label("E").EXIT()
    specs = [_spec(_writer(1), 1, 2), _spec(d, 1, 2), _spec(_writer(2), 1, 2)]
    res = O.run_job(_job(specs, streams=[0, 1, 2]))
    assert res.launches_completed == 1
    assert sorted({(r[0], r[3]) for r in _cross(res)}) == [(1, 0)]


def test_bad_dependencies_rejected():
    specs = [_spec(_writer(1), 1, 2)] * 2
    for deps in ([(1, 0)], [(0, 0)], [(0, 2)]):
        with pytest.raises(ValueError):
            O.run_job(_job(specs, streams=[0, 1], deps=deps))


# ---- brute-force pins over random small jobs --------------------------------

def _orders(n, streams, deps):
    """Every order of the launches that keeps each stream's order and every dependency."""
    out = []
    for p in itertools.permutations(range(n)):
        pos = {l: i for i, l in enumerate(p)}
        ok = all(pos[a] < pos[b] for a, b in deps)
        ok = ok and all(pos[a] < pos[b] for a in range(n) for b in range(a + 1, n) if streams[a] == streams[b])
        if ok:
            out.append(p)
    return out


def _random_launch(rng):
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0)
    for _ in range(rng.randint(1, 3)):
        base, off = rng.choice([(15, rng.randint(0, 5)), (3, rng.randint(0, 3)), (0, 2)])
        if rng.random() < 0.5:
            a.LDG(5, base, off)
        else:
            a.ADDI(6, 3, rng.randint(1, 50)).STG(base, off, 6)
    a.EXIT()
    return _spec(a, rng.randint(1, 2), rng.randint(1, 3))


def _random_job(rng):
    n = rng.randint(2, 4)
    specs = [_random_launch(rng) for _ in range(n)]
    streams = [rng.randint(0, 2) for _ in range(n)]
    deps = sorted({tuple(sorted(rng.sample(range(n), 2))) for _ in range(rng.randint(0, 2))})
    return Job(specs, np.arange(16, dtype=np.int32) * 7 + 1, streams=streams, deps=deps)


def _pairwise(job, res):
    """Cross-launch tuples from the records, pair of records by pair of records."""
    n = len(job.launches)
    orders = _orders(n, job.streams, job.deps)
    recs = res.record_log
    out = set()
    for i in range(n):
        for j in range(i + 1, n):
            if not any(o.index(j) < o.index(i) for o in orders):
                continue                    # i always runs before j
            nti, ntj = job.launches[i].n_threads, job.launches[j].n_threads
            ri = [r for r in recs if r["launch"] == i and r["space"] == 1]
            rj = [r for r in recs if r["launch"] == j and r["space"] == 1]
            for x in sorted({int(r["addr"]) for r in ri} & {int(r["addr"]) for r in rj}):
                gi = [(int(r["block"]) * nti + int(r["tid"]), int(r["kind"])) for r in ri if r["addr"] == x]
                gj = [(int(r["block"]) * ntj + int(r["tid"]), int(r["kind"])) for r in rj if r["addr"] == x]
                pairs = [(a, b) for a in gj for b in gi if a[1] or b[1]]
                if pairs:
                    out.add((j, 1, 2, i, NONE, x, min(a[0] for a, _ in pairs), min(b[0] for _, b in pairs)))
    return sorted(out)


@pytest.mark.parametrize("seed", range(60))
def test_random_jobs_against_pairwise_records(seed):
    rng = random.Random(seed)
    job = _random_job(rng)
    res = O.run_job(job, keep_records=True)
    assert res.launches_completed == len(job.launches)
    assert _cross(res) == _pairwise(job, res)


def _disjoint_job(rng):
    """Launch k reads shared inputs (words 0..3) and, at random, the output
    region of another launch, and writes its own region (words 4 + 6k + g)."""
    n = rng.randint(2, 4)
    specs = []
    for k in range(n):
        a = ir.Asm()
        a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0)
        a.LDG(5, 15, rng.randint(0, 3))
        if rng.random() < 0.4:
            a.LDG(6, 3, 4 + 6 * rng.randrange(n)).ADD(5, 5, 6)
        a.ADD(5, 5, 3).STG(3, 4 + 6 * k, 5).EXIT()
        specs.append(_spec(a, rng.randint(1, 2), rng.randint(1, 3)))
    streams = [rng.randint(0, 2) for _ in range(n)]
    deps = sorted({tuple(sorted(rng.sample(range(n), 2))) for _ in range(rng.randint(0, 2))})
    return Job(specs, np.arange(32, dtype=np.int32) * 5 + 2, streams=streams, deps=deps)


def test_race_free_jobs_are_order_independent():
    rng = random.Random(2024)
    checked = 0
    for _ in range(300):
        job = _disjoint_job(rng)
        res = O.run_job(job)
        if len(res.races) or len(res.faults):
            continue
        orders = _orders(len(job.launches), job.streams, job.deps)
        checked += len(orders) > 1
        for order in orders:
            serial = Job([job.launches[k] for k in order], job.memory)
            assert np.array_equal(O.run_job(serial).memory, res.memory), order
    assert checked >= 50
