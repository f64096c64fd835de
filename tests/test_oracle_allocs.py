"""Pin the oracle's memory-object check: a job may list its device
allocations (word ranges of its memory); a global access to a word outside
every allocation is an illegal access (paper Section 3: the tool checks for
out-of-bounds and illegal device or host memory access).  Each block that
made such accesses to a word gets one ALLOC finding
{block, epoch 0xFFFFFFFF, a = 2 + stored, b = smallest accessing tid,
c = word, d = smallest storing tid or 0xFFFFFFFF}; the accesses still take
effect.

Pins: hand-derived findings; the findings recomputed from the oracle's
records by a plain scan; everything else in the report and the final memory
unchanged by the check; allocations covering the whole memory give no
finding and an empty list makes every access illegal."""
import random

import numpy as np
import pytest

from oracle import oracle as O
from paper_1211_6193_amd import ir
from paper_1211_6193_amd.workloads import Job, LaunchSpec

NONE = 0xFFFFFFFF
ALLOC = 6


def _spec(a, nb, nt, shmem=0):
    return LaunchSpec(np.array(a.assemble(), dtype=np.uint64), (nb, 1, 1), (nt, 1, 1), shmem, ())


def _store_load():
    """Global thread g stores g to word 6 + g and loads word 20 - g."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0)
    a.STG(3, 6, 3).MOVI(4, 20).SUB(4, 4, 3).LDG(5, 4, 0).EXIT()
    return a


def _alloc_faults(res):
    return [tuple(int(v) for v in f) for f in res.faults if f["kind"] == ALLOC]


def test_hand_findings():
    # allocations [0, 8) and [16, 24) of 32 words; 2 blocks x 4 threads.
    # Block 0 stores words 6..9 (8 and 9 illegal, tids 2 and 3) and loads
    # 20..17 (allocated).  Block 1 stores words 10..13 (tids 0..3, illegal)
    # and loads 16, 15, 14, 13 (tids 0..3; 15, 14, 13 illegal; tid 3 both
    # loads and stores word 13).
    job = Job([_spec(_store_load(), 2, 4)], np.arange(32, dtype=np.int32), allocs=[(0, 8), (16, 8)])
    res = O.run_job(job)
    assert _alloc_faults(res) == [
        (0, ALLOC, 0, NONE, 3, 2, 8, 2), (0, ALLOC, 0, NONE, 3, 3, 9, 3),
        (0, ALLOC, 1, NONE, 2, 1, 15, NONE), (0, ALLOC, 1, NONE, 2, 2, 14, NONE),
        (0, ALLOC, 1, NONE, 3, 0, 10, 0), (0, ALLOC, 1, NONE, 3, 1, 11, 1),
        (0, ALLOC, 1, NONE, 3, 2, 12, 2), (0, ALLOC, 1, NONE, 3, 3, 13, 3)]
    # the accesses took effect
    assert list(res.memory[6:14]) == list(range(8))


def test_whole_memory_none_and_empty():
    base = Job([_spec(_store_load(), 2, 4)], np.arange(32, dtype=np.int32))
    plain = O.run_job(base)
    for allocs in (None, [(0, 32)], [(0, 16), (16, 16)], [(0, 20), (10, 22)]):
        res = O.run_job(Job(base.launches, base.memory, allocs=allocs))
        assert _alloc_faults(res) == []
        assert res.fault_tuples() == plain.fault_tuples()
    res = O.run_job(Job(base.launches, base.memory, allocs=[]))
    # nothing allocated: every accessed word is illegal (8 stores, 8 loads,
    # word 13 both in block 1)
    f = _alloc_faults(res)
    assert len(f) == 15 and {x[6] for x in f} == set(range(6, 21))


def test_bad_regions_rejected():
    for allocs in ([(0, 33)], [(30, 3)], [(33, 0)]):
        with pytest.raises(ValueError):
            O.run_job(Job([_spec(_store_load(), 2, 4)], np.arange(32, dtype=np.int32), allocs=allocs))


def _random_job(rng):
    launches = []
    for _ in range(rng.randint(1, 3)):
        a = ir.Asm()
        a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0)
        for _ in range(rng.randint(1, 5)):
            base, off = rng.choice([(15, rng.randint(0, 23)), (3, rng.randint(0, 15)), (0, rng.randint(0, 9))])
            op = rng.random()
            if op < 0.4:
                a.LDG(5, base, off)
            elif op < 0.8:
                a.ADDI(6, 3, rng.randint(1, 50)).STG(base, off, 6)
            elif op < 0.9:
                a.STS(0, 0, 3).LDS(7, 15, 0)
            else:
                a.BAR()
        a.EXIT()
        launches.append(_spec(a, rng.randint(1, 3), rng.randint(1, 4), 16))
    allocs = [(b, rng.randint(0, 24 - b)) for b in sorted(rng.sample(range(24), rng.randint(0, 3)))]
    return Job(launches, np.arange(24, dtype=np.int32) * 3, allocs=allocs)


def _scan(job, res):
    ok = np.zeros(len(job.memory), bool)
    for b, w in job.allocs:
        ok[b:b + w] = True
    groups = {}
    for r in res.record_log:
        if r["space"] != 1 or ok[r["addr"]]:
            continue
        key = (int(r["launch"]), int(r["block"]), int(r["addr"]))
        groups.setdefault(key, []).append((int(r["tid"]), int(r["kind"])))
    out = []
    for (l, b, x), acc in groups.items():
        w = [t for t, k in acc if k == 1]
        out.append((l, ALLOC, b, NONE, 3 if w else 2, min(t for t, _ in acc), x, min(w) if w else NONE))
    return sorted(out, key=lambda f: (f[0], f[2], f[3], f[1], f[4], f[5], f[6], f[7]))


@pytest.mark.parametrize("seed", range(80))
def test_random_jobs_against_record_scan(seed):
    rng = random.Random(seed)
    job = _random_job(rng)
    res = O.run_job(job, keep_records=True)
    assert _alloc_faults(res) == _scan(job, res)
    plain = O.run_job(Job(job.launches, job.memory))
    assert np.array_equal(res.memory, plain.memory)
    assert res.race_tuples() == plain.race_tuples() and res.records == plain.records
    assert [f for f in res.fault_tuples() if f[1] != ALLOC] == plain.fault_tuples()
