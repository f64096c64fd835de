"""Pin the oracle against brute-force enumeration of all interleavings.

For random tiny kernels (at most 4 threads in 1-2 blocks, a handful of memory
operations, barriers and tid-dependent branches) every interleaving the
semantics admits is explored by ``brute.enumerate_launch``:

(i)   the oracle reports a race  <=>  some interleaving races  <=>  all do;
(ii)  race-free  =>  one outcome (memory, deadlock, record multiset), equal to
      the oracle's;
(iii) racy  =>  the oracle's final memory is one of the reachable ones;
(iv)  race-free  =>  the oracle reports a deadlock  <=>  every maximal
      interleaving is stuck.
"""
import random
from collections import Counter

import numpy as np
import pytest

import brute
from oracle import oracle as O
from paper_1211_6193_amd import ir
from paper_1211_6193_amd.workloads import Job, LaunchSpec

SH_WORDS = 4
G_WORDS = 6


def random_kernel(rng: random.Random):
    """Straight-line code with forward branches only (always terminates)."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").ADDI(2, 0, 10).MULI(3, 1, 7)
    n_stmt = rng.randint(2, 6)
    lab = 0
    for _ in range(n_stmt):
        kind = rng.choice(["sts", "lds", "stg", "ldg", "alu", "bar", "barp", "cond"])
        base = rng.choice([0, 15, 1])
        if kind == "sts":
            a.STS(rng.choice([0, 15]), rng.randint(0, 2), rng.choice([2, 3, 4]))
        elif kind == "lds":
            a.LDS(rng.choice([2, 3, 4]), rng.choice([0, 15]), rng.randint(0, 2))
        elif kind == "stg":
            a.STG(base, rng.randint(0, 3), rng.choice([2, 3, 4]))
        elif kind == "ldg":
            a.LDG(rng.choice([2, 3, 4]), base, rng.randint(0, 3))
        elif kind == "alu":
            a.ADD(rng.choice([2, 3, 4]), rng.choice([2, 3, 4]), rng.choice([0, 1, 2]))
        elif kind == "bar":
            a.BAR()
        elif kind == "barp":
            a.BARP(rng.choice([2, 3, 4]), rng.choice([0, 2, 3, 4]), rng.choice(["COUNT", "AND", "OR"]))
        else:
            lab += 1
            a.SEQI(8, 0, rng.randint(0, 2)).BZ(8, f"S{lab}")
            inner = rng.choice(["bar", "barp", "sts", "stg", "exit"])
            if inner == "bar":
                a.BAR()
            elif inner == "barp":
                a.BARP(3, 0, rng.choice(["COUNT", "AND", "OR"]))
            elif inner == "sts":
                a.STS(15, rng.randint(0, 2), 2)
            elif inner == "stg":
                a.STG(15, rng.randint(0, 3), 2)
            else:
                a.EXIT()
            a.label(f"S{lab}")
    if rng.random() < 0.8:
        a.EXIT()
    return a.assemble()


def _cases(n, seed):
    rng = random.Random(seed)
    out = []
    while len(out) < n:
        nb = rng.choice([1, 1, 2])
        nt = rng.choice([1, 2, 3]) if nb == 1 else rng.choice([1, 2])
        prog = random_kernel(rng)
        mem = [rng.randint(-3, 9) for _ in range(G_WORDS)]
        out.append((prog, nb, nt, mem))
    return out


def _oracle(prog, nb, nt, mem):
    job = Job([LaunchSpec(np.array(prog, dtype=np.uint64), (nb, 1, 1), (nt, 1, 1), 4 * SH_WORDS, ())],
              np.array(mem, dtype=np.int32))
    return O.run_job(job, keep_records=True)


def _rec_multiset(res):
    return Counter((int(r["space"]), int(r["addr"]), int(r["block"]), int(r["epoch"]), int(r["tid"]),
                    int(r["kind"])) for r in res.record_log)


@pytest.mark.parametrize("chunk", range(8))
def test_oracle_vs_all_interleavings(chunk):
    n_racy = n_free = 0
    for prog, nb, nt, mem in _cases(25, 7000 + chunk):
        res = _oracle(prog, nb, nt, mem)
        outs = brute.enumerate_launch(prog, nb, nt, SH_WORDS, mem)
        assert outs
        racy_flags = {o.racy for o in outs}
        oracle_racy = len(res.races) > 0
        # (i)
        assert racy_flags == {oracle_racy}, (ir.disassemble(prog), nb, nt)
        oracle_dead = any(int(f["kind"]) == O.F_DEADLOCK for f in res.faults)
        if not oracle_racy:
            n_free += 1
            # (ii) and (iv)
            assert len({(o.memory, o.deadlock, o.records) for o in outs}) == 1
            o = outs[0]
            assert list(o.memory) == res.memory.tolist()
            assert o.deadlock == oracle_dead
            assert Counter(dict(o.records)) == _rec_multiset(res)
        else:
            n_racy += 1
            # (iii)
            assert tuple(res.memory.tolist()) in {o.memory for o in outs}
    assert n_racy + n_free == 25
