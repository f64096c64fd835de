"""Pin the oracle against brute-force enumeration of all interleavings.

For random tiny kernels (at most 4 threads in 1-2 blocks, a handful of memory
operations, barriers and tid-dependent branches) every interleaving the
semantics admits is explored by ``brute.enumerate_launch``:

(i)   the oracle reports a race  <=>  some interleaving races  <=>  all do;
(ii)  race-free  =>  one outcome (memory, deadlock, record multiset), equal to
      the oracle's;
(iii) racy  =>  the oracle's final memory is one of the reachable ones;
(iv)  race-free  =>  the oracle reports a deadlock  <=>  every maximal
      interleaving is stuck;
(v)   race-free  =>  the out-of-bounds, division-by-zero and fuel findings
      (every field) are the same in every interleaving and equal the
      oracle's; racy  =>  the oracle's (memory, findings) pair is reachable.

The kernels reach shared and global addresses below zero and past the end
(constant and data-dependent bases), divide by zero, and, in the fuel cases,
run out of fuel part-way.
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
    # r5 = 5 * bid - 1: a global base of -1 in block 0 and 4 in block 1
    a.SREG(0, "TID").SREG(1, "BID").ADDI(2, 0, 10).MULI(3, 1, 7).MULI(5, 1, 5).ADDI(5, 5, -1)
    n_stmt = rng.randint(2, 6)
    lab = 0
    for _ in range(n_stmt):
        kind = rng.choice(["sts", "lds", "stg", "ldg", "alu", "div", "bar", "barp", "cond"])
        # constant bases (tid, zero, bid, r5) and, now and then, a loaded value
        base = rng.choice([0, 15, 1, 5, 5, 4])
        if kind == "sts":
            a.STS(rng.choice([0, 15, 0, 15, 4]), rng.randint(-1, 3), rng.choice([2, 3, 4]))
        elif kind == "lds":
            a.LDS(rng.choice([2, 3, 4]), rng.choice([0, 15, 0, 15, 4]), rng.randint(-1, 3))
        elif kind == "stg":
            a.STG(base, rng.randint(-1, 4), rng.choice([2, 3, 4]))
        elif kind == "ldg":
            a.LDG(rng.choice([2, 3, 4]), base, rng.randint(-1, 4))
        elif kind == "div":
            # divisor zero (r15), the tid (zero in thread 0) or a loaded value
            getattr(a, rng.choice(["DIV", "REM"]))(rng.choice([2, 3, 4]), rng.choice([0, 2, 3]),
                                                   rng.choice([15, 0, 2, 4]))
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


def _oracle(prog, nb, nt, mem, fuel=O.DEFAULT_FUEL):
    job = Job([LaunchSpec(np.array(prog, dtype=np.uint64), (nb, 1, 1), (nt, 1, 1), 4 * SH_WORDS, ())],
              np.array(mem, dtype=np.int32))
    return O.run_job(job, keep_records=True, fuel=fuel, uninit=True)


# Per-access findings: the ones the brute-force interpreter produces too.
_ACCESS_KINDS = (O.F_OOB, O.F_FUEL, O.F_ARITH, O.F_UNINIT)


def _access_findings(res):
    """The oracle's OOB / FUEL / ARITH / UNINIT findings as brute's
    (kind, block, epoch, a, b, c); UNINIT's load pc (d) is pinned elsewhere."""
    out = set()
    for f in res.faults:
        if int(f["kind"]) in _ACCESS_KINDS:
            assert int(f["launch"]) == 0 and (int(f["d"]) == 0 or int(f["kind"]) == O.F_UNINIT)
            out.add((int(f["kind"]), int(f["block"]), int(f["epoch"]), int(f["a"]), int(f["b"]), int(f["c"])))
    return frozenset(out)


def _compare(prog, nb, nt, mem, fuel=O.DEFAULT_FUEL):
    """Check (i)-(v) for one kernel; returns whether it races."""
    res = _oracle(prog, nb, nt, mem, fuel)
    outs = brute.enumerate_launch(prog, nb, nt, SH_WORDS, mem, fuel=fuel)
    assert outs
    racy_flags = {o.racy for o in outs}
    oracle_racy = len(res.races) > 0
    # (i)
    assert racy_flags == {oracle_racy}, (ir.disassemble(prog), nb, nt)
    oracle_dead = any(int(f["kind"]) == O.F_DEADLOCK for f in res.faults)
    found = _access_findings(res)
    if not oracle_racy:
        # (ii), (iv) and (v)
        assert len({(o.memory, o.deadlock, o.records, o.findings) for o in outs}) == 1
        o = outs[0]
        assert list(o.memory) == res.memory.tolist()
        assert o.deadlock == oracle_dead
        assert Counter(dict(o.records)) == _rec_multiset(res)
        assert o.findings == found, (ir.disassemble(prog), nb, nt, sorted(o.findings), sorted(found))
    else:
        # (iii) and (v)
        assert (tuple(res.memory.tolist()), found) in {(o.memory, o.findings) for o in outs}
    return oracle_racy


def _rec_multiset(res):
    return Counter((int(r["space"]), int(r["addr"]), int(r["block"]), int(r["epoch"]), int(r["tid"]),
                    int(r["kind"])) for r in res.record_log)


@pytest.mark.parametrize("chunk", range(8))
def test_oracle_vs_all_interleavings(chunk):
    n_racy = 0
    for prog, nb, nt, mem in _cases(25, 7000 + chunk):
        n_racy += _compare(prog, nb, nt, mem)
    assert 0 < n_racy < 25


# Fuel small enough that some threads of most kernels run out part-way.
FUEL_CASES = [4, 6, 7, 9, 12]


def fuel_cases(n, seed):
    """(prog, nb, nt, mem, fuel) cases for the fuel pins (also run on the GPU)."""
    rng = random.Random(seed)
    return [c + (rng.choice(FUEL_CASES),) for c in _cases(n, seed)]


@pytest.mark.parametrize("chunk", range(3))
def test_oracle_vs_all_interleavings_with_little_fuel(chunk):
    for prog, nb, nt, mem, fuel in fuel_cases(20, 8100 + chunk):
        _compare(prog, nb, nt, mem, fuel)


def test_cases_reach_every_access_finding_field():
    """The random kernels exercise what the findings pins need: OOB loads and
    stores in both spaces at negative and past-the-end addresses, in epochs
    above 0 and in block 1, division by zero, and fuel running out."""
    seen = set()
    for chunk in range(8):
        for prog, nb, nt, mem in _cases(25, 7000 + chunk):
            for f in _oracle(prog, nb, nt, mem).faults:
                k = int(f["kind"])
                if k == O.F_OOB:
                    c = int(np.int32(np.uint32(f["c"])))
                    seen.add(("oob", int(f["a"]), "neg" if c < 0 else "past"))
                    if int(f["epoch"]) > 0:
                        seen.add(("oob-epoch>0",))
                    if int(f["block"]) > 0:
                        seen.add(("oob-block1",))
                elif k == O.F_ARITH:
                    seen.add(("arith",))
                elif k == O.F_UNINIT:
                    seen.add(("uninit", "block1" if int(f["block"]) else "block0",
                              "epoch>0" if int(f["epoch"]) else "epoch0"))
    for chunk in range(3):
        for prog, nb, nt, mem, fuel in fuel_cases(20, 8100 + chunk):
            if any(int(f["kind"]) == O.F_FUEL for f in _oracle(prog, nb, nt, mem, fuel).faults):
                seen.add(("fuel",))
    want = {("oob", a, side) for a in range(4) for side in ("neg", "past")}
    want |= {("oob-epoch>0",), ("oob-block1",), ("arith",), ("fuel",)}
    want |= {("uninit", b, e) for b in ("block0", "block1") for e in ("epoch0", "epoch>0")}
    assert want <= seen, sorted(want - seen)
