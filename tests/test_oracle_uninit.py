"""Oracle pins of the uninitialised shared-memory check (the tool's checks
inherited from the C semantics include uninitialised memory accesses,
Section 3.2; CUDA leaves shared memory undefined at block start).

A load of a shared word no thread of the block has stored to earlier in the
block's lockstep order is a finding UNINIT {epoch, a = 0, b = tid, c = word,
d = pc of the load}.  Hand-derived cases fix every field and the order rules
(program order of one thread, earlier epochs, an earlier step; the loads of a
step before its stores); the brute-force enumeration (test_oracle_brute.py)
checks the findings against every interleaving of random kernels."""
import numpy as np

from oracle import oracle as O
from paper_1211_6193_amd import ir
from paper_1211_6193_amd.workloads import Job, LaunchSpec

UNINIT = 7


def _job(a, grid=1, block=4, sh_words=8, mem=None):
    prog = np.array(a.assemble(), dtype=np.uint64)
    mem = np.zeros(4, np.int32) if mem is None else mem
    return Job([LaunchSpec(prog, (grid, 1, 1), (block, 1, 1), 4 * sh_words, ())], mem, {})


def _uninit(res):
    return [f for f in res.fault_tuples() if f[1] == UNINIT]


def test_read_before_any_store_then_after_barrier():
    # pc: 0 SREG, 1 LDS sh[t+1], 2 STS sh[t], 3 BAR, 4 LDS sh[t+1], 5 EXIT
    a = ir.Asm()
    a.SREG(0, "TID").LDS(1, 0, 1).STS(0, 0, 0).BAR().LDS(2, 0, 1).EXIT()
    res = O.run_job(_job(a, grid=2, block=4, sh_words=5), uninit=True)
    # epoch 0: every thread reads word t+1 before anyone stored it (word 4 is
    # never stored: thread 3 reads it uninitialised in both epochs)
    want = [(0, UNINIT, b, 0, 0, t, t + 1, 1) for b in (0, 1) for t in range(4)]
    want += [(0, UNINIT, b, 1, 0, 3, 4, 4) for b in (0, 1)]
    assert sorted(_uninit(res)) == sorted(want)
    # off by default
    assert _uninit(O.run_job(_job(a, grid=2, block=4, sh_words=5))) == []


def test_own_store_initialises_for_the_same_thread():
    a = ir.Asm()
    a.SREG(0, "TID").STS(0, 0, 0).LDS(1, 0, 0).EXIT()
    assert _uninit(O.run_job(_job(a), uninit=True)) == []


def test_loads_of_a_step_come_before_its_stores():
    # thread 0 stores word 0 at the same step (pc 3 vs pc 5 after equal-length
    # paths) at which the others load it: the load reads it uninitialised
    # pc: 0 SREG, 1 BNZ r0 -> 4, 2 STS sh[0], 3 EXIT, 4 LDS sh[0], 5 EXIT
    a = ir.Asm()
    a.SREG(0, "TID").BNZ(0, "LD").STS(15, 0, 0).EXIT()
    a.label("LD").LDS(1, 15, 0).EXIT()
    res = O.run_job(_job(a), uninit=True)
    assert sorted(_uninit(res)) == [(0, UNINIT, 0, 0, 0, t, 0, 4) for t in (1, 2, 3)]
    assert len(res.races) == 1          # the same pair also races


def test_store_one_step_earlier_initialises():
    # thread 0's store is at step 2, the others' load at step 3 (one more
    # instruction on their path): initialised in the lockstep order
    a = ir.Asm()
    a.SREG(0, "TID").BNZ(0, "LD").STS(15, 0, 0).EXIT()
    a.label("LD").MOVI(2, 7).LDS(1, 15, 0).EXIT()
    res = O.run_job(_job(a), uninit=True)
    assert _uninit(res) == []


def test_out_of_bounds_load_is_not_uninit_and_findings_are_a_set():
    # a loop loads the same uninitialised word three times (one finding), and
    # an out-of-bounds word (an OOB finding only)
    a = ir.Asm()
    a.SREG(0, "TID").MOVI(2, 3)
    a.label("L").LDS(1, 15, 5).LDS(1, 15, 8).ADDI(2, 2, -1).BNZ(2, "L").EXIT()
    res = O.run_job(_job(a, block=2, sh_words=8), uninit=True)
    assert sorted(_uninit(res)) == [(0, UNINIT, 0, 0, 0, t, 5, 2) for t in (0, 1)]
    assert sorted(f for f in res.fault_tuples() if f[1] == O.F_OOB) == [(0, O.F_OOB, 0, 0, 0, t, 8, 0) for t in (0, 1)]


def test_each_block_starts_uninitialised():
    # block 0 stores word 0; block 1 only loads it: the store of another block
    # does not initialise a block's shared memory
    a = ir.Asm()
    a.SREG(0, "BID").BNZ(0, "LD").STS(15, 0, 0).EXIT()
    a.label("LD").LDS(1, 15, 0).EXIT()
    res = O.run_job(_job(a, grid=2, block=1), uninit=True)
    assert _uninit(res) == [(0, UNINIT, 1, 0, 0, 0, 0, 4)]


def test_check_changes_nothing_else():
    """Records, races, other findings and memory are the same with the check
    on and off, on the random kernels of the brute-force pins."""
    import test_oracle_brute as TB
    for prog, nb, nt, mem in TB._cases(25, 7000):
        job = Job([LaunchSpec(np.array(prog, dtype=np.uint64), (nb, 1, 1), (nt, 1, 1), 4 * TB.SH_WORDS, ())],
                  np.array(mem, dtype=np.int32))
        on, off = O.run_job(job, uninit=True), O.run_job(job)
        assert on.records == off.records and on.race_tuples() == off.race_tuples()
        assert [f for f in on.fault_tuples() if f[1] != UNINIT] == off.fault_tuples()
        assert np.array_equal(on.memory, off.memory)
