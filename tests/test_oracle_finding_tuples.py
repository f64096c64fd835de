"""Hand-derived pins of every field of the oracle's per-access findings.

Finding tuples are (launch, kind, block, epoch, a, b, c, d), sorted, without
repeats:
  OOB   = 3: a = 2 * space + (1 for a store) (space 0 shared, 1 global),
             b = tid, c = the address as a 32-bit two's-complement value;
             the load yields 0, the store is dropped, no access record;
  FUEL  = 4: b = tid (the thread's turn comes with no fuel left; it exits);
  ARITH = 5: b = tid, c = pc of the division.
The paper's tool flags out-of-bounds accesses and undefined behaviour
(Section 3.2, the kcc checks); division by zero and running out of fuel are
this build's readings of undefined behaviour and of termination.  Each
expected tuple below is worked out by hand from the kernel in the test, so a
swapped field (kind * 2 + space, an unsigned address, the wrong epoch, a pc
off by one, findings deduplicated across epochs) fails one of them.
"""
import numpy as np

from oracle import oracle as O
from paper_1211_6193_amd import ir
from paper_1211_6193_amd.workloads import Job, LaunchSpec

OOB, FUEL, ARITH, DEADLOCK = O.F_OOB, O.F_FUEL, O.F_ARITH, O.F_DEADLOCK
U32 = 1 << 32


def _run(asm, grid, block, shmem_words, memory, fuel=O.DEFAULT_FUEL):
    prog = np.array(asm.assemble(), dtype=np.uint64)
    job = Job([LaunchSpec(prog, (grid, 1, 1), (block, 1, 1), 4 * shmem_words, ())],
              np.array(memory, dtype=np.int32))
    return O.run_job(job, fuel=fuel, keep_records=True)


def test_oob_shared_load_past_the_end_in_epoch_1():
    # 4 threads, 2 shared words.  Epoch 0: thread t stores t+1 to shared[t]
    # (threads 2, 3: OOB stores at 2, 3).  Epoch 1: thread t loads shared[t]
    # (threads 2, 3: OOB loads at 2, 3, yielding 0) and stores the value to
    # global[t].
    a = ir.Asm()
    a.SREG(0, "TID").ADDI(1, 0, 1).STS(0, 0, 1).BAR().LDS(2, 0, 0).STG(0, 0, 2).EXIT()
    r = _run(a, 1, 4, 2, [-5, -5, -5, -5])
    assert r.fault_tuples() == [
        (0, OOB, 0, 0, 1, 2, 2, 0), (0, OOB, 0, 0, 1, 3, 3, 0),     # shared stores, epoch 0
        (0, OOB, 0, 1, 0, 2, 2, 0), (0, OOB, 0, 1, 0, 3, 3, 0),     # shared loads, epoch 1
    ]
    assert r.memory.tolist() == [1, 2, 0, 0]
    # in-bounds accesses only: 2 STS + 2 LDS + 4 STG
    assert r.records == 8


def test_oob_shared_store_at_negative_addresses():
    # thread t stores to shared[t - 3]: threads 0..2 hit -3, -2, -1 (dropped);
    # thread 3 writes shared[0] = 7, which thread 3 then copies to global[0].
    a = ir.Asm()
    a.SREG(0, "TID").MOVI(1, 7).STS(0, -3, 1).BAR().LDS(2, 15, 0).SEQI(3, 0, 3).BZ(3, "end") \
        .STG(15, 0, 2).label("end").EXIT()
    r = _run(a, 1, 4, 1, [0])
    assert r.fault_tuples() == [(0, OOB, 0, 0, 1, t, (t - 3) % U32, 0) for t in range(3)]
    assert r.memory.tolist() == [7]


def test_oob_global_load_and_store_both_ends_in_block_1():
    # 2 blocks x 2 threads, 5 global words.  g = 2*bid + tid.
    # load global[g + 2]: g = 3 -> 5 is past the end (block 1, tid 1), load 0;
    # store global[g - 2] = loaded value: g = 0, 1 -> -2, -1 (block 0), dropped.
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").MULI(2, 1, 2).ADD(2, 2, 0).LDG(3, 2, 2).STG(2, -2, 3).EXIT()
    r = _run(a, 2, 2, 0, [10, 11, 12, 13, 14])
    assert r.fault_tuples() == [
        (0, OOB, 0, 0, 3, 0, (-2) % U32, 0), (0, OOB, 0, 0, 3, 1, (-1) % U32, 0),
        (0, OOB, 1, 0, 2, 1, 5, 0),
    ]
    # g = 2 loads 14 and stores it to word 0; g = 3 loads 0 and stores it to word 1
    assert r.memory.tolist() == [14, 0, 12, 13, 14]
    assert r.records == 3 + 2          # loads of g = 0, 1, 2; stores of g = 2, 3


def test_oob_in_a_loop_is_one_finding_per_epoch():
    # thread 0 loads global[-1] five times in epoch 0 and twice in epoch 1:
    # identical tuples are reported once, so one finding per epoch.
    a = ir.Asm()
    a.SREG(0, "TID").BNZ(0, "skip").MOVI(1, 5).label("l0").LDG(2, 15, -1).ADDI(1, 1, -1).BNZ(1, "l0") \
        .label("skip").BAR().BNZ(0, "end").MOVI(1, 2).label("l1").LDG(2, 15, -1).ADDI(1, 1, -1) \
        .BNZ(1, "l1").label("end").EXIT()
    r = _run(a, 1, 2, 0, [3])
    assert r.fault_tuples() == [(0, OOB, 0, 0, 2, 0, U32 - 1, 0), (0, OOB, 0, 1, 2, 0, U32 - 1, 0)]
    assert r.records == 0


def test_fuel_in_epoch_1_per_block():
    # SREG, BAR, MOV, then a countdown of tid iterations (BZ, ADDI, JMP), then
    # the taken BZ and EXIT: thread t needs 5 + 3t instructions.  With fuel 9,
    # threads 0 (5) and 1 (8) finish; threads 2 and 3 spend their 9th unit on
    # the second iteration's JMP and find no fuel at the loop head in epoch 1.
    a = ir.Asm()
    a.SREG(0, "TID").BAR().MOV(2, 0).label("top").BZ(2, "end").ADDI(2, 2, -1).JMP("top") \
        .label("end").EXIT()
    r = _run(a, 2, 4, 0, [0], fuel=9)
    assert r.fault_tuples() == [(0, FUEL, b, 1, 0, t, 0, 0) for b in (0, 1) for t in (2, 3)]
    assert r.instructions == 2 * (5 + 8 + 9 + 9)


def test_fuel_before_a_barrier_then_deadlock():
    # countdown of tid iterations before the barrier: thread t needs 3 + 3t to
    # reach it, 4 + 3t to wait.  With fuel 12 thread 3 (13) arrives at the
    # barrier's pc with no fuel: FUEL in epoch 0, it exits, and threads 0-2
    # wait for ever: DEADLOCK {a = 3 waiting, b = 0, c = 3}.
    a = ir.Asm()
    a.SREG(0, "TID").MOV(2, 0).label("top").BZ(2, "bar").ADDI(2, 2, -1).JMP("top") \
        .label("bar").BAR().EXIT()
    r = _run(a, 1, 4, 0, [0], fuel=12)
    assert r.fault_tuples() == [(0, DEADLOCK, 0, 0, 3, 0, 3, 0), (0, FUEL, 0, 0, 0, 3, 0, 0)]
    assert r.launches_completed == 0


def test_fuel_at_the_end_of_the_program_is_no_finding():
    # one instruction and no EXIT: with fuel 1 the thread spends it and then
    # falls off the end, which is an exit, not a FUEL finding.
    a = ir.Asm()
    a.SREG(0, "TID")
    r = _run(a, 1, 3, 0, [0], fuel=1)
    assert r.fault_tuples() == []
    r = _run(a.EXIT(), 1, 3, 0, [0], fuel=1)
    assert r.fault_tuples() == [(0, FUEL, 0, 0, 0, t, 0, 0) for t in range(3)]


def test_arith_tid_and_pc():
    # pc 2: DIV by (t - 2): thread 2 in epoch 0.  pc 4: REMI by 0: every
    # thread in epoch 1.  pc 6: DIV by (t < 1): threads 1..3 in epoch 1.
    a = ir.Asm()
    a.SREG(0, "TID").ADDI(1, 0, -2).DIV(3, 0, 1).BAR().REMI(4, 0, 0).SLTI(5, 0, 1).DIV(6, 0, 5) \
        .MULI(7, 0, 3).STG(7, 0, 3).STG(7, 1, 4).STG(7, 2, 6).EXIT()
    r = _run(a, 1, 4, 0, [9] * 12)
    want = [(0, ARITH, 0, 0, 0, 2, 2, 0)]
    want += sorted([(0, ARITH, 0, 1, 0, t, 4, 0) for t in range(4)] +
                   [(0, ARITH, 0, 1, 0, t, 6, 0) for t in range(1, 4)])
    assert r.fault_tuples() == want
    # quotients t / (t - 2) = 0, -1, 0 (x/0), 3; remainders all 0; t / (t < 1) = 0 (0/1), then x/0 = 0
    assert r.memory.reshape(4, 3).tolist() == [[0, 0, 0], [-1, 0, 0], [0, 0, 0], [3, 0, 0]]


def test_arith_in_block_3_of_a_3d_grid():
    # DIV by (bid - 3) at pc 2 for every thread of block 3 only
    a = ir.Asm()
    a.SREG(0, "BID").ADDI(1, 0, -3).DIV(2, 0, 1).EXIT()
    prog = np.array(a.assemble(), dtype=np.uint64)
    job = Job([LaunchSpec(prog, (2, 2, 1), (2, 1, 1), 0, ())], np.zeros(1, np.int32))
    r = O.run_job(job)
    assert r.fault_tuples() == [(0, ARITH, 3, 0, 0, t, 2, 0) for t in range(2)]
