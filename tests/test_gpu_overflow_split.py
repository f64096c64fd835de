"""A batch whose access-record key cannot hold its units' fields together.

4,096 jobs in one batch: 4,095 of one 64-thread block over 64 words and one of
65,536 blocks over 2^22 words, all running a program with 200 barriers (each
thread adds to its own word between them).  Together the key needs 12 unit
bits beside 6 tid, 16 block and 22 address bits, which leaves room for 30
epochs where the program has 201: the library splits the batch into smaller groups
(memories back at the launch start) instead of failing.  Every job's report
and final memory equal those of the job run alone, and a sample equals the
oracle's."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import assert_same, say
from oracle import oracle as O
from paper_1211_6193_amd import ir, kc
from paper_1211_6193_amd import workloads as W

pytestmark = pytest.mark.gpu

N_BAR = 200


def barrier_loop_program():
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").SREG(3, "PARAM0")
    a.MUL(4, 1, 2).ADD(4, 4, 0).REM(4, 4, 3)          # word = (bid * T + tid) % n
    a.MOVI(5, N_BAR)
    a.label("LOOP")
    a.BZ(5, "END")
    a.LDG(6, 4, 0).ADD(6, 6, 5).STG(4, 0, 6).BAR()
    a.ADDI(5, 5, -1).JMP("LOOP")
    a.label("END")
    a.EXIT()
    return np.array(a.assemble(), dtype=np.uint64)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = kc.Context(0)
    yield c
    c.close()


def test_overwide_batch_is_split_not_refused(ctx):
    prog = barrier_loop_program()
    rng = np.random.default_rng(3)
    jobs = []
    for i in range(4095):
        mem = rng.integers(0, 1000, 64).astype(np.int32)
        jobs.append(W.Job([W.LaunchSpec(prog, (1, 1, 1), (64, 1, 1), 0, (64,))], mem, {"i": i}))
    big = rng.integers(0, 1000, 1 << 22).astype(np.int32)
    jobs.append(W.Job([W.LaunchSpec(prog, (1 << 16, 1, 1), (64, 1, 1), 0, (1 << 22,))], big, {"i": 4095}))
    ctx.reset_stats()
    say("4096 jobs whose record key does not fit together")
    reps, mems = kc.run_jobs(ctx, jobs)
    assert ctx.stat("stage_splits") >= 1
    for i in list(range(0, 4095, 257)) + [4095]:
        j = jobs[i]
        L = j.launches[0]
        m = torch.from_numpy(j.memory.copy()).cuda()
        alone = kc.launch(ctx, ctx.program(L.program), L.grid, L.block, L.shmem_bytes, m, L.params)
        assert alone.records == reps[i].records and alone.race_tuples() == reps[i].race_tuples()
        assert alone.fault_tuples() == reps[i].fault_tuples()
        assert torch.equal(m, mems[i]), i
    for i in (0, 1, 2, 4094):
        assert_same(reps[i], mems[i], O.run_job(jobs[i]), f"job {i}")
    # the big job's result has a closed form: each word (one thread's) gains 200 + 199 + ... + 1
    want = jobs[4095].memory.astype(np.int64) + N_BAR * (N_BAR + 1) // 2
    assert np.array_equal(mems[4095].cpu().numpy(), want.astype(np.int32))
