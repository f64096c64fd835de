"""Oracle pins of the warp-aware model (option warp).

The paper's Section 4 names a finer model of the scheduler as future work:
threads grouped into warps that execute instructions in lock-step, which the
race check could then take into account.  Reading: warps are 32 consecutive
linear tids; two accesses of one block and epoch by threads of one warp are
ordered by the warp's instruction order unless they run at the same lockstep
step, so only then do they conflict; threads of different warps are unordered
until the barrier, as before.  The tuple reports w = the smallest thread with
a conflicting write and o = the smallest other thread whose access conflicts
with one of w's writes.  Every case below is derived by hand."""
import numpy as np

from oracle import oracle as O
from paper_1211_6193_amd import ir
from paper_1211_6193_amd.workloads import Job, LaunchSpec


def _job(a, grid=1, block=32, sh_words=64, mem=None):
    prog = np.array(a.assemble(), dtype=np.uint64)
    mem = np.zeros(8, np.int32) if mem is None else mem
    return Job([LaunchSpec(prog, (grid, 1, 1), (block, 1, 1), 4 * sh_words, ())], mem, {})


def warp_sync_reduction(first_barrier=True, start=16):
    """sh[t] = t + 1; [barrier]; for s = start, start/2, .., 1: if t < s:
    sh[t] += sh[t + s] -- no barrier inside the loop; thread 0 stores the sum."""
    a = ir.Asm()
    a.SREG(0, "TID").ADDI(1, 0, 1).STS(0, 0, 1)
    if first_barrier:
        a.BAR()
    a.MOVI(2, start)
    a.label("L").BZ(2, "DONE").SLT(3, 0, 2).BZ(3, "SKIP")
    a.ADD(4, 0, 2).LDS(5, 0, 0).LDS(6, 4, 0).ADD(5, 5, 6).STS(0, 0, 5)
    a.label("SKIP").SHRAI(2, 2, 1).JMP("L")
    a.label("DONE").BNZ(0, "END").LDS(5, 15, 0).STG(15, 0, 5)
    a.label("END").EXIT()
    return a


def test_warp_synchronous_reduction_in_one_warp_is_race_free():
    job = _job(warp_sync_reduction(), block=32)
    std, wrp = O.run_job(job), O.run_job(job, warp=True)
    assert len(std.races) > 0                   # unordered by barriers: races in the plain model
    assert wrp.races.size == 0                  # ordered by the warp's lock-step
    assert int(wrp.memory[0]) == 32 * 33 // 2   # the sum
    assert np.array_equal(std.memory, wrp.memory) and std.records == wrp.records


def test_two_warps_behind_a_barrier_are_race_free():
    # level 32 reads the other warp's words, stored before the barrier
    job = _job(warp_sync_reduction(start=32), block=64)
    assert O.run_job(job, warp=True).races.size == 0
    assert int(O.run_job(job, warp=True).memory[0]) == 64 * 65 // 2


def test_other_warp_without_the_barrier_races():
    # without the barrier, warp 0 reads warp 1's words in the epoch they are
    # stored: one tuple per such word, (w = the storing thread of warp 1, o = the
    # reading thread of warp 0); same-warp pairs stay ordered
    job = _job(warp_sync_reduction(first_barrier=False, start=32), block=64)
    got = O.run_job(job, warp=True).race_tuples()
    assert got == [(0, 0, 0, 0, 0, a, a, a - 32) for a in range(32, 64)]
    assert len(O.run_job(job).races) > 32       # the plain model also reports the same-warp words


def test_one_instruction_storing_twice_races():
    # lanes 2k and 2k+1 store word k in the same instruction: the same step
    a = ir.Asm()
    a.SREG(0, "TID").SHRAI(1, 0, 1).STS(1, 0, 0).EXIT()
    got = O.run_job(_job(a, block=4, sh_words=2), warp=True).race_tuples()
    assert got == [(0, 0, 0, 0, 0, 0, 0, 1), (0, 0, 0, 0, 0, 1, 2, 3)]


def _diverged(extra_on_load_path):
    # lane 0 stores word 0 on one path, lane 1 loads it on the other
    a = ir.Asm()
    a.SREG(0, "TID").BNZ(0, "LD").STS(15, 0, 0).EXIT()
    a.label("LD").SEQI(1, 0, 1).BZ(1, "END")
    for _ in range(extra_on_load_path):
        a.MOVI(2, 0)
    a.LDS(3, 15, 0)
    a.label("END").EXIT()
    return a


def test_diverged_lanes_race_only_at_the_same_step():
    # steps: SREG 0, BNZ 1; lane 0: STS at 2.  lane 1: SEQI 2, BZ 3, [MOVI 4], LDS 4 [5]
    same = _job(_diverged(0), block=2, sh_words=1)
    later = _job(_diverged(1), block=2, sh_words=1)
    # lane 0 stores at step 2, lane 1 loads at step 4 or 5: ordered within the warp
    assert O.run_job(same, warp=True).races.size == 0 and O.run_job(later, warp=True).races.size == 0
    # a store and a load at the same step: put lane 0's store two steps later
    a = ir.Asm()
    a.SREG(0, "TID").BNZ(0, "LD").MOVI(2, 0).MOVI(2, 0).STS(15, 0, 0).EXIT()
    a.label("LD").SEQI(1, 0, 1).BZ(1, "END").LDS(3, 15, 0)
    a.label("END").EXIT()
    got = O.run_job(_job(a, block=2, sh_words=1), warp=True).race_tuples()
    assert got == [(0, 0, 0, 0, 0, 0, 0, 1)]
    for j in (same, later):
        assert O.run_job(j).race_tuples() == [(0, 0, 0, 0, 0, 0, 0, 1)]   # the plain model: always


def test_other_thread_is_the_smallest_conflicting_one():
    # word 0: stored by thread 0 (step 2), loaded by thread 1 (a later step,
    # same warp) and thread 32 (another warp): o = 32, not 1
    a = ir.Asm()
    a.SREG(0, "TID").BNZ(0, "LD").STS(15, 0, 0).EXIT()
    a.label("LD").MOVI(2, 0).MOVI(2, 0).LDS(3, 15, 0).EXIT()
    job = _job(a, block=64, sh_words=1)
    assert O.run_job(job, warp=True).race_tuples() == [(0, 0, 0, 0, 0, 0, 0, 32)]
    assert O.run_job(job).race_tuples() == [(0, 0, 0, 0, 0, 0, 0, 1)]


def test_global_memory_follows_the_same_rule_and_cross_block_is_unchanged():
    # global word 0: same block, same warp, different steps -> ordered;
    # two blocks storing global word 1 -> a cross-block race in both models
    a = ir.Asm()
    a.SREG(0, "TID").BNZ(0, "LD").STG(15, 0, 0).MOVI(4, 1).SREG(5, "BID").STG(4, 0, 5).EXIT()
    a.label("LD").MOVI(2, 0).MOVI(2, 0).LDG(3, 15, 0).EXIT()
    job = _job(a, grid=2, block=2, sh_words=0)
    wrp = O.run_job(job, warp=True).race_tuples()
    std = O.run_job(job).race_tuples()
    cross = [r for r in std if r[2] == 1]
    assert cross and [r for r in wrp if r[2] == 1] == cross
    assert [r for r in wrp if r[2] == 0 and r[5] == 0] == []
    assert [r for r in std if r[2] == 0 and r[5] == 0] == [(0, 1, 0, b, 0, 0, 0, 1) for b in (0, 1)]


def test_model_changes_nothing_but_intra_block_tuples():
    """Records, findings, memory and cross-block tuples are the same in both
    models on the brute-force pins' random kernels, and every warp-aware
    intra-block tuple's location also races in the plain model."""
    import test_oracle_brute as TB
    for prog, nb, nt, mem in TB._cases(25, 7000):
        job = Job([LaunchSpec(np.array(prog, dtype=np.uint64), (nb, 1, 1), (nt, 1, 1), 4 * TB.SH_WORDS, ())],
                  np.array(mem, dtype=np.int32))
        w, s = O.run_job(job, warp=True), O.run_job(job)
        assert w.records == s.records and w.fault_tuples() == s.fault_tuples()
        assert np.array_equal(w.memory, s.memory)
        assert [r for r in w.race_tuples() if r[2] != 0] == [r for r in s.race_tuples() if r[2] != 0]
        plain_locs = {r[:6] for r in s.race_tuples() if r[2] == 0}
        assert {r[:6] for r in w.race_tuples() if r[2] == 0} <= plain_locs
