"""GPU parity: every report (races, findings, record count, completed
launches) and the final memory equal the CPU oracle's, bit for bit.

Cases: Figure 1 in all variants (plain and as a two-launch job), random tiny
kernels, tree reductions with injected faults, the three mixed families with
every fault, workload 2 at full size, a sample of workload 3, the ping-pong
stencil with cross-block races, and edge cases (fuel, division by zero,
out-of-bounds, 3-D shapes, 1024-thread blocks, falling off the program)."""
import random

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import test_oracle_brute as TB
from gpu_util import assert_same, check_jobs, say
from oracle import oracle as O
from paper_1211_6193_amd import ir, kc
from paper_1211_6193_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = kc.Context(0)
    yield c
    c.close()


def test_fig1_all_variants_as_jobs(ctx):
    for job in W.config1_jobs():
        say(f"fig1 job {job.meta}")
        rep, mem = kc.run_job(ctx, job)
        assert_same(rep, mem, O.run_job(job), str(job.meta))
    rep, mem = kc.run_job(ctx, W.fig1_job("BASE"))
    assert int(mem[18]) == 767


def test_fig1_plain_launch(ctx):
    for v in W.SUM_VARIANTS:
        job = W.fig1_job(v)
        job.launches = job.launches[:1]
        say(f"fig1 plain launch {v}")
        mem = torch.from_numpy(job.memory.copy()).cuda()
        L = job.launches[0]
        rep = kc.launch(ctx, ctx.program(L.program), L.grid, L.block, L.shmem_bytes, mem, L.params)
        assert_same(rep, mem, O.run_job(job), v)


def test_random_tiny_kernels(ctx):
    jobs = []
    for chunk in range(8):
        for prog, nb, nt, mem in TB._cases(25, 7000 + chunk):
            jobs.append(W.Job([W.LaunchSpec(np.array(prog, dtype=np.uint64), (nb, 1, 1), (nt, 1, 1),
                                            4 * TB.SH_WORDS, ())], np.array(mem, dtype=np.int32)))
    check_jobs(ctx, jobs, label="tiny-batched")
    for i, j in enumerate(jobs[:40]):
        say(f"tiny plain {i}")
        rep, mem = kc.run_job(ctx, j)
        assert_same(rep, mem, O.run_job(j), f"tiny {i}")


def test_random_tiny_kernels_with_little_fuel(ctx):
    """The brute-force fuel cases: threads run out of fuel part-way, next to
    out-of-bounds accesses and divisions by zero (every finding field)."""
    by_fuel = {}
    for chunk in range(3):
        for prog, nb, nt, mem, fuel in TB.fuel_cases(20, 8100 + chunk):
            by_fuel.setdefault(fuel, []).append(
                W.Job([W.LaunchSpec(np.array(prog, dtype=np.uint64), (nb, 1, 1), (nt, 1, 1), 4 * TB.SH_WORDS,
                                    ())], np.array(mem, dtype=np.int32)))
    try:
        for fuel, jobs in sorted(by_fuel.items()):
            ctx.set_option("fuel", fuel)
            check_jobs(ctx, jobs, fuel=fuel, label=f"tiny-fuel-{fuel}")
    finally:
        ctx.set_option("fuel", O.DEFAULT_FUEL)


def test_tree_tables_with_faults(ctx):
    job = W.tree256_job(n_blocks=64, threads=256, drop_frac=0.0, div_frac=0.0, seed=11)
    n = job.meta["n"]
    for b, k in [(3, 0), (7, 3), (20, 6), (21, 7), (40, 1)]:
        job.memory[n + 64 + b] = k
    for b, j in [(9, 2), (50, 5)]:
        job.memory[n + 128 + b] = j
    say("tree 64x256 with drops/divs")
    rep, mem = kc.run_job(ctx, job)
    assert_same(rep, mem, O.run_job(job), "tree")


@pytest.mark.parametrize("family", W.FAMILIES)
def test_families_every_fault(ctx, family):
    rng = np.random.default_rng(hash(family) % 1000)
    jobs = []
    for threads in (32, 96, 256, 1024):
        for nb in (1, 3, 7):
            for fault in (None,) + W.FAULTS[family]:
                fb = int(rng.integers(0, nb))
                lvl = int(rng.integers(0, 5))
                jobs.append(W.family_job(family, nb, threads, rng, fault, fb, lvl))
    check_jobs(ctx, jobs, label=f"{family}-faults")


def test_workload2_full_size(ctx):
    job = W.tree256_job()
    say("workload 2 full: 4096 x 256")
    rep, mem = kc.run_job(ctx, job)
    assert_same(rep, mem, O.run_job(job), "workload2")
    assert len(rep.races) > 0


def test_workload3_sample(ctx):
    jobs = W.config3_jobs(n=300)
    check_jobs(ctx, jobs, label="workload3-sample")


def test_pingpong_cross_block(ctx):
    job = W.stencil_pingpong_job(n=1 << 14, threads=256, steps=4, bug_frac=0.0, seed=3)
    n, nb = job.meta["n"], job.meta["n_blocks"]
    for b in (0, 5, 6, 30, nb - 1):
        job.memory[2 * n + b] = 1
    say("ping-pong stencil 2^14 x 4 steps with in-place bugs")
    rep, mem = kc.run_job(ctx, job)
    assert_same(rep, mem, O.run_job(job), "pingpong")
    assert any(r[2] == 1 for r in rep.race_tuples())


def _single(prog, grid, block, shmem, mem, params=()):
    return W.Job([W.LaunchSpec(np.array(prog, dtype=np.uint64), grid, block, shmem, params)],
                 np.array(mem, dtype=np.int32))


def test_edge_cases(ctx):
    cases = []
    # infinite loop -> FUEL for every thread
    a = ir.Asm(); a.label("L").ADDI(1, 1, 1).JMP("L")
    cases.append(("fuel", _single(a.assemble(), (2, 1, 1), (70, 1, 1), 0, [0])))
    # division by zero and INT_MIN / -1
    a = ir.Asm(); a.SREG(0, "TID").MOVI(1, -2**31).MOVI(2, -1).DIV(3, 1, 2).REM(4, 1, 0).STG(0, 0, 3).STG(0, 8, 4).EXIT()
    cases.append(("arith", _single(a.assemble(), (1, 1, 1), (8, 1, 1), 0, [0] * 16)))
    # out-of-bounds loads and stores in both spaces
    a = ir.Asm(); a.SREG(0, "TID").ADDI(1, 0, -2).LDS(2, 1, 0).STS(1, 5, 0).LDG(3, 0, 10).STG(0, 12, 3).EXIT()
    cases.append(("oob", _single(a.assemble(), (2, 1, 1), (8, 1, 1), 16, list(range(16)))))
    # 3-D grid and block, all special registers
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0).MULI(3, 3, 24)
    for i in range(24):
        a.SREG(4, i).STG(3, i, 4)
    a.EXIT()
    cases.append(("3d", _single(a.assemble(), (3, 2, 2), (5, 3, 2), 0, [0] * (12 * 30 * 24),
                                tuple(range(-3, 5)))))
    # 1024-thread block, shared-memory race across waves
    a = ir.Asm(); a.SREG(0, "TID").ANDI(1, 0, 7).STS(1, 0, 0).LDS(2, 1, 1).STG(0, 0, 2).EXIT()
    cases.append(("1024", _single(a.assemble(), (2, 1, 1), (1024, 1, 1), 64, [0] * 1024)))
    # falling off the end, empty shared memory
    a = ir.Asm(); a.SREG(0, "TID").STG(0, 0, 0)
    cases.append(("falloff", _single(a.assemble(), (1, 1, 1), (33, 1, 1), 0, [0] * 33)))
    # barrier divergence inside one wave, then deadlock
    a = ir.Asm(); a.SREG(0, "TID").ANDI(1, 0, 1).BZ(1, "E").BAR().BAR().label("E").BAR().EXIT()
    cases.append(("wave-div", _single(a.assemble(), (2, 1, 1), (6, 1, 1), 0, [0])))
    fuel = 5000
    ctx.set_option("fuel", fuel)
    try:
        for name, job in cases:
            say(f"edge {name}")
            rep, mem = kc.run_job(ctx, job)
            assert_same(rep, mem, O.run_job(job, fuel=fuel), name)
    finally:
        ctx.set_option("fuel", O.DEFAULT_FUEL)


def _redirect_program(reader_block_reads_0: bool):
    """Block 0: thread 0 writes shared[0] = 5 while thread 1 reads shared[0]
    without a barrier and stores its tid to global[that value].  Under the
    canonical lockstep schedule thread 1 reads 0; a free-running wave may read 5.
    Block 1 (optional) reads global[0]."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(3, "BID").BNZ(3, "B1")
    a.BNZ(0, "L1").MOVI(1, 5).STS(15, 0, 1).JMP("END")
    a.label("L1").SEQI(4, 0, 1).BZ(4, "END").LDS(2, 15, 0).STG(2, 0, 0).JMP("END")
    a.label("B1")
    if reader_block_reads_0:
        a.BNZ(0, "END").LDG(5, 15, 0).STG(15, 9, 5)
    a.label("END").EXIT()
    return a.assemble()


def test_replay_paths(ctx):
    for reads0 in (False, True):
        job = _single(_redirect_program(reads0), (2, 1, 1), (2, 1, 1), 16, [7] * 10)
        say(f"replay path, second block reads global[0]: {reads0}")
        ctx.reset_stats()
        rep, mem = kc.run_job(ctx, job)
        assert_same(rep, mem, O.run_job(job), f"redirect {reads0}")
        assert ctx.stat("replays") >= 1


def test_replay_exactness_paths(ctx):
    """Logs (of the free run or of a replay) whose records are all
    representatives and share no written location between blocks are checked
    through a hash table of locations (no sort); cross-block components take
    the sorted check.  Both must equal the oracle."""
    job = W.tree256_job(n_blocks=256, drop_frac=0.05, div_frac=0.01, seed=9)
    say("tree replay: hash-table exactness")
    ctx.reset_stats()
    rep, mem = kc.run_job(ctx, job)
    assert_same(rep, mem, O.run_job(job), "tree replay")
    assert ctx.stat("replays") >= 1 and ctx.stat("replay_sorted_checks") == 0 and ctx.stat("fallbacks") == 0
    assert ctx.stat("sorted_checks") == 0          # its free-run log had no cross-block conflict either
    # the same on a memory much larger than the log: locations go to the hash
    # table instead of one entry per memory word
    job = W.tree256_job(n_blocks=64, drop_frac=0.1, div_frac=0.03, seed=10)
    job.memory = np.concatenate([job.memory, np.zeros(1 << 20, np.int32)])
    say("tree replay on a large memory: hash-table check")
    ctx.reset_stats()
    rep, mem = kc.run_job(ctx, job)
    assert_same(rep, mem, O.run_job(job), "tree replay, large memory")
    assert ctx.stat("replays") >= 1 and ctx.stat("sorted_checks") == 0 and ctx.stat("replay_sorted_checks") == 0
    job = W.stencil_pingpong_job(n=1 << 12, threads=256, steps=2, bug_frac=0.0, seed=4)
    n, nb = job.meta["n"], job.meta["n_blocks"]
    for b in (1, 6, nb - 1):
        job.memory[2 * n + b] = 1
    say("cross-block components: sorted check")
    ctx.reset_stats()
    rep, mem = kc.run_job(ctx, job)
    assert_same(rep, mem, O.run_job(job), "pingpong components")
    assert ctx.stat("replays") >= 1 and ctx.stat("replay_sorted_checks") >= 1 and ctx.stat("sorted_checks") >= 1


def test_instruction_count_of_race_free_runs(ctx):
    # A race-free free run executes the canonical per-thread traces, so the
    # library's count of executed thread-instructions equals the oracle's.
    rng = np.random.default_rng(7)
    jobs = [W.family_job(f, 4, 96, rng) for f in ("TREE", "STENCIL", "TRANSPOSE")]
    jobs.append(W.tree256_job(n_blocks=96, drop_frac=0.0, div_frac=0.0))
    for job in jobs:
        orc = O.run_job(job)
        assert len(orc.races) == 0
        ctx.reset_stats()
        rep, mem = kc.run_job(ctx, job)
        assert_same(rep, mem, orc, job.meta["family"])
        assert int(ctx.stat("instructions")) == orc.instructions, job.meta["family"]


def _hot_word_program():
    """Every thread of every block reads global[0] and global[1], stores its
    tid to shared[0] (a write-write race among all threads of a block) and, in
    block 5, thread 3 writes global[0] (a cross-block race with every reader);
    thread 9 of every block writes global[1] (intra- and cross-block races);
    after a barrier every thread reads shared[0].  The conflict segments of
    global[0], global[1] and shared[0] are far longer than a head thread
    reduces alone."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").MOVI(3, 0)
    a.LDG(2, 3, 0).LDG(4, 3, 1).STS(3, 0, 0)
    a.SEQI(5, 1, 5).SEQI(6, 0, 3).AND(5, 5, 6).BZ(5, "N").STG(3, 0, 0)
    a.label("N").SEQI(6, 0, 9).BZ(6, "M").STG(3, 1, 0)
    a.label("M").BAR().LDS(7, 3, 0).ADD(7, 7, 2).ADD(7, 7, 4).STG(1, 16, 7).EXIT()
    return a.assemble()


@pytest.mark.parametrize("local", [1, 0])
def test_long_conflict_segments(ctx, local):
    job = _single(_hot_word_program(), (40, 1, 1), (256, 1, 1), 4, [3, 4] + [0] * 14 + [0] * 40)
    say(f"long segments, local check {local}")
    ctx.set_option("local", local)
    try:
        rep, mem = kc.run_job(ctx, job)
        orc = O.run_job(job)
        assert len(orc.races) > 0
        assert_same(rep, mem, orc, f"long segments local={local}")
    finally:
        ctx.set_option("local", 1)


def test_replay_with_long_shared_reads(ctx):
    """Every block reads global[1]; block 7 races on shared memory and is
    replayed.  The exactness check then meets a location with many free-run
    records (all reads), which a whole workgroup scans; the replay stays exact."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").MOVI(3, 0).LDG(2, 3, 1)
    a.SEQI(5, 1, 7).BZ(5, "N").STS(3, 0, 0)
    a.label("N").BAR().BNZ(0, "E").LDS(6, 3, 0).ADD(6, 6, 2).STG(1, 16, 6)
    a.label("E").EXIT()
    for local in (1, 0):
        job = _single(a.assemble(), (64, 1, 1), (128, 1, 1), 4, [0, 11] + [0] * 14 + [0] * 64)
        say(f"replay with long read segment, local check {local}")
        ctx.set_option("local", local)
        try:
            ctx.reset_stats()
            rep, mem = kc.run_job(ctx, job)
            orc = O.run_job(job)
            assert len(orc.races) == 1
            assert_same(rep, mem, orc, f"long read segment local={local}")
            assert ctx.stat("replays") >= 1 and ctx.stat("fallbacks") == 0
        finally:
            ctx.set_option("local", 1)
