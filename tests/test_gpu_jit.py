"""Program-specialised kernels: with option "jit" = 1 every free run compiles
(at first use) and runs its program's specialised kernels, and the replay of a
single-program stage runs its specialised lockstep kernel, so these cases run
the specialised code
(checked through the "jit_launches" statistic) and must equal the CPU oracle
bit for bit, like the interpreter.  Covers the Figure 1 variants, random tiny
kernels, the fault families, workload 2 at full size, fuel exhaustion inside
basic blocks, division by zero, out-of-bounds accesses, 3-D shapes, 1024-thread
blocks, falling off the program, barrier divergence inside a wave, long
conflict segments and replays next to specialised free runs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import test_gpu_parity as P
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
    c.set_option("jit", 1)
    yield c
    c.close()


def _run(ctx, job, what, fuel=O.DEFAULT_FUEL):
    ctx.reset_stats()
    rep, mem = kc.run_job(ctx, job)
    orc = O.run_job(job, fuel=fuel)
    assert_same(rep, mem, orc, what)
    ran = min(len(job.launches), orc.launches_completed + 1)      # a deadlocked launch ends the job
    assert ctx.stat("jit_launches") >= ran, (what, "specialised kernels did not run")


def test_jit_fig1(ctx):
    for job in W.config1_jobs():
        say(f"jit fig1 {job.meta}")
        _run(ctx, job, str(job.meta))


def test_jit_random_tiny_kernels(ctx):
    jobs = []
    for prog, nb, nt, mem in TB._cases(24, 9100):
        jobs.append(W.Job([W.LaunchSpec(np.array(prog, dtype=np.uint64), (nb, 1, 1), (nt, 1, 1),
                                        4 * TB.SH_WORDS, ())], np.array(mem, dtype=np.int32)))
    for i, j in enumerate(jobs):
        say(f"jit tiny {i}")
        _run(ctx, j, f"tiny {i}")
    ctx.reset_stats()
    check_jobs(ctx, jobs, label="jit tiny batched")
    assert ctx.stat("jit_launches") >= 1


def test_jit_families(ctx):
    rng = np.random.default_rng(5)
    jobs = []
    for family in W.FAMILIES:
        for threads in (32, 256, 1024):
            for fault in (None,) + W.FAULTS[family]:
                nb = int(rng.integers(1, 6))
                jobs.append(W.family_job(family, nb, threads, rng, fault, int(rng.integers(0, nb)),
                                         int(rng.integers(0, 5))))
    ctx.reset_stats()
    check_jobs(ctx, jobs, label="jit families")
    assert ctx.stat("jit_launches") >= 1


def test_jit_workload2_full_size(ctx):
    say("jit workload 2 full size")
    _run(ctx, W.tree256_job(), "workload2")
    assert ctx.stat("jit_replays") >= 1          # its racy blocks replay on specialised kernels


def test_jit_edge_cases(ctx):
    cases = []
    a = ir.Asm(); a.label("L").ADDI(1, 1, 1).JMP("L")
    cases.append(("fuel-loop", P._single(a.assemble(), (2, 1, 1), (70, 1, 1), 0, [0])))
    # fuel running out inside a long basic block, differently per lane
    a = ir.Asm(); a.SREG(0, "TID").MULI(0, 0, 40).label("L").BZ(0, "E").SUBI(0, 0, 1)
    for _ in range(9):
        a.ADDI(2, 2, 3)
    a.STG(15, 0, 2).JMP("L").label("E").EXIT()
    cases.append(("fuel-in-block", P._single(a.assemble(), (1, 1, 1), (64, 1, 1), 0, [0])))
    a = ir.Asm(); a.SREG(0, "TID").MOVI(1, -2**31).MOVI(2, -1).DIV(3, 1, 2).REM(4, 1, 0).STG(0, 0, 3).STG(0, 8, 4).EXIT()
    cases.append(("arith", P._single(a.assemble(), (1, 1, 1), (8, 1, 1), 0, [0] * 16)))
    a = ir.Asm(); a.SREG(0, "TID").DIVI(3, 0, 0).REMI(4, 0, -1).ADD(5, 3, 4).STG(0, 0, 5).EXIT()
    cases.append(("arith-imm", P._single(a.assemble(), (1, 1, 1), (8, 1, 1), 0, [0] * 8)))
    a = ir.Asm(); a.SREG(0, "TID").ADDI(1, 0, -2).LDS(2, 1, 0).STS(1, 5, 0).LDG(3, 0, 10).STG(0, 12, 3).EXIT()
    cases.append(("oob", P._single(a.assemble(), (2, 1, 1), (8, 1, 1), 16, list(range(16)))))
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0).MULI(3, 3, 24)
    for i in range(24):
        a.SREG(4, i).STG(3, i, 4)
    a.EXIT()
    cases.append(("3d", P._single(a.assemble(), (3, 2, 2), (5, 3, 2), 0, [0] * (12 * 30 * 24), tuple(range(-3, 5)))))
    a = ir.Asm(); a.SREG(0, "TID").ANDI(1, 0, 7).STS(1, 0, 0).LDS(2, 1, 1).STG(0, 0, 2).EXIT()
    cases.append(("1024", P._single(a.assemble(), (2, 1, 1), (1024, 1, 1), 64, [0] * 1024)))
    a = ir.Asm(); a.SREG(0, "TID").STG(0, 0, 0)
    cases.append(("falloff", P._single(a.assemble(), (1, 1, 1), (33, 1, 1), 0, [0] * 33)))
    a = ir.Asm(); a.SREG(0, "TID").ANDI(1, 0, 1).BZ(1, "E").BAR().BAR().label("E").BAR().EXIT()
    cases.append(("wave-div", P._single(a.assemble(), (2, 1, 1), (6, 1, 1), 0, [0])))
    fuel = 5000
    ctx.set_option("fuel", fuel)
    try:
        for name, job in cases:
            say(f"jit edge {name}")
            _run(ctx, job, name, fuel=fuel)
    finally:
        ctx.set_option("fuel", O.DEFAULT_FUEL)


def test_jit_long_segments_and_replay(ctx):
    job = P._single(P._hot_word_program(), (40, 1, 1), (256, 1, 1), 4, [3, 4] + [0] * 14 + [0] * 40)
    say("jit long segments")
    _run(ctx, job, "long segments")
    for reads0 in (False, True):
        job = P._single(P._redirect_program(reads0), (2, 1, 1), (2, 1, 1), 16, [7] * 10)
        say(f"jit replay path {reads0}")
        _run(ctx, job, f"redirect {reads0}")
