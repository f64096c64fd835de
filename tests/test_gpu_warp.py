"""GPU parity of the warp-aware model (option warp): reports and final memory
equal the oracle's in that model, through the interpreter and the
program-specialised kernels, on the oracle pins' hand-written kernels,
random tiny kernels (interpreter), the mixed workload-3 families with every
fault, racy tree reductions, and a tree reduction whose last five levels are
warp-synchronous (race-free in this model, racy in the plain one) in 512
blocks of 256 threads."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import test_oracle_brute as TB
import test_oracle_warp as TW
from gpu_util import assert_same, say
from oracle import oracle as O
from paper_1211_6193_amd import ir, kc
from paper_1211_6193_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[0, 1], ids=["interp", "jit"])
def ctx(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = kc.Context(0)
    c.set_option("warp", 1)
    c.set_option("jit", request.param)
    yield c
    c.close()


def _check(ctx, jobs, label):
    say(f"{label}: {len(jobs)} jobs")
    reps, mems = kc.run_jobs(ctx, jobs)
    for i, (j, r, m) in enumerate(zip(jobs, reps, mems)):
        assert_same(r, m, O.run_job(j, warp=True), f"{label}[{i}]")
    return reps


def test_hand_written_kernels(ctx):
    jobs = [TW._job(TW.warp_sync_reduction(), block=32),
            TW._job(TW.warp_sync_reduction(start=32), block=64),
            TW._job(TW.warp_sync_reduction(first_barrier=False, start=32), block=64),
            TW._job(TW._diverged(0), block=2, sh_words=1), TW._job(TW._diverged(1), block=2, sh_words=1)]
    a = ir.Asm()
    a.SREG(0, "TID").SHRAI(1, 0, 1).STS(1, 0, 0).EXIT()
    jobs.append(TW._job(a, block=4, sh_words=2))
    a = ir.Asm()
    a.SREG(0, "TID").BNZ(0, "LD").MOVI(2, 0).MOVI(2, 0).STS(15, 0, 0).EXIT()
    a.label("LD").SEQI(1, 0, 1).BZ(1, "END").LDS(3, 15, 0)
    a.label("END").EXIT()
    jobs.append(TW._job(a, block=2, sh_words=1))
    a = ir.Asm()
    a.SREG(0, "TID").BNZ(0, "LD").STS(15, 0, 0).EXIT()
    a.label("LD").MOVI(2, 0).MOVI(2, 0).LDS(3, 15, 0).EXIT()
    jobs.append(TW._job(a, block=64, sh_words=1))
    a = ir.Asm()
    a.SREG(0, "TID").BNZ(0, "LD").STG(15, 0, 0).MOVI(4, 1).SREG(5, "BID").STG(4, 0, 5).EXIT()
    a.label("LD").MOVI(2, 0).MOVI(2, 0).LDG(3, 15, 0).EXIT()
    jobs.append(TW._job(a, grid=2, block=2, sh_words=0))
    reps = _check(ctx, jobs, "hand-written")
    assert reps[0].races.size == 0 and reps[2].races.size == 32


def test_random_tiny_kernels(ctx):
    if ctx.stat("option.jit"):
        pytest.skip("a hundred programs: the interpreter covers them (each would be compiled)")
    jobs = []
    for chunk in range(4):
        for prog, nb, nt, mem in TB._cases(25, 7100 + chunk):
            jobs.append(W.Job([W.LaunchSpec(np.array(prog, dtype=np.uint64), (nb, 1, 1), (nt, 1, 1),
                                            4 * TB.SH_WORDS, ())], np.array(mem, dtype=np.int32)))
    _check(ctx, jobs, "tiny")


def test_families_and_trees(ctx):
    rng = np.random.default_rng(41)
    jobs = [W.family_job(f, 3, t, rng, x, 1, 1) for f in W.FAMILIES for t in (64, 256, 1024)
            for x in (None,) + W.FAULTS[f]]
    jobs += W.config3_jobs(n=150, seed=321)
    jobs += [W.tree256_job(n_blocks=96, drop_frac=0.1, div_frac=0.05, seed=s) for s in (3, 4)]
    _check(ctx, jobs, "families")


def warp_sync_tree(n_blocks, threads=256):
    """Tree reduction with barriers down to s = 32 and no barrier for the last
    five levels (one warp); thread 0 stores the block's sum."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0)
    a.LDG(4, 3, 0).STS(0, 0, 4).BAR()
    a.SHRAI(5, 2, 1)
    a.label("L").BZ(5, "DONE").SLT(6, 0, 5).BZ(6, "SKIP")
    a.ADD(7, 0, 5).LDS(8, 0, 0).LDS(9, 7, 0).ADD(8, 8, 9).STS(0, 0, 8)
    a.label("SKIP").SLTI(6, 5, 33).BNZ(6, "NOBAR").BAR()
    a.label("NOBAR").SHRAI(5, 5, 1).JMP("L")
    a.label("DONE").BNZ(0, "END").LDS(8, 15, 0).SREG(10, "PARAM0").ADD(10, 10, 1).STG(10, 0, 8)
    a.label("END").EXIT()
    n = n_blocks * threads
    rng = np.random.default_rng(7)
    mem = np.zeros(n + n_blocks, np.int32)
    mem[:n] = rng.integers(0, 1 << 16, n)
    prog = np.array(a.assemble(), dtype=np.uint64)
    return W.Job([W.LaunchSpec(prog, (n_blocks, 1, 1), (threads, 1, 1), 4 * threads, (n,))], mem, {})


def test_warp_synchronous_tree_at_scale(ctx):
    job = warp_sync_tree(512)
    ctx.reset_stats()
    rep = _check(ctx, [job], "warp-synchronous tree")[0]
    assert rep.races.size == 0
    assert ctx.stat("replays") == 512          # every block races in the plain model and is replayed
    want = job.memory[:512 * 256].reshape(512, 256).astype(np.int64).sum(axis=1)
    plain = O.run_job(job)
    assert len(plain.races) > 0
    assert np.array_equal(plain.memory[512 * 256:], want.astype(np.int32))
