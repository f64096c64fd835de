"""The replay queued behind the free run (option queue_replay) against the
host-driven replay and the oracle:

* reports and final memories equal the oracle's with the option on and off,
  through the interpreter and the program-specialised kernels, on racy tree
  reductions (dropped and tid-dependent barriers), Figure 1's variants and
  the mixed families with every fault, each job run alone;
* a launch with both an intra-block race and a location written by two
  blocks: the queued replay ran but cannot stand (the log needs its sorted
  check), so the stage runs again without it -- same results;
* every block racy (far more race tuples than the first race lists hold):
  the stage runs again, the capacities grow, and a second launch of the same
  shape keeps the queued replay."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

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
    c.set_option("jit", request.param)
    yield c
    c.close()


def _alone(ctx, job, label):
    rep, mem = kc.run_job(ctx, job)
    assert_same(rep, mem, O.run_job(job), label)
    return rep


def _jobs():
    rng = np.random.default_rng(77)
    jobs = [W.tree256_job(n_blocks=n, drop_frac=0.05, div_frac=0.02, seed=s) for n, s in ((64, 1), (512, 2))]
    jobs += [W.fig1_job(v) for v in W.SUM_VARIANTS]
    jobs += [W.family_job(f, 4, t, rng, x, 1, 1) for f in W.FAMILIES for t in (64, 256)
             for x in (None,) + W.FAULTS[f]]
    return jobs


@pytest.mark.parametrize("queued", [1, 0], ids=["queued", "host-driven"])
def test_same_results_queued_or_not(ctx, queued):
    ctx.set_option("queue_replay", queued)
    try:
        ctx.reset_stats()
        jobs = _jobs()
        say(f"{len(jobs)} jobs alone, queue_replay={queued}")
        for i, j in enumerate(jobs):
            _alone(ctx, j, f"job {i}")
        if queued:
            assert ctx.stat("spec_replays") > 0
        else:
            assert ctx.stat("spec_replays") == 0
    finally:
        ctx.set_option("queue_replay", 1)


def _local_and_cross_block_race(n_blocks=8, threads=64):
    """Each thread stores sh[t] and, with no barrier, loads sh[t+1] (an
    intra-block race); thread 0 of every block also stores the first word
    of the next block's output (written by that block too: a cross-block
    race)."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0)
    a.STS(0, 0, 3).ADDI(4, 0, 1).LDS(5, 4, 0).STG(3, 0, 5)
    a.BNZ(0, "E").ADD(6, 3, 2).MOVI(7, 9).STG(6, 0, 7)
    a.label("E").EXIT()
    n = n_blocks * threads
    prog = np.array(a.assemble(), dtype=np.uint64)
    return W.Job([W.LaunchSpec(prog, (n_blocks, 1, 1), (threads, 1, 1), 4 * (threads + 1), ())],
                 np.zeros(n + threads, np.int32), {})


def test_queued_replay_that_cannot_stand_runs_the_stage_again(ctx):
    job = _local_and_cross_block_race()
    ctx.reset_stats()
    rep = _alone(ctx, job, "local + cross-block")
    assert any(t[2] == 0 for t in rep.race_tuples()) and any(t[2] == 1 for t in rep.race_tuples())
    assert ctx.stat("spec_retries") == 1 and ctx.stat("spec_replays") == 0


def test_race_list_overflow_then_capacity_learned():
    with kc.Context(0) as c:
        job = W.tree256_job(n_blocks=1024, drop_frac=1.0, div_frac=0.0, seed=9)
        c.reset_stats()
        say("every block racy: first launch")
        rep = _alone(c, job, "all racy (first)")
        assert len(rep.races) > 4096
        assert c.stat("spec_retries") + c.stat("retries") >= 1     # a list overflowed: run again
        c.reset_stats()
        say("every block racy: second launch")
        _alone(c, job, "all racy (second)")
        assert c.stat("spec_retries") == 0 and c.stat("retries") == 0 and c.stat("spec_replays") == 1
