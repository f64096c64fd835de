"""GPU parity of race source sites (option "sites"): after a stage, the racy
blocks are replayed once more with a table of the stage's race tuples, and
each tuple gets the smallest pc of its writer's stores to the location and of
its other thread's accesses to it.  Sites, reports and final memory must
equal the CPU oracle's on: the paper's Figure 1 variants (the racy one is
reported at line 17), seeded workload-3 instances with every injected fault,
tree reductions with dropped barriers, in-place ping-pong stencils
(cross-block tuples) and a job with races between launches (no sites for
those), with the interpreter and with program-specialised replays."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import test_oracle_streams as S
from gpu_util import assert_same, say
from oracle import oracle as O
from paper_1211_6193_amd import kc
from paper_1211_6193_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = kc.Context(0)
    c.set_option("sites", 1)
    yield c
    c.close()


def _jobs():
    jobs = [W.fig1_job(v) for v in W.SUM_VARIANTS]
    rng = np.random.default_rng(31)
    for fam, faults in W.FAULTS.items():
        for f in faults:
            for threads in (32, 96, 256):
                jobs.append(W.family_job(fam, 3, threads, rng, f, 1, 1))
    jobs.append(W.tree256_job(n_blocks=64, drop_frac=0.1, div_frac=0.0, seed=41))
    pp = W.stencil_pingpong_job(n=1 << 12, threads=256, steps=2, bug_frac=0.0, seed=42)
    for b in (1, 6, pp.meta["n_blocks"] - 1):
        pp.memory[2 * pp.meta["n"] + b] = 1
    jobs.append(pp)
    jobs.append(S._job([S._spec(S._writer(100), 1, 4), S._spec(S._reader_of(3), 2, 1)], streams=[0, 1]))
    return jobs


def _check(rep, mem, orc, what):
    assert_same(rep, mem, orc, what)
    assert rep.race_sites() == orc.race_sites(), (what, rep.race_sites()[:6], orc.race_sites()[:6])


@pytest.mark.parametrize("jit", [0, 1])
def test_sites_match_oracle(ctx, jit):
    ctx.set_option("jit", jit)
    try:
        jobs = _jobs()
        n_sites = 0
        for i, job in enumerate(jobs):
            say(f"jit={jit} sites job {i}: {job.meta.get('family', 'streams')}")
            rep, mem = kc.run_job(ctx, job)
            orc = O.run_job(job)
            _check(rep, mem, orc, f"sites job {i}")
            n_sites += sum(1 for w, o in orc.race_sites() if w != 0xFFFFFFFF)
        assert n_sites > 100
        say(f"jit={jit} sites jobs batched")
        reps, mems = kc.run_jobs(ctx, jobs)
        for i, (j, r, m) in enumerate(zip(jobs, reps, mems)):
            _check(r, m, O.run_job(j), f"batched sites job {i}")
    finally:
        ctx.set_option("jit", 0)


def test_sites_off_by_default(ctx):
    c = kc.Context(0)
    try:
        rep, _ = kc.run_job(c, W.fig1_job("NOBAR14"))
        assert len(rep.races) == 6 and rep.race_sites() == [(0xFFFFFFFF, 0xFFFFFFFF)] * 6
    finally:
        c.close()
