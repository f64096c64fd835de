"""GPU parity of streams and events: jobs whose launches name streams and
event dependencies, so that some launches may run in parallel; races between
such launches (scope 2) come from per-launch access summaries built on the
device from the logs each stage leaves (free run, less the replayed blocks,
plus the replay's records).  Reports and final memory must equal the CPU
oracle's bit for bit:

* the oracle's hand-derived cases and random small jobs, batched;
* launches of thousands of threads in different streams (stencil ping-pong
  steps, tree reductions) with intra-launch races, so that replays feed the
  summaries, with more cross-launch races than the first result buffer takes;
* the same with the sort path, with program-specialised kernels, and with
  dependencies that order every launch (no cross-launch races)."""
import random

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
    yield c
    c.close()


def _hand_jobs():
    w = S._spec(S._writer(1), 1, 2)
    d = S.ir.Asm()
    d.SREG(0, "TID").STG(0, 0, 0).BZ(0, "E").BAR().label("E").EXIT()
    return [
        S._job([S._spec(S._writer(100), 1, 4), S._spec(S._reader_of(3), 2, 1)], streams=[0, 1]),
        S._job([S._spec(S._writer(100), 1, 4), S._spec(S._reader_of(3), 2, 1)], streams=[0, 1], deps=[(0, 1)]),
        S._job([S._spec(S._writer(10), 1, 2), S._spec(S._writer(20), 1, 3), S._spec(S._reader_of(3), 1, 2)],
               streams=[0, 1, 2]),
        S._job([w, w, w], streams=[0, 1, 0], deps=[(0, 1)]),
        S._job([w, w, w], streams=[0, 1, 2], deps=[(0, 1), (1, 2)]),
        S._job([S._spec(S._writer(1), 1, 2), S._spec(d, 1, 2), S._spec(S._writer(2), 1, 2)], streams=[0, 1, 2]),
    ]


def test_small_stream_jobs_batched(ctx):
    rng = random.Random(7)
    jobs = _hand_jobs() + [S._random_job(rng) for _ in range(60)] + [S._disjoint_job(rng) for _ in range(30)]
    say(f"stream jobs: {len(jobs)} batched")
    ctx.reset_stats()
    reps, mems = kc.run_jobs(ctx, jobs)
    n_cross = 0
    for i, (j, r, m) in enumerate(zip(jobs, reps, mems)):
        orc = O.run_job(j)
        n_cross += sum(1 for x in orc.races if x["scope"] == 2)
        assert_same(r, m, orc, f"stream job {i}")
    assert n_cross > 0 and ctx.stat("cross_launch_races") == n_cross
    say("stream jobs one by one")
    for i, j in enumerate(jobs[:12]):
        r, m = kc.run_job(ctx, j)
        assert_same(r, m, O.run_job(j), f"single stream job {i}")


def _pingpong(seed, bug_frac, steps=3):
    job = W.stencil_pingpong_job(n=1 << 13, threads=256, steps=steps, bug_frac=bug_frac, seed=seed)
    job.streams = [k % 2 for k in range(steps)]        # neighbouring steps may overlap
    return job


def _trees(seed):
    t = W.tree256_job(n_blocks=64, drop_frac=0.1, div_frac=0.0, seed=seed)
    # the same reduction three times: L0 and L1 in parallel, L2 after both
    t.launches = t.launches * 3
    t.streams = [0, 1, 0]
    t.deps = [(1, 2)]
    return t


def _large_jobs():
    jobs = [_pingpong(4, 0.1), _trees(11)]
    pp = _pingpong(5, 0.0)
    n, nb = pp.meta["n"], pp.meta["n_blocks"]
    for b in (1, 6, nb - 1):            # cross-block components: the sorted replay path
        pp.memory[2 * n + b] = 1
    jobs.append(pp)
    ordered = _pingpong(6, 0.1)
    ordered.deps = [(0, 1), (1, 2)]     # events order every launch: no cross-launch races
    jobs.append(ordered)
    return jobs


@pytest.mark.parametrize("mode", ["default", "sort", "jit"])
def test_large_stream_jobs(ctx, mode):
    opts = {"default": {}, "sort": {"local": 0}, "jit": {"jit": 1}}[mode]
    for k, v in opts.items():
        ctx.set_option(k, v)
    try:
        jobs = _large_jobs()
        for i, job in enumerate(jobs):
            say(f"{mode}: large stream job {i} ({len(job.launches)} launches, {len(job.memory)} words)")
            ctx.reset_stats()
            rep, mem = kc.run_job(ctx, job)
            orc = O.run_job(job)
            assert_same(rep, mem, orc, f"{mode} large stream job {i}")
            n_cross = sum(1 for x in orc.races if x["scope"] == 2)
            if i < 3:
                assert n_cross > 0
            else:
                assert n_cross == 0
        say(f"{mode}: large stream jobs batched")
        reps, mems = kc.run_jobs(ctx, jobs)
        for i, (j, r, m) in enumerate(zip(jobs, reps, mems)):
            assert_same(r, m, O.run_job(j), f"{mode} batched large stream job {i}")
    finally:
        ctx.set_option("local", 1)
        ctx.set_option("jit", 0)


def test_pingpong_has_many_cross_launch_races(ctx):
    # more tuples than the first result buffer of a stage takes (4096)
    job = _pingpong(8, 0.0)
    orc = O.run_job(job)
    assert sum(1 for x in orc.races if x["scope"] == 2) > 4096
    rep, mem = kc.run_job(ctx, job)
    assert_same(rep, mem, orc, "many cross-launch races")


def test_invalid_dependencies_rejected(ctx):
    job = S._job([S._spec(S._writer(1), 1, 2)] * 2, streams=[0, 1], deps=[(1, 0)])
    with pytest.raises(kc.KcError):
        kc.run_job(ctx, job)
