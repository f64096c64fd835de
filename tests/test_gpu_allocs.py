"""GPU parity of the memory-object check: jobs that list their device
allocations get an ALLOC finding per block and word accessed outside them,
computed on the device from the stage's canonical logs (free run less the
replayed blocks, plus the replay's records).  Reports and final memory must
equal the CPU oracle's bit for bit on the oracle's hand case, random small
jobs, and launches of thousands of threads (more findings than the first
result buffer takes; intra-launch races, so that replays feed the scan), in
the default, sort-only and program-specialised modes, alone and together with
streams."""
import random

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import test_oracle_allocs as A
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


def _n_alloc(res):
    return sum(1 for f in res.faults if f["kind"] == A.ALLOC)


def test_small_alloc_jobs_batched(ctx):
    rng = random.Random(3)
    hand = W.Job([A._spec(A._store_load(), 2, 4)], np.arange(32, dtype=np.int32), allocs=[(0, 8), (16, 8)])
    empty = W.Job(hand.launches, hand.memory, allocs=[])
    jobs = [hand, empty] + [A._random_job(rng) for _ in range(80)]
    say(f"alloc jobs: {len(jobs)} batched")
    reps, mems = kc.run_jobs(ctx, jobs)
    total = 0
    for i, (j, r, m) in enumerate(zip(jobs, reps, mems)):
        orc = O.run_job(j)
        total += _n_alloc(orc)
        assert_same(r, m, orc, f"alloc job {i}")
    assert total > 0


def _large_jobs():
    t = W.tree256_job(n_blocks=64, drop_frac=0.1, div_frac=0.0, seed=21)
    n = 64 * 256
    t.allocs = [(0, 12000), (n, len(t.memory) - n)]         # inputs from 12000 on are not allocated
    p = W.stencil_pingpong_job(n=1 << 13, threads=256, steps=2, bug_frac=0.1, seed=22)
    p.allocs = [(0, 1 << 13), (2 << 13, len(p.memory) - (2 << 13))]     # array B is not allocated
    s = W.stencil_pingpong_job(n=1 << 13, threads=256, steps=3, bug_frac=0.1, seed=23)
    s.allocs = [(0, len(s.memory) - 8)]
    s.streams = [0, 1, 0]
    return [t, p, s]


@pytest.mark.parametrize("mode", ["default", "sort", "jit"])
def test_large_alloc_jobs(ctx, mode):
    opts = {"default": {}, "sort": {"local": 0}, "jit": {"jit": 1}}[mode]
    for k, v in opts.items():
        ctx.set_option(k, v)
    try:
        jobs = _large_jobs()
        for i, job in enumerate(jobs):
            say(f"{mode}: large alloc job {i} ({len(job.launches)} launches, {len(job.memory)} words)")
            rep, mem = kc.run_job(ctx, job)
            orc = O.run_job(job)
            assert_same(rep, mem, orc, f"{mode} large alloc job {i}")
            if i < 2:
                assert _n_alloc(orc) > 4096
        say(f"{mode}: large alloc jobs batched")
        reps, mems = kc.run_jobs(ctx, jobs)
        for i, (j, r, m) in enumerate(zip(jobs, reps, mems)):
            assert_same(r, m, O.run_job(j), f"{mode} batched large alloc job {i}")
    finally:
        ctx.set_option("local", 1)
        ctx.set_option("jit", 0)


def test_allocation_outside_memory_rejected(ctx):
    job = W.Job([A._spec(A._store_load(), 2, 4)], np.arange(32, dtype=np.int32), allocs=[(30, 3)])
    with pytest.raises(kc.KcError):
        kc.run_job(ctx, job)
