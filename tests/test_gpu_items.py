"""GPU parity of memory transfers and host synchronisation: jobs given as host
programs (launches and copies in streams, host reads and writes, host waits,
events).  Copies and host writes run as device kernels on the job's memory,
their access summaries are written from their word ranges, and races between
steps that may run in parallel come from the same scan as between launches.
Reports and final memory must equal the CPU oracle's bit for bit:

* Figure 1's host program with every synchronous / asynchronous variant;
* the oracle pins' hand-written jobs and random small host programs, batched;
* the two-stream reduction as a host program at 512 and 4096 blocks of 256
  threads, with each synchronisation left out in turn (one of them races on
  every word of a 2^20-word buffer), through the interpreter and the
  program-specialised kernels;
* malformed items are refused before anything runs."""
import random

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import test_oracle_items as T
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


def _check(ctx, jobs, label):
    say(f"{label}: {len(jobs)} jobs batched")
    reps, mems = kc.run_jobs(ctx, jobs)
    for i, (j, r, m) in enumerate(zip(jobs, reps, mems)):
        assert_same(r, m, O.run_job(j), f"{label}[{i}]")
    return reps


def _hand_jobs():
    jobs = [T.fig1_items_job(s, y, w) for s in (0, 1) for y in (False, True) for w in (False, True)]
    jobs.append(T.fig1_items_job(variant="NOBAR14"))
    mem = np.arange(16, dtype=np.int32)
    jobs.append(W.Job([], mem, items=[W.host_write(8, 4, 7), W.copy_item(0, 8, 4, stream=2), W.host_wait(1),
                                      W.host_write(10, 4, 9), W.host_read(0, 4)]))
    c, hw = W.copy_item(0, 8, 4, stream=1), W.host_write(10, 2, 5)
    jobs += [W.Job([], mem, items=[c, hw]), W.Job([], mem, items=[c, W.host_wait(0), hw]),
             W.Job([], mem, items=[c, W.host_wait(), hw])]
    items = [W.launch_item(0, stream=0), W.copy_item(8, 2, 4, stream=1)]
    jobs += [W.Job([T._writer(100, 4)], np.zeros(16, np.int32), items=items, deps=d) for d in ([], [(0, 1)])]
    jobs.append(W.Job([], np.arange(8, dtype=np.int32),
                      items=[W.copy_item(0, 4, 1, stream=0), W.copy_item(0, 5, 1, stream=1), W.host_wait(0),
                             W.host_read(0, 1)]))
    a = T.ir.Asm()
    a.SREG(0, "TID").BNZ(0, "E").BAR()
    a.label("E").EXIT()
    dead = W.LaunchSpec(np.array(a.assemble(), dtype=np.uint64), (1, 1, 1), (2, 1, 1), 0, ())
    jobs.append(W.Job([dead], np.zeros(4, np.int32),
                      items=[W.host_write(0, 1, 3), W.launch_item(0), W.copy_item(1, 0, 1)]))
    return jobs


def test_hand_written_host_programs(ctx):
    reps = _check(ctx, _hand_jobs(), "hand-written")
    assert int(reps[0].launches_completed) == 5


def test_random_small_host_programs(ctx):
    rng = random.Random(99)
    jobs = [T._random_item_job(rng) for _ in range(120)]
    reps = _check(ctx, jobs, "random")
    assert sum(1 for r in reps if any(t[2] == 2 for t in r.race_tuples())) >= 20


@pytest.mark.parametrize("jit", [0, 1], ids=["interp", "jit"])
def test_two_stream_reduction_host_program(ctx, jit):
    ctx.set_option("jit", jit)
    try:
        jobs = [W.host_program_job(512, bug) for bug in W.HOST_PROGRAM_BUGS]
        ctx.reset_stats()
        reps = _check(ctx, jobs, "host program 512")
        assert ctx.stat("item_steps") > 0
        assert [sum(1 for t in r.race_tuples() if t[2] == 2) for r in reps] == [0, 512, 131076, 131072]
        for bug in (None, "reuse"):
            job = W.host_program_job(4096, bug)
            say(f"host program 4096 blocks, bug {bug}")
            rep, mem = kc.run_job(ctx, job)
            assert_same(rep, mem, O.run_job(job), f"host program 4096 {bug}")
    finally:
        ctx.set_option("jit", 0)


@pytest.mark.parametrize("items,deps", [
    ([W.copy_item(0, 2, 4)], []),
    ([W.copy_item(14, 0, 4)], []),
    ([W.host_read(15, 2)], []),
    ([W.copy_item(0, 8, 1), W.host_write(1, 1, 0)], [(0, 1)]),
    ([W.copy_item(0, 8, 1), W.host_wait(1)], []),
    ([W.host_write(0, 1, 0), W.host_wait(0)], []),
    ([W.launch_item(1)], []),
])
def test_malformed_items_refused(ctx, items, deps):
    job = W.Job([T._writer(1, 2)], np.zeros(16, np.int32), items=items, deps=deps)
    with pytest.raises(ValueError):
        O.run_job(job)
    mem = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(kc.KcError) as e:
        kc.run_job(ctx, job, mem)
    assert e.value.status == kc.KC_E_INVAL
    assert int(mem.abs().sum()) == 0


def test_streams_with_items_refused(ctx):
    job = W.Job([T._writer(1, 2)], np.zeros(16, np.int32), streams=[0], items=[W.launch_item(0)])
    mem = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(kc.KcError):
        kc.run_job(ctx, job, mem)
