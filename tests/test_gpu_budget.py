"""The library's HBM accounting and the tunable work layout.

* kc_batch_footprint: the part every batch reserves, growth with the jobs, the
  additive bound the serving admission relies on, and the same argument checks
  as kc_batch_submit;
* the context's device bytes ("device_bytes", "device_bytes_peak") follow its
  buffers, a budget below what a run needs is KC_E_BUDGET, and concurrent
  batches stay within the budget together;
* every radix digit width (option sort_bits) and every split of a batch
  step's launches over side streams (option side_streams) leaves reports and
  memories equal to the oracle's, with the sort's multi-pass path taken."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import assert_same, check_jobs, say
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


def test_footprint_bounds_and_checks(ctx):
    jobs = W.config3_jobs(n=40, seed=5) + [W.tree256_job(n_blocks=256)]
    fixed = kc.jobs_footprint(ctx, [])
    assert fixed > 0
    alone = [kc.jobs_footprint(ctx, [j]) for j in jobs]
    assert all(a > fixed for a in alone)
    both = kc.jobs_footprint(ctx, jobs)
    assert max(alone) <= both <= fixed + sum(a - fixed for a in alone)
    # items and streams add the summaries they hold
    hp = W.host_program_job(256)
    assert kc.jobs_footprint(ctx, [hp]) > kc.jobs_footprint(ctx, [W.Job(hp.launches, hp.memory)])
    bad = W.Job(hp.launches, hp.memory, items=[W.copy_item(0, 2, 4)])
    with pytest.raises(kc.KcError) as e:
        kc.jobs_footprint(ctx, [bad])
    assert e.value.status == kc.KC_E_INVAL


def test_device_bytes_follow_the_buffers_and_the_budget_is_enforced():
    jobs = W.config3_jobs(n=60, seed=6)
    with kc.Context(0) as c:
        assert c.stat("device_bytes") == 0
        need = kc.jobs_footprint(c, jobs)
        check_jobs(c, jobs, label="unbounded")
        live, peak = c.stat("device_bytes"), c.stat("device_bytes_peak")
        say(f"footprint {need} B, live {live:.0f} B, peak {peak:.0f} B")
        assert 0 < live <= peak
    with kc.Context(0, hbm_budget_bytes=1 << 20) as c:
        mems = [torch.from_numpy(np.ascontiguousarray(j.memory)).cuda() for j in jobs]
        with pytest.raises(kc.KcError) as e:
            kc.run_jobs(c, jobs, mems)
        assert e.value.status == kc.KC_E_BUDGET
    budget = 4 * need
    with kc.Context(0, hbm_budget_bytes=budget) as c:
        check_jobs(c, jobs, label="within budget")
        assert c.stat("device_bytes_peak") <= budget


def test_concurrent_batches_stay_within_the_budget():
    # two batches in flight hold a workspace each (the budget bounds their sum);
    # a larger batch afterwards may need an idle one freed
    small = W.config3_jobs(n=30, seed=7)
    big = [W.tree256_job(n_blocks=2048)]
    with kc.Context(0) as probe:
        need_small = kc.jobs_footprint(probe, small)
        need_big = kc.jobs_footprint(probe, big)
    budget = max(need_big, 2 * need_small) + need_small // 2
    with kc.Context(0, hbm_budget_bytes=budget) as c:
        b = kc.Batch(c)
        mems = [[torch.from_numpy(np.ascontiguousarray(j.memory)).cuda() for j in small] for _ in range(2)]
        tickets = [b.submit([kc.job_item(c, j, m, i) for i, (j, m) in enumerate(zip(small, ms))]) for ms in mems]
        for t, ms in zip(tickets, mems):
            reps = b.poll(t, wait=True)
            for i, (j, m) in enumerate(zip(small, ms)):
                assert_same(reps[i], m, O.run_job(j), f"concurrent[{i}]")
        check_jobs(c, big, label="big after two small")
        say(f"budget {budget} B, peak {c.stat('device_bytes_peak'):.0f} B, trims {c.stat('budget_trims'):.0f}")
        assert c.stat("device_bytes_peak") <= budget


@pytest.mark.parametrize("bits", [4, 5, 6, 7, 8])
def test_sort_digit_widths(ctx, bits):
    job = W.stencil_pingpong_job(n=1 << 18, threads=256, steps=2, bug_frac=0.004, seed=12116197)
    ctx.set_option("sort_bits", bits)
    ctx.set_option("hash_check", 0)
    try:
        ctx.reset_stats()
        say(f"sort with {bits}-bit digits")
        rep, mem = kc.run_job(ctx, job)
        assert ctx.stat("sorted_checks") == 2 and ctx.stat("sort_keys") > 16384
        assert_same(rep, mem, O.run_job(job), f"sort_bits={bits}")
    finally:
        ctx.set_option("sort_bits", 8)
        ctx.set_option("hash_check", 1)


@pytest.mark.parametrize("n_side", [1, 2, 4])
def test_side_stream_splits(ctx, n_side):
    ctx.set_option("side_streams", n_side)
    try:
        jobs = W.config3_jobs(n=80, seed=8)
        check_jobs(ctx, jobs, label=f"side_streams={n_side}")
    finally:
        ctx.set_option("side_streams", 4)
