"""Batched and served forms: each instance gives the same report and final
memory alone (one plain launch per instance) as inside a large batch, and as a
request inside the served mix; batched results equal the oracle's."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import assert_same, say
from oracle import oracle as O
from paper_1211_6193_amd import kc, server, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = kc.Context(0)
    yield c
    c.close()


def _same(a, b, what):
    assert a.records == b.records and a.launches_completed == b.launches_completed, what
    assert a.race_tuples() == b.race_tuples() and a.fault_tuples() == b.fault_tuples(), what


def test_batch_equals_alone_and_oracle(ctx):
    jobs = W.config3_jobs(n=1000)
    say("1000 workload-3 instances in one batch")
    reps, mems = kc.run_jobs(ctx, jobs)
    rng = np.random.default_rng(5)
    for i in rng.choice(len(jobs), 60, replace=False):
        j = jobs[int(i)]
        say(f"instance {int(i)} alone")
        L = j.launches[0]
        m = torch.from_numpy(j.memory.copy()).cuda()
        alone = kc.launch(ctx, ctx.program(L.program), L.grid, L.block, L.shmem_bytes, m, L.params)
        _same(alone, reps[int(i)], f"alone vs batch {int(i)}")
        assert torch.equal(m, mems[int(i)])
        assert_same(alone, m, O.run_job(j), f"oracle {int(i)}")


def test_sort_tile_invariance(ctx):
    jobs = W.config3_jobs(n=200, seed=77)
    base, bm = kc.run_jobs(ctx, jobs)
    for tile in (1024, 4096, 8192):
        ctx.set_option("sort_tile", tile)
        say(f"sort tile {tile}")
        reps, mems = kc.run_jobs(ctx, jobs)
        for i in range(len(jobs)):
            _same(base[i], reps[i], f"tile {tile} job {i}")
            assert torch.equal(bm[i], mems[i])
    ctx.set_option("sort_tile", 2048)


def test_served_mix_equals_alone(ctx):
    stream = list(W.request_stream(rate=2000.0, duration_s=0.25, big_p=0.05, big_blocks=64))
    say(f"serving {len(stream)} requests")
    srv = server.Server(ctx, budget_bytes=8 << 30, slots=3)
    out = srv.run(stream, keep_reports=True, keep_memory=True)
    assert out["requests"] == len(stream)
    rng = np.random.default_rng(1)
    for i in rng.choice(len(stream), min(40, len(stream)), replace=False):
        _, job = stream[int(i)]
        rep, mem = kc.run_job(ctx, job)
        _same(rep, out["reports"][int(i)], f"served {int(i)}")
        assert np.array_equal(mem.cpu().numpy(), out["memories"][int(i)])


def test_served_sample_at_bench_shapes_vs_oracle(ctx):
    """The served mix the benchmark runs (workload-3 instances and 4096 x 256
    trees drawn from a seeded pool, continuous batching under a 64 GiB budget):
    every 10th request's report and final memory equal the oracle's, the big
    trees included."""
    small, big = W.request_pool(n_small=256, n_big=3)
    reqs = W.pooled_requests(4000.0, 0.25, small, big, big_p=0.05, seed=W.BASE_SEED + 77)
    say(f"serving {len(reqs)} pooled requests")
    srv = server.Server(ctx, budget_bytes=64 << 30, slots=4)
    out = srv.run(reqs, keep_every=10)
    sample = out["sample"]
    assert len(sample) >= len(reqs) // 10
    assert any(j.meta.get("family") == "TREE256" for j, _, _ in sample), "no 4096 x 256 tree in the sample"
    for j, r, m in sample:
        assert_same(r, m, O.run_job(j), f"served {j.meta.get('family')}")


def test_local_check_modes_agree(ctx):
    """Epoch-local checking in LDS (global locations in the shadow table, or
    staged and sorted), its spill path (tiny staging areas) and the all-global
    path give identical reports and memory."""
    rng = np.random.default_rng(21)
    jobs = W.config3_jobs(n=150, seed=99) + [W.tree256_job(n_blocks=128, seed=4, drop_frac=0.05, div_frac=0.02)]
    jobs += [W.family_job(f, 5, t, rng, x, 2, 1) for f in W.FAMILIES for t in (64, 256, 1024)
             for x in (None,) + W.FAULTS[f]]
    settings = [("local", 0), ("stage_bytes", 8192), ("stage_bytes", 98304), ("local", 1),
                ("shadow_global", 0), ("stage_bytes", 8192), ("shadow_global", 1),
                ("hash_check", 0), ("hash_check", 1)]
    for key, val in settings:
        ctx.set_option(key, val)
        say(f"{key}={val}")
        reps, mems = kc.run_jobs(ctx, jobs)
        for i, (j, r, m) in enumerate(zip(jobs, reps, mems)):
            assert_same(r, m, O.run_job(j), f"{key}={val} job {i}")
