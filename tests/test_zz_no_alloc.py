"""kc_launch_noalloc (the launch for callers that cannot allocate device
memory) against kc_launch: the same report, element by element, and the same
final memory, on two calls in a row through the C ABI -- the second with a
smaller input, so it runs in a static scratch area that still holds the first
call's contents.  The inputs carry races, divergence and a deadlock-free
dropped barrier (tree reductions with injected faults) and the racy Figure 1
variant.  A memory the area cannot hold is rejected before any kernel runs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import say
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


def _both(ctx, job):
    """The job's single launch through kc_launch and kc_launch_noalloc, each
    from the job's initial memory."""
    L = job.launches[0]
    prog = ctx.program(L.program)
    m_ref = torch.from_numpy(np.ascontiguousarray(job.memory)).cuda()
    m_new = m_ref.clone()
    ref = kc.launch(ctx, prog, L.grid, L.block, L.shmem_bytes, m_ref, L.params)
    got = kc.launch_noalloc(ctx, prog, L.grid, L.block, L.shmem_bytes, m_new, L.params)
    return ref, m_ref, got, m_new


def _assert_same(ref, m_ref, got, m_new, what):
    assert got.records == ref.records, (what, got.records, ref.records)
    assert got.launches_completed == ref.launches_completed, what
    assert got.race_tuples() == ref.race_tuples(), (what, got.race_tuples()[:6], ref.race_tuples()[:6])
    assert got.fault_tuples() == ref.fault_tuples(), (what, got.fault_tuples()[:6], ref.fault_tuples()[:6])
    assert torch.equal(m_new, m_ref), what


def test_noalloc_matches_launch_twice_second_smaller(ctx):
    ctx.reset_stats()
    # first call: the workload-2 tree at full size (4096 x 256, 1% dropped
    # barriers, 0.1% tid-dependent barriers)
    big = W.tree256_job()
    say("noalloc: workload-2 tree 4096x256")
    ref, m_ref, got, m_new = _both(ctx, big)
    assert ref.races.size > 0 and ref.faults.size > 0
    _assert_same(ref, m_ref, got, m_new, "tree 4096x256")
    peak = ctx.stat("noalloc_scratch_peak")
    assert 0 < peak <= 64 << 20
    # second call, smaller: 96 blocks with a higher fault rate
    small = W.tree256_job(n_blocks=96, drop_frac=0.1, div_frac=0.05, seed=4242)
    say("noalloc: tree 96x256")
    ref, m_ref, got, m_new = _both(ctx, small)
    assert ref.races.size > 0
    _assert_same(ref, m_ref, got, m_new, "tree 96x256")
    # third, smaller still: Figure 1's racy variant, launch 0 (2 blocks x 9 threads)
    fig = W.fig1_job("NOBAR14")
    fig.launches = fig.launches[:1]
    say("noalloc: Figure 1 NOBAR14")
    ref, m_ref, got, m_new = _both(ctx, fig)
    assert ref.races.size == 6
    _assert_same(ref, m_ref, got, m_new, "fig1 NOBAR14")
    assert ctx.stat("noalloc_calls") == 3


def test_noalloc_rejects_memory_beyond_the_area(ctx):
    fig = W.fig1_job("BASE")
    L = fig.launches[0]
    mem = torch.zeros((64 << 20) // 4 + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(kc.KcError) as e:
        kc.launch_noalloc(ctx, ctx.program(L.program), L.grid, L.block, L.shmem_bytes, mem, L.params)
    assert e.value.status == kc.KC_E_BUDGET
    # the context is still usable afterwards
    fig.launches = fig.launches[:1]
    ref, m_ref, got, m_new = _both(ctx, fig)
    _assert_same(ref, m_ref, got, m_new, "fig1 after a rejected call")
