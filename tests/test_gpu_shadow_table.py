"""GPU parity of the epoch-local check of global accesses through the LDS
shadow table (option "shadow_global" = 1, the default) and through staging and
sorting (0).  Reports and final memory must equal the CPU oracle's bit for bit
in both modes, on:

* many distinct locations per block and epoch, beyond what the table takes
  (the epoch overflows: the table's tuples and the staged records go to the
  global check unreduced), with intra-block write-write races and cross-block
  read-write races over a barrier;
* lanes sharing locations four at a time, a writer among readers (concurrent
  merges into one slot);
* whole waves storing to one word (the one-location path with a store);
* 32- and 1024-thread blocks (the smallest and largest tables);
* the same cases on program-specialised kernels."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import assert_same, say
from oracle import oracle as O
from paper_1211_6193_amd import ir, kc
from paper_1211_6193_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = kc.Context(0)
    yield c
    c.close()


def _job(prog, nb, nt, mem_words, seed, shmem=0):
    rng = np.random.default_rng(seed)
    mem = rng.integers(0, 1 << 16, mem_words).astype(np.int32)
    return W.Job([W.LaunchSpec(np.array(prog, dtype=np.uint64), (nb, 1, 1), (nt, 1, 1), shmem, ())], mem)


def _many_locations(k):
    """Thread g reads k distinct words [k*g, k*g + k), stores their sum to
    out[g] and to pair[g/2] (two threads per word: a write-write race), then
    after a barrier reads out[g+1] (the next block's first thread for the
    last thread of a block: a cross-block read-write race)."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0)      # r3 = g
    a.MULI(4, 3, k).MOVI(6, 0)
    for i in range(k):
        a.LDG(5, 4, i).ADD(6, 6, 5)
    return a


def _many_program(k, n_total):
    a = _many_locations(k)
    out, pair, out3 = k * n_total, k * n_total + n_total + 1, k * n_total + n_total + 1 + n_total // 2 + 1
    a.STG(3, out, 6).SHRAI(8, 3, 1).STG(8, pair, 6).BAR()
    a.LDG(10, 3, out + 1).STG(3, out3, 10).EXIT()
    return a.assemble(), out3 + n_total + 1


def _group_program(n_total):
    """Groups of four consecutive threads read one word; the group's first
    thread then overwrites it (read-write races inside the group); after a
    barrier every thread stores what it read."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0)
    a.SHRAI(4, 3, 2).LDG(5, 4, 0).ANDI(6, 0, 3).BNZ(6, "S").STG(4, 0, 0)
    a.label("S").BAR().STG(3, n_total, 5).EXIT()
    return a.assemble(), 2 * n_total


def _broadcast_store_program(n_blocks):
    """Every thread of block b stores its tid to word b (a write-write race
    among all of them) and reads word n_blocks (one location for the whole
    grid); after a barrier thread 0 stores the value it read."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").STG(1, 0, 0).MOVI(2, n_blocks).LDG(3, 2, 0).BAR()
    a.BNZ(0, "E").STG(1, n_blocks + 1, 3)
    a.label("E").EXIT()
    return a.assemble(), 2 * n_blocks + 2


def _cases():
    cases = []
    for nb, nt, k in ((6, 256, 8), (3, 1024, 3), (9, 32, 20)):
        prog, words = _many_program(k, nb * nt)
        cases.append((f"many k={k} {nb}x{nt}", _job(prog, nb, nt, words, 11 + k)))
    for nb, nt in ((5, 256), (2, 1024), (7, 32)):
        prog, words = _group_program(nb * nt)
        cases.append((f"groups {nb}x{nt}", _job(prog, nb, nt, words, 5)))
        prog, words = _broadcast_store_program(nb)
        cases.append((f"broadcast store {nb}x{nt}", _job(prog, nb, nt, words, 6)))
    return cases


@pytest.mark.parametrize("shadow_global", [1, 0])
def test_shadow_table_cases(ctx, shadow_global):
    ctx.set_option("shadow_global", shadow_global)
    try:
        for name, job in _cases():
            say(f"shadow_global={shadow_global} {name}")
            rep, mem = kc.run_job(ctx, job)
            orc = O.run_job(job)
            assert len(orc.races) > 0, name
            assert_same(rep, mem, orc, f"{name} shadow_global={shadow_global}")
    finally:
        ctx.set_option("shadow_global", 1)


def test_shadow_table_batched_and_specialised(ctx):
    jobs = [job for _, job in _cases()]
    say(f"shadow table cases batched: {len(jobs)} jobs")
    reps, mems = kc.run_jobs(ctx, jobs)
    for i, (j, r, m) in enumerate(zip(jobs, reps, mems)):
        assert_same(r, m, O.run_job(j), f"batched {i}")
    ctx.set_option("jit", 1)
    try:
        for name, job in _cases()[:4]:
            say(f"specialised {name}")
            ctx.reset_stats()
            rep, mem = kc.run_job(ctx, job)
            assert_same(rep, mem, O.run_job(job), f"specialised {name}")
            assert ctx.stat("jit_launches") >= 1
    finally:
        ctx.set_option("jit", 0)
