"""GPU parity of the uninitialised shared-memory check (option "uninit"):
reports and final memory equal the oracle's with the check on, through the
interpreter and the program-specialised kernels, on the oracle pins'
hand-written kernels, random tiny kernels (interpreter), the mixed workload-3 families
with every fault (a halo read off by one, two threads writing one slot, ...
leave words unstored) and racy tree reductions (whose blocks the replay
re-executes)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import test_oracle_brute as TB
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
    c.set_option("uninit", 1)
    c.set_option("jit", request.param)
    yield c
    c.close()


def _check(ctx, jobs, label):
    say(f"{label}: {len(jobs)} jobs")
    reps, mems = kc.run_jobs(ctx, jobs)
    n_uninit = 0
    for i, (j, r, m) in enumerate(zip(jobs, reps, mems)):
        orc = O.run_job(j, uninit=True)
        assert_same(r, m, orc, f"{label}[{i}]")
        n_uninit += sum(1 for f in orc.fault_tuples() if f[1] == O.F_UNINIT)
    return n_uninit


def _job(a, grid, block, sh_words):
    return W.Job([W.LaunchSpec(np.array(a.assemble(), dtype=np.uint64), (grid, 1, 1), (block, 1, 1),
                               4 * sh_words, ())], np.zeros(4, np.int32), {})


def test_hand_written_kernels(ctx):
    jobs = []
    a = ir.Asm()
    a.SREG(0, "TID").LDS(1, 0, 1).STS(0, 0, 0).BAR().LDS(2, 0, 1).EXIT()
    jobs.append(_job(a, 2, 4, 5))
    a = ir.Asm()
    a.SREG(0, "TID").BNZ(0, "LD").STS(15, 0, 0).EXIT()
    a.label("LD").LDS(1, 15, 0).EXIT()
    jobs.append(_job(a, 1, 4, 8))              # same step: the loads come first
    a = ir.Asm()
    a.SREG(0, "TID").BNZ(0, "LD").STS(15, 0, 0).EXIT()
    a.label("LD").MOVI(2, 7).LDS(1, 15, 0).EXIT()
    jobs.append(_job(a, 1, 4, 8))              # one step later: stored
    a = ir.Asm()
    a.SREG(0, "TID").MOVI(2, 3)
    a.label("L").LDS(1, 15, 5).LDS(1, 15, 8).ADDI(2, 2, -1).BNZ(2, "L").EXIT()
    jobs.append(_job(a, 1, 2, 8))
    a = ir.Asm()
    a.SREG(0, "TID").LDS(1, 0, 64).STS(0, 0, 0).BAR().LDS(2, 0, 1).EXIT()
    jobs.append(_job(a, 3, 128, 160))          # two waves, words read across the wave boundary
    assert _check(ctx, jobs, "hand-written") > 0


def test_random_tiny_kernels(ctx):
    if ctx.stat("option.jit"):
        pytest.skip("a hundred programs: the interpreter covers them (each would be compiled)")
    jobs = []
    for chunk in range(4):
        for prog, nb, nt, mem in TB._cases(25, 7000 + chunk):
            jobs.append(W.Job([W.LaunchSpec(np.array(prog, dtype=np.uint64), (nb, 1, 1), (nt, 1, 1),
                                            4 * TB.SH_WORDS, ())], np.array(mem, dtype=np.int32)))
    assert _check(ctx, jobs, "tiny") > 0


def test_mixed_families_with_every_fault(ctx):
    rng = np.random.default_rng(31)
    jobs = [W.family_job(f, 3, t, rng, x, 1, 1) for f in W.FAMILIES for t in (64, 256, 1024)
            for x in (None,) + W.FAULTS[f]]
    jobs += W.config3_jobs(n=200, seed=123)
    assert _check(ctx, jobs, "families") > 0


def test_racy_tree_reductions(ctx):
    jobs = [W.tree256_job(n_blocks=96, drop_frac=0.1, div_frac=0.05, seed=s) for s in (1, 2)]
    _check(ctx, jobs, "trees")
