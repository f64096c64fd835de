"""Oracle pins of the barriers with a predicate (the paper's Section 3 feature
list: __syncthreads_count, __syncthreads_and, __syncthreads_or), against
closed forms: every thread stores what its barrier returned, and the stored
values are checked against the count, all and any of the predicates computed
here in plain Python.  Also: a thread at a plain barrier in the same episode
counts as predicate 0 (and the differing sites are a DIVERGENCE finding), a
deadlocked episode returns nothing, and blocks are independent."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1211_6193_amd import ir
from paper_1211_6193_amd import workloads as W


def _job(prog, nb, nt, words):
    return W.Job([W.LaunchSpec(np.array(prog, dtype=np.uint64), (nb, 1, 1), (nt, 1, 1), 0, ())],
                 np.zeros(words, np.int32))


def _pred_program(mod, kinds=("COUNT", "AND", "OR")):
    """pred = (tid % mod == bid % mod); thread g stores the result of each
    kind at out[3 g + k]."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0).MULI(3, 3, 3)
    a.MOVI(4, mod).REM(5, 0, 4).REM(6, 1, 4).SEQ(7, 5, 6)
    for k, kind in enumerate(kinds):
        a.BARP(8 + k, 7, kind).STG(3, k, 8 + k)
    a.EXIT()
    return a.assemble()


@pytest.mark.parametrize("nb,nt,mod", [(1, 1, 1), (1, 7, 3), (3, 64, 5), (2, 130, 1), (4, 33, 40)])
def test_count_and_or_closed_form(nb, nt, mod):
    res = O.run_job(_job(_pred_program(mod), nb, nt, 3 * nb * nt))
    assert len(res.faults) == 0 and len(res.races) == 0
    out = res.memory.reshape(nb, nt, 3)
    for b in range(nb):
        preds = [(t % mod) == (b % mod) for t in range(nt)]
        assert (out[b, :, 0] == sum(preds)).all()
        assert (out[b, :, 1] == int(all(preds))).all()
        assert (out[b, :, 2] == int(any(preds))).all()
    assert res.records == 3 * nb * nt


def test_plain_barrier_counts_as_zero_and_diverges():
    """Thread 0 waits at a plain barrier, the rest at BARP with predicate 1:
    the count is nt - 1, AND is 0, OR is 1; the sites differ (DIVERGENCE)."""
    nt = 10
    for kind, want in (("COUNT", nt - 1), ("AND", 0), ("OR", 1)):
        a = ir.Asm()
        a.SREG(0, "TID").MOVI(1, 1).BNZ(0, "P").BAR().JMP("E")
        a.label("P").BARP(2, 1, kind).STG(0, 0, 2)
        a.label("E").EXIT()
        prog = a.assemble()
        res = O.run_job(_job(prog, 1, nt, nt))
        assert res.memory[0] == 0 and (res.memory[1:] == want).all(), kind
        div = [f for f in res.faults if int(f["kind"]) == O.F_DIVERGENCE]
        bar_pc, barp_pc = ir.pcs_of(prog, "BAR")[0], ir.pcs_of(prog, "BARP")[0]
        assert len(div) == 1 and int(div[0]["a"]) == min(bar_pc, barp_pc)


def test_deadlocked_predicate_barrier_returns_nothing():
    a = ir.Asm()
    a.SREG(0, "TID").MOVI(1, 5).MOVI(2, 77).BZ(0, "E").BARP(2, 1, "COUNT").label("E").STG(0, 0, 2).EXIT()
    res = O.run_job(_job(a.assemble(), 1, 4, 4))
    dead = [f for f in res.faults if int(f["kind"]) == O.F_DEADLOCK]
    assert len(dead) == 1 and res.launches_completed == 0
    assert res.memory[0] == 77 and (res.memory[1:] == 0).all()     # only thread 0 stored, r2 untouched


def test_successive_predicate_barriers_and_epochs():
    """A count feeds the next predicate: epochs advance per episode and the
    stored results follow the closed form."""
    nt = 12
    a = ir.Asm()
    a.SREG(0, "TID").SLTI(1, 0, 5).BARP(2, 1, "COUNT")        # 5
    a.SLT(3, 0, 2).BARP(4, 3, "COUNT")                          # tid < 5 -> 5
    a.SEQ(5, 4, 2).BARP(6, 5, "AND").STG(0, 0, 6).EXIT()        # all equal -> 1
    res = O.run_job(_job(a.assemble(), 1, nt, nt))
    assert (res.memory == 1).all() and len(res.faults) == 0
