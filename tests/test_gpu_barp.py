"""GPU parity of the barriers with a predicate (count / and / or): reports and
final memory equal the oracle's bit for bit on the interpreter and on the
program-specialised kernels, for blocks of 1 to 1024 threads (partial waves
included), mixed plain and predicate barriers (DIVERGENCE), a deadlocked
predicate barrier, successive predicate barriers, and racy blocks that the
lockstep replay re-executes through predicate barriers."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import test_oracle_barp as TB
from gpu_util import assert_same, check_jobs, say
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


def _racy_barp_program():
    """Every thread stores its tid to shared word 0 (a write-write race: the
    block is replayed), then BARP COUNT over (tid odd), then thread g stores
    the count plus the shared word it reads after the barrier."""
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0)
    a.STS(15, 0, 0).ANDI(4, 0, 1).BARP(5, 4, "COUNT").LDS(6, 15, 0).ADD(5, 5, 6).STG(3, 0, 5).EXIT()
    return a.assemble()


def _cases():
    cases = []
    for nb, nt, mod in ((1, 1, 1), (1, 7, 3), (3, 64, 5), (2, 130, 1), (4, 33, 40), (2, 256, 7), (1, 1024, 2)):
        cases.append((f"pred {nb}x{nt} mod {mod}", TB._job(TB._pred_program(mod), nb, nt, 3 * nb * nt)))
    for kind in ("COUNT", "AND", "OR"):
        a = ir.Asm()
        a.SREG(0, "TID").MOVI(1, 1).BNZ(0, "P").BAR().JMP("E")
        a.label("P").BARP(2, 1, kind).STG(0, 0, 2)
        a.label("E").EXIT()
        cases.append((f"plain+pred {kind}", TB._job(a.assemble(), 1, 100, 100)))
    a = ir.Asm()
    a.SREG(0, "TID").MOVI(1, 5).MOVI(2, 77).BZ(0, "E").BARP(2, 1, "COUNT").label("E").STG(0, 0, 2).EXIT()
    cases.append(("deadlock", TB._job(a.assemble(), 2, 70, 70)))
    a = ir.Asm()
    a.SREG(0, "TID").SLTI(1, 0, 5).BARP(2, 1, "COUNT").SLT(3, 0, 2).BARP(4, 3, "COUNT")
    a.SEQ(5, 4, 2).BARP(6, 5, "AND").STG(0, 0, 6).EXIT()
    cases.append(("successive", TB._job(a.assemble(), 1, 200, 200)))
    for nb, nt in ((3, 64), (2, 256), (1, 1000)):
        cases.append((f"racy replay {nb}x{nt}", W.Job([W.LaunchSpec(np.array(_racy_barp_program(), dtype=np.uint64),
                                                                     (nb, 1, 1), (nt, 1, 1), 4, ())],
                                                       np.zeros(nb * nt, np.int32))))
    return cases


@pytest.mark.parametrize("jit", [0, 1])
def test_predicate_barriers(ctx, jit):
    ctx.set_option("jit", jit)
    try:
        for name, job in _cases():
            say(f"jit={jit} {name}")
            ctx.reset_stats()
            rep, mem = kc.run_job(ctx, job)
            orc = O.run_job(job)
            assert_same(rep, mem, orc, f"{name} jit={jit}")
            if name.startswith("racy"):
                assert len(orc.races) > 0 and ctx.stat("replays") >= 1
                if jit:
                    assert ctx.stat("jit_replays") >= 1
        check_jobs(ctx, [job for _, job in _cases()], label=f"predicate barriers batched jit={jit}")
    finally:
        ctx.set_option("jit", 0)
