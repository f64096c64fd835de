"""Pin the oracle's int32 arithmetic against numpy's two's-complement routines.

Expected values come from numpy int32/uint32 array operations (wrapping add,
sub, mul, shifts, C-style ``fmod``) rather than from a second copy of the
oracle's formulas.
"""
import itertools

import numpy as np

from oracle import oracle as O
from paper_1211_6193_amd import ir
from paper_1211_6193_amd.workloads import Job, LaunchSpec

EDGE = [0, 1, -1, 2, -2, 3, -7, 31, 32, 33, -32, 255, 12345678, -98765, 2**31 - 1, -2**31]


def _np_ref(name, x, y):
    a = np.array([x], dtype=np.int32)
    b = np.array([y], dtype=np.int32)
    ua, ub = a.view(np.uint32), b.view(np.uint32)
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        if name == "ADD": return int((a + b)[0])
        if name == "SUB": return int((a - b)[0])
        if name == "MUL": return int((a * b)[0])
        if name in ("DIV", "REM"):
            if y == 0:
                return 0
            a64, b64 = a.astype(np.int64), b.astype(np.int64)
            r = np.fmod(a64, b64)                     # C remainder: sign of the dividend
            q = (a64 - r) // b64                      # exact, so truncating quotient
            v = (q if name == "DIV" else r).astype(np.int32)   # wraps INT_MIN/-1
            return int(v[0])
        if name == "AND": return int((a & b)[0])
        if name == "OR": return int((a | b)[0])
        if name == "XOR": return int((a ^ b)[0])
        sh = ub & np.uint32(31)
        if name == "SHL": return int(np.left_shift(ua, sh).view(np.int32)[0])
        if name == "SHRA": return int(np.right_shift(a, sh.astype(np.int32))[0])
        if name == "SHRL": return int(np.right_shift(ua, sh).view(np.int32)[0])
        if name == "MIN": return int(np.minimum(a, b)[0])
        if name == "MAX": return int(np.maximum(a, b)[0])
        if name == "SLT": return int((a < b)[0])
        if name == "SLE": return int((a <= b)[0])
        if name == "SEQ": return int((a == b)[0])
        if name == "SNE": return int((a != b)[0])
        if name == "SLTU": return int((ua < ub)[0])
    raise ValueError(name)


def _run(cases, imm_form):
    a = ir.Asm()
    for slot, (name, x, y) in enumerate(cases):
        a.MOVI(1, x)
        if imm_form:
            getattr(a, name + "I")(3, 1, y)
        else:
            a.MOVI(2, y)
            getattr(a, name)(3, 1, 2)
        a.MOVI(4, slot).STG(4, 0, 3)
    a.EXIT()
    prog = np.array(a.assemble(), dtype=np.uint64)
    job = Job([LaunchSpec(prog, (1, 1, 1), (1, 1, 1), 0, ())], np.zeros(len(cases), np.int32))
    return O.run_job(job)


def test_alu_matches_numpy_register_and_immediate_forms():
    cases = [(n, x, y) for n in ir.ALU_RR for x, y in itertools.product(EDGE, EDGE)]
    for imm_form in (False, True):
        r = _run(cases, imm_form)
        got = r.memory.tolist()
        want = [_np_ref(n, x, y) for n, x, y in cases]
        bad = [(c, g, w) for c, g, w in zip(cases, got, want) if g != w]
        assert not bad, bad[:10]


def test_division_by_zero_is_an_arith_finding():
    cases = [("DIV", 5, 0), ("REM", -5, 0), ("DIV", -2**31, -1), ("REM", -2**31, -1)]
    r = _run(cases, False)
    assert r.memory.tolist() == [0, 0, -2**31, 0]
    kinds = sorted(int(f["kind"]) for f in r.faults)
    assert kinds == [O.F_ARITH, O.F_ARITH]


def test_special_registers_3d():
    a = ir.Asm()
    names = list(ir.SREGS)
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS").MUL(3, 1, 2).ADD(3, 3, 0).MULI(3, 3, len(names))
    for i, nm in enumerate(names):
        a.SREG(4, nm).STG(3, i, 4)
    a.EXIT()
    prog = np.array(a.assemble(), dtype=np.uint64)
    grid, block = (2, 3, 2), (3, 2, 2)
    nb, nt = 12, 12
    params = tuple(range(100, 108))
    job = Job([LaunchSpec(prog, grid, block, 0, params)], np.zeros(nb * nt * len(names), np.int32))
    r = O.run_job(job)
    m = r.memory.reshape(nb * nt, len(names))
    for bid in range(nb):
        bz, rem = divmod(bid, grid[0] * grid[1])
        by, bx = divmod(rem, grid[0])
        for tid in range(nt):
            tz, rem = divmod(tid, block[0] * block[1])
            ty, tx = divmod(rem, block[0])
            want = [tx, ty, tz, bx, by, bz, *block, *grid, tid, bid, nt, 32, *params]
            assert m[bid * nt + tid].tolist() == want


def test_instruction_count_closed_form():
    # thread t runs a 3-instruction loop t times: 2 set-up instructions, 3 per
    # iteration and the final taken BZ, so 3 + 3t; the EXIT after the loop adds
    # one more.  Sum over T threads and B blocks.  With fuel f < 4 + 3t a
    # thread spends exactly f.
    a = ir.Asm()
    a.SREG(0, "TID").MOVI(1, 0).label("top").BZ(0, "end").ADDI(0, 0, -1).JMP("top").label("end").EXIT()
    prog = np.array(a.assemble(), dtype=np.uint64)
    B, T = 3, 37
    job = Job([LaunchSpec(prog, (B, 1, 1), (T, 1, 1), 0, ())], np.zeros(1, np.int32))
    r = O.run_job(job)
    assert r.instructions == B * sum(4 + 3 * t for t in range(T))
    fuel = 50
    r = O.run_job(job, fuel=fuel)
    assert r.instructions == B * sum(min(fuel, 4 + 3 * t) for t in range(T))
    assert len(r.faults) == sum(1 for t in range(T) if 4 + 3 * t > fuel) * B
