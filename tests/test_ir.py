"""IR encoder: round trips, text assembly, and validation rules."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1211_6193_amd import ir, workloads as W


def test_encode_decode_roundtrip():
    rng = np.random.default_rng(0)
    for _ in range(2000):
        op, d, a, b = (int(x) for x in rng.integers(0, 256, 4))
        imm = int(rng.integers(-2**31, 2**31))
        assert ir.decode(ir.encode(op, d, a, b, imm)) == (op, d, a, b, imm)


def test_text_assembler_matches_builder():
    src = """
        SREG r0, TID
        SREG r1, PARAM1
    top: ADDI r2, r2, -1
        LDS r3, [r0+4]
        STG [r1-2], r3
        SLTU r4, r2, r0
        BNZ r4, top
        BAR
        EXIT
    """
    a = ir.Asm()
    a.SREG(0, "TID").SREG(1, "PARAM1").label("top").ADDI(2, 2, -1).LDS(3, 0, 4).STG(1, -2, 3)
    a.SLTU(4, 2, 0).BNZ(4, "top").BAR().EXIT()
    assert ir.assemble_text(src) == a.assemble()


def test_disassemble_reassemble_all_workload_programs():
    progs = [W.sum_program(v) for v in W.SUM_VARIANTS] + [W.tree256_tables_program()]
    progs += [W.family_program(f, x) for f in W.FAMILIES for x in (None,) + W.FAULTS[f]]
    progs += [W.stencil_program(None, inplace_table=True)]
    for p in progs:
        text = ir.disassemble([int(w) for w in p])
        lines = [ln.split(":", 1)[1] for ln in text.splitlines()]
        assert ir.assemble_text("\n".join(lines)) == [int(w) for w in p]
        assert O.validate(p)


@pytest.mark.parametrize("bad", [
    [ir.encode(0x00)],                                   # unknown opcode
    [ir.encode(0x13)],                                   # gap in the ALU range
    [ir.encode(ir.OPCODES["ADD"], 16, 0, 0)],            # register out of range
    [ir.encode(ir.OPCODES["JMP"], imm=2)],               # target past the end
    [ir.encode(ir.OPCODES["BZ"], imm=-1)],               # negative target
    [ir.encode(ir.OPCODES["SREG"], imm=24)],             # unknown special register
    [],                                                  # empty program
])
def test_validator_rejects(bad):
    assert not O.validate(np.array(bad, dtype=np.uint64))


def test_validator_accepts_jump_to_end():
    assert O.validate(np.array([ir.encode(ir.OPCODES["JMP"], imm=1)], dtype=np.uint64))
