"""KC-IR v1: the instruction format of the simulated CUDA-C-like kernels.

The paper's checker interprets CUDA-C source through the K semantics (Section 3);
this library interprets a small register IR instead (no C front end).  The IR
covers exactly the kernel features the paper's race/deadlock tool exercises
(Section 3, feature list): thread/block indices and dimensions, int32
arithmetic, shared and global loads/stores, conditionals, bounded loops and
``__syncthreads()``.

Encoding (64-bit little-endian word per instruction)::

    bits  0..7   op
    bits  8..15  d   (destination register)
    bits 16..23  a   (first source / address base register)
    bits 24..31  b   (second source / stored-value register)
    bits 32..63  imm (signed int32)

This module only *encodes* programs (it is the input side of the library).
The CPU oracle and the HIP interpreter each decode words with their own code.
"""
from __future__ import annotations

import re
from typing import Dict, Iterable, List, Optional, Sequence, Tuple, Union

N_REGS = 16
MAX_INSTR = 1 << 16

# --- opcodes ---------------------------------------------------------------
# register-register ALU: d = a OP b.  The immediate form (d = a OP imm) has
# the same low five bits with 0x20 set.
ALU_RR = {
    "ADD": 0x01, "SUB": 0x02, "MUL": 0x03, "DIV": 0x04, "REM": 0x05,
    "AND": 0x06, "OR": 0x07, "XOR": 0x08, "SHL": 0x09, "SHRA": 0x0A,
    "SHRL": 0x0B, "MIN": 0x0C, "MAX": 0x0D, "SLT": 0x0E, "SLE": 0x0F,
    "SEQ": 0x10, "SNE": 0x11, "SLTU": 0x12,
}
ALU_RI = {name + "I": code | 0x20 for name, code in ALU_RR.items()}
OTHER = {
    "MOV": 0x40,   # d = a
    "MOVI": 0x41,  # d = imm
    "SREG": 0x42,  # d = special register #imm
    "LDS": 0x50,   # d = shared[a + imm]
    "STS": 0x51,   # shared[a + imm] = b
    "LDG": 0x52,   # d = global[a + imm]
    "STG": 0x53,   # global[a + imm] = b
    "JMP": 0x60,   # pc = imm
    "BZ": 0x61,    # if a == 0: pc = imm
    "BNZ": 0x62,   # if a != 0: pc = imm
    "BAR": 0x63,   # __syncthreads()
    "EXIT": 0x64,  # thread returns
    "BARP": 0x65,  # d = __syncthreads_count/and/or(a) for imm = 0/1/2
}
BARP_KINDS = {"COUNT": 0, "AND": 1, "OR": 2}
OPCODES: Dict[str, int] = {**ALU_RR, **ALU_RI, **OTHER}
OPNAMES: Dict[int, str] = {v: k for k, v in OPCODES.items()}

# --- special registers (operand of SREG) -----------------------------------
SREGS = {
    "TID_X": 0, "TID_Y": 1, "TID_Z": 2,
    "BID_X": 3, "BID_Y": 4, "BID_Z": 5,
    "BDIM_X": 6, "BDIM_Y": 7, "BDIM_Z": 8,
    "GDIM_X": 9, "GDIM_Y": 10, "GDIM_Z": 11,
    "TID": 12, "BID": 13, "NTHREADS": 14, "WARPSIZE": 15,
    **{f"PARAM{i}": 16 + i for i in range(8)},
}
N_SREGS = 24


def encode(op: int, d: int = 0, a: int = 0, b: int = 0, imm: int = 0) -> int:
    """Pack one instruction into its 64-bit word."""
    if not (0 <= op < 256 and 0 <= d < 256 and 0 <= a < 256 and 0 <= b < 256):
        raise ValueError("field out of range")
    if not (-(1 << 31) <= imm < (1 << 32)):
        raise ValueError("immediate out of int32 range")
    return op | (d << 8) | (a << 16) | (b << 24) | ((imm & 0xFFFFFFFF) << 32)


def decode(word: int) -> Tuple[int, int, int, int, int]:
    """Unpack a word into (op, d, a, b, imm) with imm sign-extended."""
    imm = (word >> 32) & 0xFFFFFFFF
    if imm >= 1 << 31:
        imm -= 1 << 32
    return word & 0xFF, (word >> 8) & 0xFF, (word >> 16) & 0xFF, (word >> 24) & 0xFF, imm


Label = str
Operand = Union[int, Label]


class Asm:
    """Builder for KC-IR programs with symbolic labels.

    Methods are named after the mnemonics: ``a.ADD(d, x, y)``, ``a.ADDI(d, x, 5)``,
    ``a.LDS(d, base, off)``, ``a.STS(base, off, src)``, ``a.BZ(reg, "label")``,
    ``a.SREG(d, "TID")``.  Registers are plain ints 0..15.
    """

    def __init__(self) -> None:
        self._code: List[Tuple[int, int, int, int, Operand]] = []
        self._labels: Dict[str, int] = {}

    # structural helpers --------------------------------------------------
    def label(self, name: str) -> "Asm":
        if name in self._labels:
            raise ValueError(f"duplicate label {name}")
        self._labels[name] = len(self._code)
        return self

    def here(self) -> int:
        return len(self._code)

    def _emit(self, op: str, d: int = 0, a: int = 0, b: int = 0, imm: Operand = 0) -> "Asm":
        for r in (d, a, b):
            if not (0 <= r < N_REGS):
                raise ValueError(f"register r{r} out of range")
        self._code.append((OPCODES[op], d, a, b, imm))
        return self

    def assemble(self) -> List[int]:
        words = []
        for op, d, a, b, imm in self._code:
            if isinstance(imm, str):
                if imm not in self._labels:
                    raise ValueError(f"undefined label {imm}")
                imm = self._labels[imm]
            words.append(encode(op, d, a, b, imm))
        if not words or len(words) > MAX_INSTR:
            raise ValueError("program length must be in [1, 65536]")
        return words

    # instructions --------------------------------------------------------
    def __getattr__(self, name: str):
        if name in ALU_RR:
            return lambda d, a, b: self._emit(name, d, a, b, 0)
        if name in ALU_RI:
            return lambda d, a, imm: self._emit(name, d, a, 0, imm)
        raise AttributeError(name)

    def MOV(self, d, a):
        return self._emit("MOV", d, a)

    def MOVI(self, d, imm):
        return self._emit("MOVI", d, 0, 0, imm)

    def SREG(self, d, kind: Union[str, int]):
        k = SREGS[kind] if isinstance(kind, str) else int(kind)
        return self._emit("SREG", d, 0, 0, k)

    def LDS(self, d, base, off=0):
        return self._emit("LDS", d, base, 0, off)

    def STS(self, base, off, src):
        return self._emit("STS", 0, base, src, off)

    def LDG(self, d, base, off=0):
        return self._emit("LDG", d, base, 0, off)

    def STG(self, base, off, src):
        return self._emit("STG", 0, base, src, off)

    def JMP(self, target: Operand):
        return self._emit("JMP", 0, 0, 0, target)

    def BZ(self, a, target: Operand):
        return self._emit("BZ", 0, a, 0, target)

    def BNZ(self, a, target: Operand):
        return self._emit("BNZ", 0, a, 0, target)

    def BAR(self):
        return self._emit("BAR")

    def BARP(self, d, a, kind: Union[str, int] = "COUNT"):
        """Barrier with a predicate: d = count of threads with a != 0 (COUNT),
        all of them (AND) or any (OR), once every thread of the block waits."""
        k = BARP_KINDS[kind] if isinstance(kind, str) else int(kind)
        return self._emit("BARP", d, a, 0, k)

    def EXIT(self):
        return self._emit("EXIT")


# --- text assembler ---------------------------------------------------------
_TOK = re.compile(r"\s*,\s*|\s+")


def _reg(tok: str) -> int:
    if not re.fullmatch(r"r\d+", tok):
        raise ValueError(f"expected register, got {tok!r}")
    return int(tok[1:])


def _mem(tok: str) -> Tuple[int, Operand]:
    m = re.fullmatch(r"\[\s*(r\d+)\s*(?:([+-])\s*(-?\w+))?\s*\]", tok)
    if not m:
        raise ValueError(f"expected [rX+imm], got {tok!r}")
    off = 0
    if m.group(3):
        off = int(m.group(3), 0)
        if m.group(2) == "-":
            off = -off
    return _reg(m.group(1)), off


def assemble_text(src: str) -> List[int]:
    """Assemble a text listing (one instruction per line, ``name:`` labels, ``;`` comments)."""
    a = Asm()
    for raw in src.splitlines():
        line = raw.split(";", 1)[0].strip()
        while line and re.match(r"^[A-Za-z_]\w*:", line):
            name, line = line.split(":", 1)
            a.label(name.strip())
            line = line.strip()
        if not line:
            continue
        mn, _, rest = line.partition(" ")
        mn = mn.upper()
        # memory operands may contain spaces; split by commas outside brackets
        args = [t.strip() for t in re.split(r",(?![^\[]*\])", rest) if t.strip()]
        imm = lambda t: int(t, 0) if re.fullmatch(r"-?(0x)?[0-9a-fA-F]+", t) else t
        if mn in ALU_RR:
            a._emit(mn, _reg(args[0]), _reg(args[1]), _reg(args[2]))
        elif mn in ALU_RI:
            a._emit(mn, _reg(args[0]), _reg(args[1]), 0, imm(args[2]))
        elif mn == "MOV":
            a.MOV(_reg(args[0]), _reg(args[1]))
        elif mn == "MOVI":
            a.MOVI(_reg(args[0]), imm(args[1]))
        elif mn == "SREG":
            a.SREG(_reg(args[0]), args[1].upper() if args[1].upper() in SREGS else int(args[1], 0))
        elif mn in ("LDS", "LDG"):
            base, off = _mem(args[1])
            a._emit(mn, _reg(args[0]), base, 0, off)
        elif mn in ("STS", "STG"):
            base, off = _mem(args[0])
            a._emit(mn, 0, base, _reg(args[1]), off)
        elif mn == "JMP":
            a.JMP(imm(args[0]))
        elif mn in ("BZ", "BNZ"):
            a._emit(mn, 0, _reg(args[0]), 0, imm(args[1]))
        elif mn in ("BAR", "EXIT"):
            a._emit(mn)
        elif mn == "BARP":
            k = args[2].upper()
            a.BARP(_reg(args[0]), _reg(args[1]), k if k in BARP_KINDS else int(k, 0))
        else:
            raise ValueError(f"unknown mnemonic {mn!r}")
    return a.assemble()


def disassemble(words: Sequence[int]) -> str:
    """Render words back to text (labels as absolute pcs)."""
    out = []
    sreg_names = {v: k for k, v in SREGS.items()}
    for pc, w in enumerate(words):
        op, d, a, b, imm = decode(w)
        name = OPNAMES.get(op, f"?{op:#x}")
        if name in ALU_RR:
            s = f"{name} r{d}, r{a}, r{b}"
        elif name in ALU_RI:
            s = f"{name} r{d}, r{a}, {imm}"
        elif name == "MOV":
            s = f"MOV r{d}, r{a}"
        elif name == "MOVI":
            s = f"MOVI r{d}, {imm}"
        elif name == "SREG":
            s = f"SREG r{d}, {sreg_names.get(imm, imm)}"
        elif name in ("LDS", "LDG"):
            s = f"{name} r{d}, [r{a}+{imm}]"
        elif name in ("STS", "STG"):
            s = f"{name} [r{a}+{imm}], r{b}"
        elif name == "JMP":
            s = f"JMP {imm}"
        elif name in ("BZ", "BNZ"):
            s = f"{name} r{a}, {imm}"
        elif name == "BARP":
            s = f"BARP r{d}, r{a}, {({v: k for k, v in BARP_KINDS.items()}).get(imm, imm)}"
        else:
            s = name
        out.append(f"{pc:5d}: {s}")
    return "\n".join(out)


def pcs_of(words: Sequence[int], mnemonic: str) -> List[int]:
    """Program counters of every instruction with the given mnemonic."""
    code = OPCODES[mnemonic]
    return [pc for pc, w in enumerate(words) if (w & 0xFF) == code]
