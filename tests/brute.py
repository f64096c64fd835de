"""Brute-force enumeration of every thread interleaving of a tiny launch.

Test infrastructure that pins the oracle.  The paper's semantics lets the
threads of a grid interleave arbitrarily; the only constraints are the barrier
(all threads of a block must wait before any proceeds, Section 3 "Barrier
synchronization") and grid completion (Section 3 "Threads and memory").  This
module explores *all* such interleavings, one instruction at a time, with its
own small interpreter written independently of the oracle, and reports the set
of reachable outcomes.

Per maximal execution it records: the final global memory, whether some block
ended stuck at a barrier (deadlock), the multiset of access records, whether
any two accesses conflict (same location, different threads, one a write, not
separated by a completed barrier episode of their block for intra-block pairs;
any epochs for global accesses of different blocks), and the set of per-access
findings: out-of-bounds accesses (the load yields 0, the store is dropped, no
record), division by zero, threads that run out of fuel, and loads of shared
words that no thread of the block has stored to earlier in the interleaving.

Findings use the report's numbering: (kind, block, epoch, a, b, c) with
OOB = 3 {a = 2 * space + (1 for a store), b = tid, c = the address as an
unsigned 32-bit value}, FUEL = 4 {a = 0, b = tid, c = 0} and
ARITH = 5 {a = 0, b = tid, c = pc} and UNINIT = 7 {a = 0, b = tid, c = the
shared word}.  A thread whose turn comes at the end of
the program exits; otherwise, with no fuel left, it records FUEL and exits;
otherwise it executes one instruction and spends one unit of fuel.
"""
from __future__ import annotations

from collections import Counter
from dataclasses import dataclass
from typing import Dict, FrozenSet, List, Set, Tuple

M32 = 0xFFFFFFFF


def s32(x: int) -> int:
    x &= M32
    return x - (1 << 32) if x & 0x80000000 else x


def _trunc_div(x: int, y: int) -> int:
    q = abs(x) // abs(y)
    return q if (x < 0) == (y < 0) else -q


def alu(name: str, x: int, y: int) -> int:
    """Two's-complement int32 semantics of the IR's ALU ops."""
    if name == "ADD": return s32(x + y)
    if name == "SUB": return s32(x - y)
    if name == "MUL": return s32(x * y)
    if name == "DIV":
        if y == 0: return 0
        if x == -(1 << 31) and y == -1: return x
        return s32(_trunc_div(x, y))
    if name == "REM":
        if y == 0: return 0
        if x == -(1 << 31) and y == -1: return 0
        return s32(x - _trunc_div(x, y) * y)
    if name == "AND": return s32(x & y)
    if name == "OR": return s32(x | y)
    if name == "XOR": return s32(x ^ y)
    if name == "SHL": return s32((x & M32) << (y & 31))
    if name == "SHRA": return s32(x >> (y & 31))
    if name == "SHRL": return s32((x & M32) >> (y & 31))
    if name == "MIN": return min(x, y)
    if name == "MAX": return max(x, y)
    if name == "SLT": return int(x < y)
    if name == "SLE": return int(x <= y)
    if name == "SEQ": return int(x == y)
    if name == "SNE": return int(x != y)
    if name == "SLTU": return int((x & M32) < (y & M32))
    raise ValueError(name)


_RR = ["ADD", "SUB", "MUL", "DIV", "REM", "AND", "OR", "XOR", "SHL", "SHRA", "SHRL",
       "MIN", "MAX", "SLT", "SLE", "SEQ", "SNE", "SLTU"]
_OPS: Dict[int, Tuple[str, bool]] = {}
for _i, _n in enumerate(_RR):
    _OPS[_i + 1] = (_n, False)
    _OPS[(_i + 1) | 0x20] = (_n, True)


def _dec(w: int):
    imm = (w >> 32) & M32
    return w & 0xFF, (w >> 8) & 0xFF, (w >> 16) & 0xFF, (w >> 24) & 0xFF, s32(imm)


OOB, FUEL, ARITH, UNINIT = 3, 4, 5, 7


@dataclass
class Outcome:
    memory: Tuple[int, ...]
    deadlock: bool
    racy: bool
    records: FrozenSet  # frozenset of (record, count)
    findings: FrozenSet = frozenset()   # (kind, block, epoch, a, b, c)


def _racy(recs: Counter, nt: int) -> bool:
    items = list(recs)
    for i, x in enumerate(items):
        for y in items[i:]:
            sp, ad, bl, ep, ti, ki = x
            sp2, ad2, bl2, ep2, ti2, ki2 = y
            if sp != sp2 or ad != ad2 or (ki == 0 and ki2 == 0):
                continue
            if bl == bl2:
                if ti != ti2 and ep == ep2:
                    return True
            elif sp == 1:
                return True
    return False


def enumerate_launch(prog: List[int], grid: int, block: int, shmem_words: int,
                     memory: List[int], params=(), limit_states: int = 2_000_000,
                     fuel: int = 1 << 20) -> List[Outcome]:
    """All outcomes of one launch (1-D grid/block) over every interleaving;
    each thread may execute at most ``fuel`` instructions."""
    n = len(prog)
    params = list(params) + [0] * (8 - len(params))
    nt, nb = block, grid
    code = [_dec(w) for w in prog]

    def sreg(k, tid, bid):
        table = {0: tid, 1: 0, 2: 0, 3: bid, 4: 0, 5: 0, 6: block, 7: 1, 8: 1, 9: grid, 10: 1, 11: 1,
                 12: tid, 13: bid, 14: nt, 15: 32}
        return table[k] if k < 16 else params[k - 16]

    # thread state: (pc, regs, status, bar_pc, fuel left)  status 0 run, 1 wait, 2 exit
    init_threads = tuple((0, (0,) * 16, 0, -1, fuel) for _ in range(nb * nt))
    # the last item: per block, the shared words stored to so far
    init = (init_threads, tuple(tuple([0] * shmem_words) for _ in range(nb)), tuple(memory),
            (0,) * nb, frozenset(), frozenset(), (frozenset(),) * nb)
    seen: Set = set()
    outcomes: Dict = {}
    stack = [init]
    while stack:
        st = stack.pop()
        if st in seen:
            continue
        seen.add(st)
        if len(seen) > limit_states:
            raise RuntimeError("state space too large")
        threads, shs, gm, epochs, recs, finds, stored = st
        succ = []
        # barrier releases (deterministic per block)
        released = False
        for b in range(nb):
            ts = threads[b * nt:(b + 1) * nt]
            if all(t[2] == 1 for t in ts):
                nts = list(threads)
                # predicate barriers: registers are unchanged while waiting
                preds = [code[t[3]][0] == 0x65 and t[1][code[t[3]][2]] != 0 for t in ts]
                for k in range(nt):
                    pc, rg, s, bp, fl = ts[k]
                    op_b, d_b, _, _, kind = code[bp]
                    if op_b == 0x65:
                        rg = list(rg)
                        rg[d_b] = [sum(preds), int(all(preds)), int(any(preds))][kind]
                        rg = tuple(rg)
                    nts[b * nt + k] = (bp + 1, rg, 0, -1, fl)
                ne = list(epochs); ne[b] += 1
                succ.append((tuple(nts), shs, gm, tuple(ne), recs, finds, stored))
                released = True
                break
        if not released:
            for g in range(nb * nt):
                pc, rg, s, bp, fl = threads[g]
                if s != 0:
                    continue
                b, t = divmod(g, nt)
                nts = list(threads); nshs = shs; ngm = gm; nrec = recs; nfind = finds; nst = stored
                if pc == n:
                    nts[g] = (pc, rg, 2, -1, fl)
                    succ.append((tuple(nts), nshs, ngm, epochs, nrec, nfind, nst))
                    continue
                if fl == 0:
                    nts[g] = (pc, rg, 2, -1, fl)
                    succ.append((tuple(nts), nshs, ngm, epochs, nrec, finds | {(FUEL, b, epochs[b], 0, t, 0)}, nst))
                    continue
                op, d, a, bb, imm = code[pc]
                regs = list(rg)
                npc, ns, nbp = pc + 1, 0, -1

                def addrec(space, addr, kind):
                    c = Counter(dict(recs))
                    c[(space, addr, b, epochs[b], t, kind)] += 1
                    return frozenset(c.items())

                def finding(kind, a_, c_):
                    return finds | {(kind, b, epochs[b], a_, t, c_ & M32)}

                if op in _OPS:
                    name, isimm = _OPS[op]
                    y = imm if isimm else regs[bb]
                    regs[d] = alu(name, regs[a], y)
                    if name in ("DIV", "REM") and y == 0:
                        nfind = finding(ARITH, 0, pc)
                elif op == 0x40: regs[d] = regs[a]
                elif op == 0x41: regs[d] = imm
                elif op == 0x42: regs[d] = sreg(imm, t, b)
                elif op in (0x50, 0x52):
                    addr = s32(regs[a] + imm)
                    if op == 0x50:
                        ok = 0 <= addr < shmem_words
                        regs[d] = shs[b][addr] if ok else 0
                        if ok:
                            nrec = addrec(0, addr, 0)
                            if addr not in stored[b]:
                                nfind = finding(UNINIT, 0, addr)
                        else:
                            nfind = finding(OOB, 0, addr)
                    else:
                        ok = 0 <= addr < len(gm)
                        regs[d] = gm[addr] if ok else 0
                        if ok: nrec = addrec(1, addr, 0)
                        else: nfind = finding(OOB, 2, addr)
                elif op in (0x51, 0x53):
                    addr = s32(regs[a] + imm)
                    if op == 0x51:
                        if 0 <= addr < shmem_words:
                            row = list(shs[b]); row[addr] = regs[bb]
                            nshs = shs[:b] + (tuple(row),) + shs[b + 1:]
                            nrec = addrec(0, addr, 1)
                            nst = stored[:b] + (stored[b] | {addr},) + stored[b + 1:]
                        else:
                            nfind = finding(OOB, 1, addr)
                    else:
                        if 0 <= addr < len(gm):
                            m = list(gm); m[addr] = regs[bb]; ngm = tuple(m)
                            nrec = addrec(1, addr, 1)
                        else:
                            nfind = finding(OOB, 3, addr)
                elif op == 0x60: npc = imm
                elif op == 0x61: npc = imm if regs[a] == 0 else pc + 1
                elif op == 0x62: npc = imm if regs[a] != 0 else pc + 1
                elif op in (0x63, 0x65): ns, nbp = 1, pc
                elif op == 0x64: ns = 2
                else:
                    raise ValueError(f"bad opcode {op:#x}")
                nts[g] = (npc, tuple(regs), ns, nbp, fl - 1)
                succ.append((tuple(nts), nshs, ngm, epochs, nrec, nfind, nst))
        if not succ:
            deadlock = any(any(threads[b * nt + k][2] == 1 for k in range(nt)) for b in range(nb))
            c = Counter(dict(recs))
            oc = Outcome(gm, deadlock, _racy(c, nt), recs, finds)
            outcomes[(gm, deadlock, oc.racy, recs, finds)] = oc
        else:
            stack.extend(succ)
    return list(outcomes.values())
