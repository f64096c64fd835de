"""Seeded synthetic workloads: KC-IR programs, launch shapes and initial memory.

This module only builds inputs.  It holds no interpretation or checking logic,
so both the CPU oracle (in tests) and the HIP path consume the same jobs.

Families (all int32):

* ``SUM``  -- the two-level shared-memory array sum of the paper's Figure 1,
  with the variants the paper runs in Section 3.2: the second barrier removed
  (``NOBAR14``) and a barrier inserted inside the ``if`` (``BAR11``).
* ``TREE`` -- shared-memory tree reduction.  ``tree256_tables`` is the
  table-driven 256-thread form used at scale (a per-block table selects the
  dropped barrier and the tid-dependent barrier); ``tree`` is the power-of-two
  tree with a ``t+s<T`` guard for arbitrary multiples of 32 threads.
* ``STENCIL`` -- 1-D 3-point stencil through a shared tile with halos.
* ``TRANSPOSE`` -- 32x32 tiled transpose through a 32x33 padded shared tile.

Seeds: base 12116193; workload c draws from ``numpy.random.default_rng(12116193+c)``,
per-instance streams from ``SeedSequence(12116193+c).spawn(n)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .ir import Asm

BASE_SEED = 12116193


@dataclass
class LaunchSpec:
    program: np.ndarray                 # uint64 words
    grid: Tuple[int, int, int]
    block: Tuple[int, int, int]
    shmem_bytes: int
    params: Tuple[int, ...] = ()

    @property
    def n_blocks(self) -> int:
        return self.grid[0] * self.grid[1] * self.grid[2]

    @property
    def n_threads(self) -> int:
        return self.block[0] * self.block[1] * self.block[2]


ITEM_KINDS = ("launch", "copy", "host_read", "host_write", "host_wait")


@dataclass
class Item:
    """One step of a job's host program (used when ``Job.items`` is set):
    ``launch`` runs ``launches[launch]`` in ``stream``; ``copy`` moves
    ``words`` words from ``src`` to ``dst`` in ``stream`` (``sync``: the host
    waits for it, as for a cudaMemcpy); ``host_read`` / ``host_write`` are
    the host touching words ``[dst, dst + words)`` (a write stores
    ``value``); ``host_wait`` blocks the host until item ``wait`` (None:
    every earlier device item) has finished."""
    kind: str
    stream: int = 0
    launch: int = 0
    dst: int = 0
    src: int = 0
    words: int = 0
    value: int = 0
    wait: Optional[int] = None
    sync: bool = False


def launch_item(launch: int, stream: int = 0) -> Item:
    return Item("launch", stream=stream, launch=launch)


def copy_item(dst: int, src: int, words: int, stream: int = 0, sync: bool = False) -> Item:
    return Item("copy", stream=stream, dst=dst, src=src, words=words, sync=sync)


def host_read(addr: int, words: int) -> Item:
    return Item("host_read", dst=addr, words=words)


def host_write(addr: int, words: int, value: int) -> Item:
    return Item("host_write", dst=addr, words=words, value=value)


def host_wait(item: Optional[int] = None) -> Item:
    return Item("host_wait", wait=item)


@dataclass
class Job:
    launches: List[LaunchSpec]
    memory: np.ndarray                  # int32 initial global memory
    meta: Dict = field(default_factory=dict)
    streams: Optional[List[int]] = None             # stream of each launch (None: one stream)
    deps: List[Tuple[int, int]] = field(default_factory=list)   # (before, after): after waits for before
    allocs: Optional[List[Tuple[int, int]]] = None  # device allocations (base, words); None: no check
    # host program order of launches, copies and host steps; None: the
    # launches in order (with ``streams``).  With items, ``deps`` and every
    # report's launch field index items, and ``streams`` must be None.
    items: Optional[List[Item]] = None


def _prog(a: Asm) -> np.ndarray:
    return np.array(a.assemble(), dtype=np.uint64)


# ---------------------------------------------------------------------------
# Figure 1: sum
# ---------------------------------------------------------------------------
SUM_VARIANTS = ("BASE", "NOBAR14", "BAR11")


def sum_program(variant: str = "BASE") -> np.ndarray:
    """Figure 1's ``sum`` kernel.  Registers: r0 tid, r1 bid, r2 bdim, r3 in,
    r4 out, r7 bdim/2, r13 loop counter i, r12 loop limit, r15 stays 0."""
    if variant not in SUM_VARIANTS:
        raise ValueError(variant)
    a = Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "BDIM_X").SREG(3, "PARAM0").SREG(4, "PARAM1")
    # line 9: shared[tid] = in[bid * bdim + tid]
    a.MUL(5, 1, 2).ADD(5, 5, 0).ADD(5, 5, 3).LDG(6, 5, 0).STS(0, 0, 6)
    a.BAR()                                         # line 10
    a.SHRAI(7, 2, 1).SLT(8, 0, 7).BZ(8, "L14")      # line 11: if (tid < bdim/2)
    if variant == "BAR11":
        a.BAR()                                     # barrier inserted after line 11
    a.ADD(9, 7, 0).LDS(10, 0, 0).LDS(11, 9, 0).ADD(10, 10, 11).STS(0, 0, 10)  # line 12
    a.label("L14")
    if variant != "NOBAR14":
        a.BAR()                                     # line 14
    a.SEQI(8, 0, 0).BZ(8, "END")                    # line 15: if (tid == 0)
    a.ANDI(12, 2, 1).ADD(12, 7, 12).MOVI(13, 1)     # i = 1; limit = bdim/2 + bdim%2
    a.label("LOOP")
    a.SEQ(8, 13, 12).BNZ(8, "OUT")                  # line 16: i != limit
    a.LDS(10, 15, 0).LDS(11, 13, 0).ADD(10, 10, 11).STS(15, 0, 10)  # line 17
    a.ADDI(13, 13, 1).JMP("LOOP")
    a.label("OUT")
    a.LDS(10, 15, 0).ADD(14, 4, 1).STG(14, 0, 10)   # line 19: out[bid] = shared[0]
    a.label("END")
    a.EXIT()
    return _prog(a)


PAPER_INPUT = [(21 * i + 29) % 100 for i in range(18)]


def fig1_job(variant: str = "BASE", inputs: Optional[Sequence[int]] = None,
             out_init: Sequence[int] = (0, 0)) -> Job:
    """Figure 1's host program: N=18, ``sum<<<2,9,36>>>(in,out)`` then
    ``sum<<<1,2,8>>>(out,out)`` on one memory of 20 words (in=[0,18), out=[18,20))."""
    if inputs is None:
        inputs = PAPER_INPUT
    mem = np.zeros(20, dtype=np.int32)
    mem[:18] = np.asarray(inputs, dtype=np.int32)
    mem[18:20] = np.asarray(out_init, dtype=np.int32)
    p = sum_program(variant)
    launches = [
        LaunchSpec(p, (2, 1, 1), (9, 1, 1), 36, (0, 18)),
        LaunchSpec(p, (1, 1, 1), (2, 1, 1), 8, (18, 18)),
    ]
    return Job(launches, mem, {"family": "SUM", "variant": variant})


def config1_jobs() -> List[Job]:
    """Workload 1: Figure 1 with seeded inputs uniform in [0,100) and with the
    paper's inputs, each in the three variants."""
    rng = np.random.default_rng(BASE_SEED + 1)
    seeded = rng.integers(0, 100, 18).astype(np.int32).tolist()
    jobs = []
    for inputs, tag in ((PAPER_INPUT, "paper"), (seeded, "seeded")):
        for v in SUM_VARIANTS:
            j = fig1_job(v, inputs)
            j.meta["inputs"] = tag
            jobs.append(j)
    return jobs


# ---------------------------------------------------------------------------
# Tree reduction, table-driven (workload 2)
# ---------------------------------------------------------------------------
def tree256_tables_program() -> np.ndarray:
    """Tree reduction where a per-block table entry ``drop[bid]=k`` skips the
    barrier after level k and ``div[bid]=j`` adds ``if (tid < s_j) BAR``.
    Params: P0 in, P1 out, P2 drop table, P3 div table."""
    a = Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS")
    a.SREG(5, "PARAM2").ADD(5, 5, 1).LDG(3, 5, 0)            # r3 = drop[bid]
    a.SREG(5, "PARAM3").ADD(5, 5, 1).LDG(4, 5, 0)            # r4 = div[bid]
    a.MUL(5, 1, 2).ADD(5, 5, 0).SREG(9, "PARAM0").ADD(5, 5, 9)
    a.LDG(10, 5, 0).STS(0, 0, 10).BAR()                      # sh[t] = in[g]
    a.SHRAI(6, 2, 1).MOVI(7, 0)                              # s = T/2, k = 0
    a.label("LOOP")
    a.BZ(6, "DONE")
    a.SLT(8, 0, 6).BZ(8, "SKIP")
    a.ADD(9, 0, 6).LDS(10, 0, 0).LDS(11, 9, 0).ADD(10, 10, 11).STS(0, 0, 10)
    a.label("SKIP")
    a.SEQ(9, 4, 7).AND(9, 9, 8).BZ(9, "NODIV").BAR()         # injected tid-dependent barrier
    a.label("NODIV")
    a.SEQ(9, 3, 7).BNZ(9, "NOBAR").BAR()                     # barrier after level k unless dropped
    a.label("NOBAR")
    a.SHRAI(6, 6, 1).ADDI(7, 7, 1).JMP("LOOP")
    a.label("DONE")
    a.BNZ(0, "END").LDS(10, 15, 0).SREG(9, "PARAM1").ADD(9, 9, 1).STG(9, 0, 10)
    a.label("END")
    a.EXIT()
    return _prog(a)


def tree256_job(n_blocks: int = 4096, threads: int = 256, drop_frac: float = 0.01,
                div_frac: float = 0.001, seed: int = BASE_SEED + 2) -> Job:
    """Workload 2 (defaults): N = n_blocks*threads inputs uniform in [0, 2^16),
    a seeded drop_frac of the blocks skip the barrier after level k~U{0..L-1},
    a disjoint seeded div_frac add a tid-dependent barrier at level j~U{0..L-1}."""
    rng = np.random.default_rng(seed)
    n = n_blocks * threads
    levels = int(math.log2(threads))
    if 1 << levels != threads:
        raise ValueError("threads must be a power of two")
    data = rng.integers(0, 1 << 16, n).astype(np.int32)
    n_drop = int(math.floor(drop_frac * n_blocks))
    n_div = int(math.floor(div_frac * n_blocks))
    perm = rng.permutation(n_blocks)
    drop_blocks = np.sort(perm[:n_drop])
    div_blocks = np.sort(perm[n_drop:n_drop + n_div])
    drop = np.full(n_blocks, -1, dtype=np.int32)
    div = np.full(n_blocks, -1, dtype=np.int32)
    drop[drop_blocks] = rng.integers(0, levels, n_drop)
    div[div_blocks] = rng.integers(0, levels, n_div)
    in_base, out_base = 0, n
    drop_base, div_base = n + n_blocks, n + 2 * n_blocks
    mem = np.zeros(n + 3 * n_blocks, dtype=np.int32)
    mem[:n] = data
    mem[drop_base:drop_base + n_blocks] = drop
    mem[div_base:div_base + n_blocks] = div
    spec = LaunchSpec(tree256_tables_program(), (n_blocks, 1, 1), (threads, 1, 1), 4 * threads,
                      (in_base, out_base, drop_base, div_base))
    return Job([spec], mem, {"family": "TREE256", "n": n, "threads": threads,
                             "n_blocks": n_blocks, "drop": drop, "div": div,
                             "in_base": in_base, "out_base": out_base})


def streams_reduce_job(n_blocks: int = 4096, missing_event: bool = False, seed: int = BASE_SEED + 6) -> Job:
    """Streams and events: two workload-2 tree reductions (1% dropped-barrier
    blocks) over separate input arrays, launched in two streams (they may run in parallel), then a third
    tree launch in the first stream that reduces both partial-sum arrays and
    waits for the second stream through an event (the dependency (1, 2)).
    With ``missing_event`` the wait is left out, so the final launch reads the
    second reduction's partial sums while it may still be writing them."""
    a = tree256_job(n_blocks, div_frac=0.0, seed=seed)        # dropped barriers only: every launch completes
    b = tree256_job(n_blocks, div_frac=0.0, seed=seed + 1000)
    n = n_blocks * 256
    m = 2 * n_blocks // 256                  # blocks of the final reduction
    in_a, in_b, out_a, out_b = 0, n, 2 * n, 2 * n + n_blocks
    tab_a, tab_b = 2 * n + 2 * n_blocks, 2 * n + 4 * n_blocks
    out_c, tab_c = 2 * n + 6 * n_blocks, 2 * n + 6 * n_blocks + m
    mem = np.zeros(tab_c + 2 * m, dtype=np.int32)
    mem[in_a:in_a + n] = a.memory[:n]
    mem[in_b:in_b + n] = b.memory[:n]
    mem[tab_a:tab_a + 2 * n_blocks] = a.memory[n + n_blocks:n + 3 * n_blocks]
    mem[tab_b:tab_b + 2 * n_blocks] = b.memory[n + n_blocks:n + 3 * n_blocks]
    mem[tab_c:tab_c + 2 * m] = -1
    prog = tree256_tables_program()
    launches = [LaunchSpec(prog, (n_blocks, 1, 1), (256, 1, 1), 1024, (in_a, out_a, tab_a, tab_a + n_blocks)),
                LaunchSpec(prog, (n_blocks, 1, 1), (256, 1, 1), 1024, (in_b, out_b, tab_b, tab_b + n_blocks)),
                LaunchSpec(prog, (m, 1, 1), (256, 1, 1), 1024, (out_a, out_c, tab_c, tab_c + m))]
    return Job(launches, mem, {"family": "STREAMS-REDUCE", "n_blocks": n_blocks},
               streams=[0, 1, 0], deps=[] if missing_event else [(1, 2)])


HOST_PROGRAM_BUGS = (None, "event", "wait", "reuse")


def host_program_job(n_blocks: int = 4096, bug: Optional[str] = None, seed: int = BASE_SEED + 7) -> Job:
    """The two-stream reduction of ``streams_reduce_job`` as a whole host
    program (memory transfers and host synchronisation): the two input
    arrays are copied from host buffers in streams 0 and 1 (asynchronously),
    the three tree launches run as there, the final partial sums are copied
    back to a host buffer in stream 0, the host waits for that copy (a stream
    synchronisation), reads the result and then refills the first host input
    buffer.  ``bug`` leaves out one synchronisation: "event" (the final launch
    no longer waits for stream 1), "wait" (the host reads the result before the
    copy back has finished), "reuse" (the host refills the second input buffer
    right after the launches, while its copy in may still be reading it)."""
    if bug not in HOST_PROGRAM_BUGS:
        raise ValueError(f"unknown bug {bug!r}")
    if n_blocks < 128 or n_blocks % 128:
        raise ValueError("n_blocks must be a multiple of 128 (the final launch reduces 2 * n_blocks / 256 blocks)")
    base = streams_reduce_job(n_blocks, seed=seed)
    n = n_blocks * 256
    m = 2 * n_blocks // 256
    dev_words = len(base.memory)
    h_a, h_b, h_out = dev_words, dev_words + n, dev_words + 2 * n
    mem = np.zeros(h_out + m, dtype=np.int32)
    mem[:dev_words] = base.memory
    mem[h_a:h_a + n] = base.memory[0:n]            # host copies of the inputs
    mem[h_b:h_b + n] = base.memory[n:2 * n]
    mem[0:2 * n] = 0                               # device inputs arrive by copy
    in_a, in_b, out_c = 0, n, 2 * n + 6 * n_blocks
    items = [copy_item(in_a, h_a, n, stream=0), copy_item(in_b, h_b, n, stream=1),
             launch_item(0, 0), launch_item(1, 1)]
    if bug == "reuse":
        items.append(host_write(h_b, n, 0))
    items += [launch_item(2, 0), copy_item(h_out, out_c, m, stream=0)]
    if bug != "wait":
        items.append(host_wait(len(items) - 1))
    items += [host_read(h_out, m), host_write(h_a, n, 1)]
    final = items.index(launch_item(2, 0))
    deps = [] if bug == "event" else [(3, final)]
    return Job(base.launches, mem, {"family": "HOST-PROGRAM", "n_blocks": n_blocks, "bug": bug},
               deps=deps, allocs=[(0, dev_words)], items=items)


# ---------------------------------------------------------------------------
# Mixed families (workload 3) with one optionally faulty block
# ---------------------------------------------------------------------------
FAMILIES = ("TREE", "STENCIL", "TRANSPOSE")
FAULTS = {
    "TREE": ("drop", "double", "tidbar"),
    "STENCIL": ("drop", "halo", "double", "tidbar"),
    "TRANSPOSE": ("drop", "double", "tidbar"),
}


def _fault_guard(a: Asm, reg: int) -> None:
    """reg = (bid == PARAM7), i.e. this block is the faulty one."""
    a.SREG(reg, "BID").SREG(14, "PARAM7").SEQ(reg, reg, 14)


def tree_program(fault: Optional[str] = None) -> np.ndarray:
    """Power-of-two tree with a t+s<T guard.  Params: P0 in, P1 out, P2 = P/2
    where P is the smallest power of two >= T, P6 = fault level, P7 = faulty block.
    Faults (only in block PARAM7): ``drop`` skips the barrier after level P6,
    ``double`` makes thread 1 store into slot 0, ``tidbar`` adds
    ``if (tid < T/2) BAR`` after the first barrier."""
    a = Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS")
    if fault is not None:
        _fault_guard(a, 13)                                   # r13 = faulty block?
    a.MUL(5, 1, 2).ADD(5, 5, 0).SREG(9, "PARAM0").ADD(5, 5, 9).LDG(10, 5, 0)
    a.MOV(5, 0)
    if fault == "double":                                     # slot = (faulty && t==1) ? 0 : t
        a.SEQI(9, 0, 1).AND(9, 9, 13).BZ(9, "SLOT").MOVI(5, 0)
        a.label("SLOT")
    a.STS(5, 0, 10).BAR()
    if fault == "tidbar":
        a.SHRAI(9, 2, 1).SLT(9, 0, 9).AND(9, 9, 13).BZ(9, "NOTB").BAR()
        a.label("NOTB")
    a.SREG(6, "PARAM2").MOVI(7, 0)                           # s = P/2, k = 0
    a.label("LOOP")
    a.BZ(6, "DONE")
    a.SLT(8, 0, 6).ADD(9, 0, 6).SLT(11, 9, 2).AND(8, 8, 11).BZ(8, "SKIP")
    a.LDS(10, 0, 0).LDS(11, 9, 0).ADD(10, 10, 11).STS(0, 0, 10)
    a.label("SKIP")
    if fault == "drop":
        a.SREG(9, "PARAM6").SEQ(9, 9, 7).AND(9, 9, 13).BNZ(9, "NOBAR")
    a.BAR()
    a.label("NOBAR")
    a.SHRAI(6, 6, 1).ADDI(7, 7, 1).JMP("LOOP")
    a.label("DONE")
    a.BNZ(0, "END").LDS(10, 15, 0).SREG(9, "PARAM1").ADD(9, 9, 1).STG(9, 0, 10)
    a.label("END")
    a.EXIT()
    return _prog(a)


def stencil_program(fault: Optional[str] = None, inplace_table: bool = False) -> np.ndarray:
    """3-point stencil out[g] = (l + 2c + r) >> 2 with zero boundary, through a
    shared tile of T+2 words: thread t stores in[g] at sh[t+1], thread 0 loads
    the left halo into sh[0], thread T-1 the right halo into sh[T+1].
    Params: P0 in, P1 out, P2 n (elements), P7 faulty block.
    Faults: ``drop`` removes the barrier; ``halo`` makes thread T-2 (instead of
    T-1) load the right halo into sh[t+2]; ``double`` makes thread 1 store into
    sh[1]; ``tidbar`` adds ``if (tid < T/2) BAR`` before the barrier.
    With ``inplace_table`` every thread reads ``bug = mem[P3 + bid]`` and a
    block with bug != 0 writes its output into the input array (in place)."""
    a = Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS")
    if fault is not None:
        _fault_guard(a, 13)
    a.MUL(3, 1, 2).ADD(3, 3, 0)                               # r3 = g
    a.SREG(4, "PARAM0").ADD(5, 4, 3).LDG(10, 5, 0)            # r5 = &in[g]
    a.MOV(6, 0)
    if fault == "double":
        a.SEQI(9, 0, 1).AND(9, 9, 13).BZ(9, "SLOT").MOVI(6, 0)
        a.label("SLOT")
    a.STS(6, 1, 10)                                           # sh[slot+1] = in[g]
    a.BNZ(0, "NOLEFT").MOVI(10, 0).BZ(3, "LSTORE").LDG(10, 5, -1)
    a.label("LSTORE")
    a.STS(15, 0, 10)                                          # sh[0] = left halo
    a.label("NOLEFT")
    a.ADDI(6, 2, -1)                                          # right-halo loader tid
    if fault == "halo":
        a.BZ(13, "HOK").ADDI(6, 2, -2)
        a.label("HOK")
    a.SEQ(8, 0, 6).BZ(8, "NORIGHT")
    a.MOVI(10, 0).SREG(7, "PARAM2").ADDI(9, 3, 1).SLT(8, 9, 7).BZ(8, "RSTORE").LDG(10, 5, 1)
    a.label("RSTORE")
    a.STS(0, 2, 10)                                           # sh[t+2] = right halo
    a.label("NORIGHT")
    if fault == "tidbar":
        a.SHRAI(9, 2, 1).SLT(9, 0, 9).AND(9, 9, 13).BZ(9, "NOTB").BAR()
        a.label("NOTB")
    if fault == "drop":
        a.BNZ(13, "NOBAR")
    a.BAR()
    a.label("NOBAR")
    a.LDS(10, 0, 0).LDS(11, 0, 1).LDS(12, 0, 2)
    a.ADD(10, 10, 12).SHLI(11, 11, 1).ADD(10, 10, 11).SHRAI(10, 10, 2)
    a.SREG(4, "PARAM1")
    if inplace_table:
        a.SREG(9, "PARAM3").ADD(9, 9, 1).LDG(9, 9, 0).BZ(9, "OUTOK").SREG(4, "PARAM0")
        a.label("OUTOK")
    a.ADD(4, 4, 3).STG(4, 0, 10)
    a.EXIT()
    return _prog(a)


def transpose_program(fault: Optional[str] = None) -> np.ndarray:
    """32 x (32*Bn) -> (32*Bn) x 32 transpose; block b moves columns [32b, 32b+32)
    through a 32x33 shared tile, thread t handling column t%32 and rows
    t/32, t/32 + T/32, ...  Params: P0 in, P1 out, P7 faulty block.
    Faults: ``drop`` removes the barrier; ``double`` makes thread 1 use column 0;
    ``tidbar`` adds ``if (tid < T/2) BAR`` before the barrier."""
    a = Asm()
    a.SREG(0, "TID").SREG(1, "BID").SREG(2, "NTHREADS")
    if fault is not None:
        _fault_guard(a, 13)
    a.ANDI(3, 0, 31).SHRAI(4, 0, 5).SHRAI(5, 2, 5)           # tx, ty, step
    a.SHLI(6, 1, 5).SREG(7, "GDIM_X").SHLI(7, 7, 5)          # 32b, W = 32*Bn
    a.SREG(12, "PARAM0").MOV(14, 3)                          # r14 = store column
    if fault == "double":
        a.SEQI(9, 0, 1).AND(9, 9, 13).BZ(9, "COL").MOVI(14, 0)
        a.label("COL")
    a.MOV(8, 4)
    a.label("L1")
    a.SLTI(9, 8, 32).BZ(9, "E1")
    a.MUL(10, 8, 7).ADD(10, 10, 6).ADD(10, 10, 3).ADD(10, 10, 12).LDG(11, 10, 0)
    a.MULI(10, 8, 33).ADD(10, 10, 14).STS(10, 0, 11)         # sh[row*33 + col]
    a.ADD(8, 8, 5).JMP("L1")
    a.label("E1")
    if fault == "tidbar":
        a.SHRAI(9, 2, 1).SLT(9, 0, 9).AND(9, 9, 13).BZ(9, "NOTB").BAR()
        a.label("NOTB")
    if fault == "drop":
        a.BNZ(13, "NOBAR")
    a.BAR()
    a.label("NOBAR")
    a.SREG(12, "PARAM1").MOV(8, 4)
    a.label("L2")
    a.SLTI(9, 8, 32).BZ(9, "E2")
    a.MULI(10, 3, 33).ADD(10, 10, 8).LDS(11, 10, 0)          # sh[tx*33 + row]
    a.ADD(10, 6, 8).SHLI(10, 10, 5).ADD(10, 10, 3).ADD(10, 10, 12).STG(10, 0, 11)
    a.ADD(8, 8, 5).JMP("L2")
    a.label("E2")
    a.EXIT()
    return _prog(a)


_PROGRAM_CACHE: Dict[Tuple[str, Optional[str]], np.ndarray] = {}


def family_program(family: str, fault: Optional[str]) -> np.ndarray:
    key = (family, fault)
    if key not in _PROGRAM_CACHE:
        fn = {"TREE": tree_program, "STENCIL": stencil_program, "TRANSPOSE": transpose_program}[family]
        _PROGRAM_CACHE[key] = fn(fault)
    return _PROGRAM_CACHE[key]


def family_job(family: str, n_blocks: int, threads: int, rng: np.random.Generator,
               fault: Optional[str] = None, fault_block: int = -1, fault_level: int = 0) -> Job:
    """One instance of a workload-3 family with inputs uniform in [0, 2^16)."""
    if threads % 32 or not (32 <= threads <= 1024):
        raise ValueError("threads must be a multiple of 32 in [32, 1024]")
    P7 = fault_block if fault is not None else -1
    if family == "TREE":
        n = n_blocks * threads
        mem = np.zeros(n + n_blocks, dtype=np.int32)
        mem[:n] = rng.integers(0, 1 << 16, n)
        half = 1 << (max(threads - 1, 1).bit_length() - 1)  # P/2 for P = next pow2 >= T
        if (half << 1) < threads:
            half <<= 1
        params = (0, n, half, 0, 0, 0, fault_level, P7)
        spec = LaunchSpec(family_program(family, fault), (n_blocks, 1, 1), (threads, 1, 1),
                          4 * threads, params)
        meta = {"n": n, "in_base": 0, "out_base": n, "half": half}
    elif family == "STENCIL":
        n = n_blocks * threads
        mem = np.zeros(2 * n, dtype=np.int32)
        mem[:n] = rng.integers(0, 1 << 16, n)
        params = (0, n, n, 0, 0, 0, 0, P7)
        spec = LaunchSpec(family_program(family, fault), (n_blocks, 1, 1), (threads, 1, 1),
                          4 * (threads + 2), params)
        meta = {"n": n, "in_base": 0, "out_base": n}
    elif family == "TRANSPOSE":
        n = 32 * 32 * n_blocks
        mem = np.zeros(2 * n, dtype=np.int32)
        mem[:n] = rng.integers(0, 1 << 16, n)
        params = (0, n, 0, 0, 0, 0, 0, P7)
        spec = LaunchSpec(family_program(family, fault), (n_blocks, 1, 1), (threads, 1, 1),
                          4 * 32 * 33, params)
        meta = {"n": n, "in_base": 0, "out_base": n}
    else:
        raise ValueError(family)
    meta.update({"family": family, "n_blocks": n_blocks, "threads": threads, "fault": fault,
                 "fault_block": fault_block if fault else -1, "fault_level": fault_level})
    return Job([spec], mem, meta)


def _loguniform_int(rng: np.random.Generator, hi: int) -> int:
    return int(np.clip(round(math.exp(rng.uniform(0.0, math.log(hi)))), 1, hi))


def mixed_instance(rng: np.random.Generator, fault_p: float = 0.2) -> Job:
    """Draw one workload-3 instance: family uniform, blocks log-uniform in
    [1, 64], threads 32 * log-uniform [1, 32], with probability fault_p one
    seeded block gets a fault type uniform over those that apply."""
    family = FAMILIES[int(rng.integers(0, 3))]
    n_blocks = _loguniform_int(rng, 64)
    threads = 32 * _loguniform_int(rng, 32)
    fault, fblock, flevel = None, -1, 0
    if rng.random() < fault_p:
        opts = FAULTS[family]
        fault = opts[int(rng.integers(0, len(opts)))]
        fblock = int(rng.integers(0, n_blocks))
        if family == "TREE":
            half = 1 << (max(threads - 1, 1).bit_length() - 1)
            if (half << 1) < threads:
                half <<= 1
            flevel = int(rng.integers(0, half.bit_length()))
    return family_job(family, n_blocks, threads, rng, fault, fblock, flevel)


def config3_jobs(n: int = 10000, seed: int = BASE_SEED + 3, fault_p: float = 0.2) -> List[Job]:
    """Workload 3: n independent instances, each from its own spawned stream."""
    ss = np.random.SeedSequence(seed)
    return [mixed_instance(np.random.default_rng(s), fault_p) for s in ss.spawn(n)]


# ---------------------------------------------------------------------------
# Workload 4: big ping-pong stencil with in-place bugs
# ---------------------------------------------------------------------------
def stencil_pingpong_job(n: int = 1 << 26, threads: int = 256, steps: int = 16,
                         bug_frac: float = 0.0001, seed: int = BASE_SEED + 4) -> Job:
    """n elements (A), a second array (B), a per-block bug table; ``steps``
    launches alternate A->B and B->A.  A seeded bug_frac of the blocks write
    their output in place into the array they read (cross-block race with the
    neighbours' halo loads)."""
    rng = np.random.default_rng(seed)
    if n % threads:
        raise ValueError("n must be a multiple of threads")
    n_blocks = n // threads
    n_bug = int(math.floor(bug_frac * n_blocks))
    bug_blocks = np.sort(rng.choice(n_blocks, n_bug, replace=False)) if n_bug else np.zeros(0, np.int64)
    mem = np.zeros(2 * n + n_blocks, dtype=np.int32)
    mem[:n] = rng.integers(0, 1 << 16, n)
    mem[2 * n + bug_blocks] = 1
    prog = stencil_program(None, inplace_table=True)
    A, B, T = 0, n, 2 * n
    launches = []
    for s in range(steps):
        src, dst = (A, B) if s % 2 == 0 else (B, A)
        launches.append(LaunchSpec(prog, (n_blocks, 1, 1), (threads, 1, 1), 4 * (threads + 2),
                                   (src, dst, n, T, 0, 0, 0, -1)))
    return Job(launches, mem, {"family": "STENCIL_PINGPONG", "n": n, "threads": threads,
                               "n_blocks": n_blocks, "bug_blocks": bug_blocks, "steps": steps})


# ---------------------------------------------------------------------------
# Workload 5: request stream
# ---------------------------------------------------------------------------
def request_stream(rate: float, duration_s: float, seed: int = BASE_SEED + 5,
                   big_p: float = 0.05, big_blocks: int = 4096):
    """Poisson arrivals at ``rate``/s over ``duration_s``: yields
    (arrival_time_s, Job).  A request is a workload-3 instance with probability
    1-big_p, else a workload-2-shaped tree (big_blocks x 256) with fresh seeds."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.default_rng(ss.spawn(1)[0])
    t = 0.0
    i = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            return
        sub = np.random.default_rng(np.random.SeedSequence([seed, i]))
        if sub.random() < big_p:
            job = tree256_job(n_blocks=big_blocks, seed=int(sub.integers(0, 2**63 - 1)))
        else:
            job = mixed_instance(sub)
        yield t, job
        i += 1


def request_pool(n_small: int = 2048, n_big: int = 8, big_blocks: int = 4096, seed: int = BASE_SEED + 5):
    """Pre-generated instances for a served run: ``n_small`` workload-3
    instances and ``n_big`` workload-2-shaped trees (``big_blocks`` x 256), each
    from its own seed.  Requests draw from the pool (see pooled_requests), so a
    high arrival rate needs no input generation while the clock runs."""
    small = [mixed_instance(np.random.default_rng(np.random.SeedSequence([seed, 0, i]))) for i in range(n_small)]
    big = [tree256_job(n_blocks=big_blocks,
                       seed=int(np.random.default_rng(np.random.SeedSequence([seed, 1, i])).integers(0, 2**63 - 1)))
           for i in range(n_big)]
    return small, big


def pooled_requests(rate: float, duration_s: float, small, big, big_p: float = 0.05,
                    seed: int = BASE_SEED + 5):
    """Poisson arrivals at ``rate``/s over ``duration_s``: a list of
    (arrival_time_s, Job) where each request is a pool instance, a big tree
    with probability ``big_p``, chosen uniformly by a seeded stream."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 2, int(rate)]))
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            return out
        if big and rng.random() < big_p:
            out.append((t, big[int(rng.integers(0, len(big)))]))
        else:
            out.append((t, small[int(rng.integers(0, len(small)))]))
