"""ctypes binding of the CPU oracle (kc_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library.  It accepts any
job-like object (``job.launches[i].program/grid/block/shmem_bytes/params`` and
``job.memory``) and imports nothing from the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkc_oracle.so")
SRC_PATH = os.path.join(_HERE, "kc_oracle.c")

DEFAULT_FUEL = 1 << 20

F_DEADLOCK, F_DIVERGENCE, F_OOB, F_FUEL, F_ARITH, F_ALLOC, F_UNINIT = 1, 2, 3, 4, 5, 6, 7
CHECK_UNINIT_SHARED, CHECK_WARP = 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 into a shared library next to its source."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, SRC_PATH])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Launch(C.Structure):
    _fields_ = [("grid", C.c_uint32 * 3), ("block", C.c_uint32 * 3), ("shmem_bytes", C.c_uint32),
                ("params", C.c_int32 * 8)]


ITEM_DTYPE = np.dtype([("kind", "<u4"), ("stream", "<u4"), ("ref", "<u4"), ("flags", "<u4"), ("dst", "<u8"),
                       ("src", "<u8"), ("words", "<u8"), ("value", "<i4"), ("pad", "<u4")])
IT_KINDS = {"launch": 0, "copy": 1, "host_read": 2, "host_write": 3, "host_wait": 4}
WAIT_ALL = 0xFFFFFFFF


def item_table(items) -> np.ndarray:
    """The items of a job as the C struct array the oracle reads."""
    t = np.zeros(max(len(items), 1), ITEM_DTYPE)
    for i, it in enumerate(items):
        if it.kind not in IT_KINDS:
            raise ValueError(f"unknown item kind {it.kind!r}")
        t[i]["kind"] = IT_KINDS[it.kind]
        t[i]["stream"] = it.stream
        t[i]["ref"] = it.launch if it.kind == "launch" else (
            (WAIT_ALL if it.wait is None else it.wait) if it.kind == "host_wait" else 0)
        t[i]["flags"] = 1 if it.sync else 0
        t[i]["dst"], t[i]["src"], t[i]["words"] = it.dst, it.src, it.words
        t[i]["value"] = int(np.int32(it.value))
    return t


RACE_DTYPE = np.dtype([(f, "<u4") for f in ("launch", "space", "scope", "block", "epoch", "addr", "w_tid", "o_tid",
                                            "w_pc", "o_pc")])
FAULT_DTYPE = np.dtype([(f, "<u4") for f in ("launch", "kind", "block", "epoch", "a", "b", "c", "d")])
RECORD_DTYPE = np.dtype([(f, "<u4") for f in ("launch", "space", "addr", "block", "epoch", "tid", "kind", "pc",
                                             "step")])

_lib = None
_EMPTY_ALLOCS = (C.c_uint64 * 2)()      # a non-null list of no allocations


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = C.CDLL(LIB_PATH)
        lib.ora_run_job.argtypes = [C.c_uint32, C.POINTER(C.c_void_p), C.POINTER(C.c_uint32),
                                    C.POINTER(_Launch), C.c_void_p, C.c_uint64, C.c_uint32, C.c_int,
                                    C.POINTER(C.c_void_p)]
        lib.ora_run_job.restype = C.c_int
        lib.ora_run_job_ex.argtypes = [C.c_uint32, C.POINTER(C.c_void_p), C.POINTER(C.c_uint32),
                                       C.POINTER(_Launch), C.c_void_p, C.c_uint64, C.c_uint32, C.c_int,
                                       C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32,
                                       C.POINTER(C.c_void_p)]
        lib.ora_run_job_ex.restype = C.c_int
        lib.ora_run_job_opts.argtypes = [C.c_uint32, C.POINTER(C.c_void_p), C.POINTER(C.c_uint32),
                                         C.POINTER(_Launch), C.c_void_p, C.c_uint64, C.c_uint32, C.c_int,
                                         C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32,
                                         C.c_uint32, C.POINTER(C.c_void_p)]
        lib.ora_run_job_opts.restype = C.c_int
        lib.ora_run_items.argtypes = [C.c_uint32, C.POINTER(C.c_void_p), C.POINTER(C.c_uint32),
                                      C.POINTER(_Launch), C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint64,
                                      C.c_uint32, C.c_int, C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32,
                                      C.c_uint32, C.POINTER(C.c_void_p)]
        lib.ora_run_items.restype = C.c_int
        lib.ora_records.argtypes = [C.c_void_p]
        lib.ora_records.restype = C.c_uint64
        lib.ora_instructions.argtypes = [C.c_void_p]
        lib.ora_instructions.restype = C.c_uint64
        lib.ora_launches_completed.argtypes = [C.c_void_p]
        lib.ora_launches_completed.restype = C.c_uint32
        for name in ("ora_races", "ora_faults", "ora_kept_records"):
            f = getattr(lib, name)
            f.argtypes = [C.c_void_p, C.POINTER(C.c_uint64)]
            f.restype = C.c_void_p
        lib.ora_free.argtypes = [C.c_void_p]
        lib.ora_validate.argtypes = [C.c_void_p, C.c_uint32]
        lib.ora_validate.restype = C.c_int
        _lib = lib
    return _lib


@dataclass
class OracleResult:
    records: int                  # canonical access-record count
    launches_completed: int
    races: np.ndarray             # RACE_DTYPE, canonical order
    faults: np.ndarray            # FAULT_DTYPE, canonical order, no duplicates
    memory: np.ndarray            # final global memory (int32)
    record_log: Optional[np.ndarray] = None   # RECORD_DTYPE if keep_records
    instructions: int = 0         # thread-instructions executed (fuel spent)

    def race_tuples(self) -> List[Tuple[int, ...]]:
        """(launch, space, scope, block, epoch, addr, w_tid, o_tid) per race."""
        return [tuple(int(x) for x in tuple(r)[:8]) for r in self.races]

    def race_sites(self) -> List[Tuple[int, int]]:
        """(w_pc, o_pc) per race, in the order of race_tuples()."""
        return [(int(r["w_pc"]), int(r["o_pc"])) for r in self.races]

    def fault_tuples(self) -> List[Tuple[int, ...]]:
        return [tuple(int(x) for x in f) for f in self.faults]


def _copy(ptr, n, dtype):
    if n == 0 or not ptr:
        return np.zeros(0, dtype=dtype)
    buf = (C.c_char * (n * dtype.itemsize)).from_address(ptr)
    return np.frombuffer(bytes(buf), dtype=dtype).copy()


def validate(words) -> bool:
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
    return _load().ora_validate(w.ctypes.data, len(w)) == 0


def run_job(job, fuel: int = DEFAULT_FUEL, keep_records: bool = False,
            memory: Optional[np.ndarray] = None, uninit: bool = False, warp: bool = False) -> OracleResult:
    """Run every launch of ``job`` on a copy of its memory (or on ``memory``).

    ``job.items``, when not None, is the job's host program instead: launches,
    copies, host reads and writes and host waits in order (see ``Item``);
    ``job.deps`` then links items and report launch fields are item indices.

    ``job.streams`` (one stream id per launch) and ``job.deps`` ((before,
    after) launch pairs), when the job has them, describe which launches may
    run in parallel; races between such launches are reported with scope 2.
    ``job.allocs`` ((base, words) ranges), when not None, lists the device
    allocations: accesses outside them are reported as ALLOC findings.
    ``uninit`` turns on the check of loads of shared words no thread of the
    block has stored to before (UNINIT findings); ``warp`` the warp-aware
    model (threads of one warp conflict only at the same step)."""
    lib = _load()
    progs = [np.ascontiguousarray(np.asarray(L.program, dtype=np.uint64)) for L in job.launches]
    n = len(progs)
    ptrs = (C.c_void_p * n)(*[p.ctypes.data for p in progs])
    lens = (C.c_uint32 * n)(*[len(p) for p in progs])
    ls = (_Launch * n)()
    for i, L in enumerate(job.launches):
        ls[i].grid[:] = list(L.grid)
        ls[i].block[:] = list(L.block)
        ls[i].shmem_bytes = L.shmem_bytes
        params = list(L.params) + [0] * (8 - len(L.params))
        ls[i].params[:] = [int(np.int32(p)) for p in params]
    mem = np.array(job.memory if memory is None else memory, dtype=np.int32, copy=True)
    streams = getattr(job, "streams", None)
    deps = getattr(job, "deps", None) or []
    st = None if streams is None else np.ascontiguousarray(np.asarray(streams, dtype=np.uint32))
    if st is not None and len(st) != n:
        raise ValueError("one stream per launch")
    dp = np.ascontiguousarray(np.asarray(deps, dtype=np.uint32).reshape(-1, 2))
    allocs = getattr(job, "allocs", None)
    al = None if allocs is None else np.ascontiguousarray(np.asarray(allocs, dtype=np.uint64).reshape(-1, 2))
    out = C.c_void_p()
    items = getattr(job, "items", None)
    if items is not None:
        if st is not None:
            raise ValueError("a job with items gives each launch item its stream")
        it = item_table(items)
        rc = lib.ora_run_items(n, ptrs, lens, ls, it.ctypes.data, len(items), mem.ctypes.data, len(mem), fuel,
                               int(keep_records), dp.ctypes.data if len(dp) else None, len(dp),
                               None if al is None else (al.ctypes.data if len(al) else C.addressof(_EMPTY_ALLOCS)),
                               0 if al is None else len(al),
                               (CHECK_UNINIT_SHARED if uninit else 0) | (CHECK_WARP if warp else 0), C.byref(out))
    else:
        rc = lib.ora_run_job_opts(n, ptrs, lens, ls, mem.ctypes.data, len(mem), fuel, int(keep_records),
                                  None if st is None else st.ctypes.data, dp.ctypes.data if len(dp) else None,
                                  len(dp), None if al is None else (al.ctypes.data if len(al) else
                                                                    C.addressof(_EMPTY_ALLOCS)),
                                  0 if al is None else len(al),
                                  (CHECK_UNINIT_SHARED if uninit else 0) | (CHECK_WARP if warp else 0),
                                  C.byref(out))
    if rc != 0:
        raise ValueError(f"oracle rejected the job (code {rc})")
    try:
        cnt = C.c_uint64()
        races = _copy(lib.ora_races(out, C.byref(cnt)), cnt.value, RACE_DTYPE)
        faults = _copy(lib.ora_faults(out, C.byref(cnt)), cnt.value, FAULT_DTYPE)
        log = None
        if keep_records:
            log = _copy(lib.ora_kept_records(out, C.byref(cnt)), cnt.value, RECORD_DTYPE)
        return OracleResult(int(lib.ora_records(out)), int(lib.ora_launches_completed(out)),
                            races, faults, mem, log, int(lib.ora_instructions(out)))
    finally:
        lib.ora_free(out)
