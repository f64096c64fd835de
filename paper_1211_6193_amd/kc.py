"""Python binding of libkc (argument marshalling only; all work runs in the HIP library).

PyTorch supplies device memory (int32 tensors on the GPU) and streams.
Loading fails loudly if the compiled library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import collections.abc as cabc
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# The library built in-tree; KC_LIBRARY names another build of it (for
# comparing build variants side by side).
LIB_PATH = os.environ.get("KC_LIBRARY") or os.path.join(_HERE, "libkc.so")

(KC_OK, KC_E_INVAL, KC_E_PROGRAM, KC_E_NOMEM, KC_E_DEVICE, KC_E_PENDING, KC_E_BUDGET, KC_E_OVERFLOW,
 KC_E_INTERNAL) = range(9)
STATUS_NAMES = ["KC_OK", "KC_E_INVAL", "KC_E_PROGRAM", "KC_E_NOMEM", "KC_E_DEVICE", "KC_E_PENDING",
                "KC_E_BUDGET", "KC_E_OVERFLOW", "KC_E_INTERNAL"]
DEADLOCK, DIVERGENCE, OOB, FUEL, ARITH, ALLOC, UNINIT = 1, 2, 3, 4, 5, 6, 7

# Every entry point include/kc.h declares.
EXPORTS = ["kc_ctx_create", "kc_ctx_destroy", "kc_ctx_set_option", "kc_ctx_get_stat", "kc_last_error",
           "kc_program_load", "kc_program_free", "kc_launch", "kc_launch_noalloc", "kc_batch_submit", "kc_poll",
           "kc_batch_footprint",
           "kc_report_records", "kc_report_launches_completed", "kc_report_races", "kc_report_faults",
           "kc_report_race_sites",
           "kc_report_tag", "kc_report_free", "kc_reports_collect", "kc_reports_free"]

RACE_DTYPE = np.dtype([(f, "<u4") for f in ("launch", "space", "scope", "block", "epoch", "addr", "w_tid", "o_tid")])
FAULT_DTYPE = np.dtype([(f, "<u4") for f in ("launch", "kind", "block", "epoch", "a", "b", "c", "d")])
SITE_DTYPE = np.dtype([(f, "<u4") for f in ("w_pc", "o_pc")])


class KcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {msg}")
        self.status = status


class Dim3(C.Structure):
    _fields_ = [("x", C.c_uint32), ("y", C.c_uint32), ("z", C.c_uint32)]


class LaunchDesc(C.Structure):
    _fields_ = [("prog", C.c_void_p), ("grid", Dim3), ("block", Dim3), ("shmem_bytes", C.c_uint32),
                ("params", C.c_int32 * 8), ("n_params", C.c_uint32)]


class Dep(C.Structure):
    _fields_ = [("before", C.c_uint32), ("after", C.c_uint32)]


class Region(C.Structure):
    _fields_ = [("base", C.c_uint64), ("words", C.c_uint64)]


class ItemDesc(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("stream", C.c_uint32), ("ref", C.c_uint32), ("flags", C.c_uint32),
                ("dst", C.c_uint64), ("src", C.c_uint64), ("words", C.c_uint64), ("value", C.c_int32),
                ("pad", C.c_uint32)]


# kc_item kinds (KC_ITEM_*), KC_ITEM_SYNC and KC_WAIT_ALL
ITEM_KINDS = {"launch": 0, "copy": 1, "host_read": 2, "host_write": 3, "host_wait": 4}
ITEM_SYNC = 1
WAIT_ALL = 0xFFFFFFFF


class JobDesc(C.Structure):
    _fields_ = [("launches", C.POINTER(LaunchDesc)), ("n_launches", C.c_uint32), ("dev_mem", C.c_void_p),
                ("n_words", C.c_uint64), ("tag", C.c_uint64), ("streams", C.POINTER(C.c_uint32)),
                ("deps", C.POINTER(Dep)), ("n_deps", C.c_uint32), ("allocs", C.POINTER(Region)),
                ("n_allocs", C.c_uint32), ("items", C.POINTER(ItemDesc)), ("n_items", C.c_uint32)]


def _item_desc(it) -> ItemDesc:
    """One step of a host program (an object with the fields of
    workloads.Item) as a kc_item."""
    if it.kind not in ITEM_KINDS:
        raise ValueError(f"unknown item kind {it.kind!r}")
    ref = it.launch if it.kind == "launch" else (
        (WAIT_ALL if it.wait is None else it.wait) if it.kind == "host_wait" else 0)
    return ItemDesc(ITEM_KINDS[it.kind], it.stream, ref, ITEM_SYNC if it.sync else 0, it.dst, it.src, it.words,
                    int(C.c_int32(it.value).value), 0)


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libkc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1211_6193_amd/build.py (no CPU fallback exists)")
    lib = C.CDLL(path)
    vp, u32, u64, i64 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int64
    sig = {
        "kc_ctx_create": ([C.c_int, u64, C.c_char_p, C.POINTER(vp)], C.c_int),
        "kc_ctx_destroy": ([vp], None),
        "kc_ctx_set_option": ([vp, C.c_char_p, i64], C.c_int),
        "kc_ctx_get_stat": ([vp, C.c_char_p], C.c_double),
        "kc_last_error": ([vp], C.c_char_p),
        "kc_program_load": ([vp, vp, u32, C.POINTER(vp)], C.c_int),
        "kc_program_free": ([vp], None),
        "kc_launch": ([vp, C.POINTER(LaunchDesc), vp, u64, vp, C.POINTER(vp)], C.c_int),
        "kc_launch_noalloc": ([vp, C.POINTER(LaunchDesc), vp, u64, vp, C.POINTER(vp)], C.c_int),
        "kc_batch_submit": ([vp, C.POINTER(JobDesc), u32, vp, C.POINTER(u64)], C.c_int),
        "kc_poll": ([vp, u64, C.c_int, C.POINTER(vp), u32], C.c_int),
        "kc_batch_footprint": ([vp, C.POINTER(JobDesc), u32, C.POINTER(u64)], C.c_int),
        "kc_report_records": ([vp], u64),
        "kc_report_launches_completed": ([vp], u32),
        "kc_report_races": ([vp, C.POINTER(u64)], vp),
        "kc_report_faults": ([vp, C.POINTER(u64)], vp),
        "kc_report_race_sites": ([vp, C.POINTER(u64)], vp),
        "kc_report_tag": ([vp], u64),
        "kc_report_free": ([vp], None),
        "kc_reports_collect": ([vp, u32, vp, vp, vp, vp, vp, vp, vp, vp], C.c_int),
        "kc_reports_free": ([vp, u32], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _copy(ptr, n, dtype):
    if n == 0 or not ptr:
        return np.zeros(0, dtype=dtype)
    return np.frombuffer((C.c_char * (n * dtype.itemsize)).from_address(ptr), dtype=dtype).copy()


@dataclass
class Report:
    records: int
    launches_completed: int
    races: np.ndarray
    faults: np.ndarray
    tag: int = 0
    sites: Optional[np.ndarray] = None     # SITE_DTYPE, parallel to races

    def race_tuples(self) -> List[Tuple[int, ...]]:
        return [tuple(int(x) for x in r) for r in self.races]

    def race_sites(self) -> List[Tuple[int, int]]:
        """(w_pc, o_pc) per race (0xFFFFFFFF where not computed)."""
        if self.sites is None:
            return [(0xFFFFFFFF, 0xFFFFFFFF)] * len(self.races)
        return [(int(x["w_pc"]), int(x["o_pc"])) for x in self.sites]

    def fault_tuples(self) -> List[Tuple[int, ...]]:
        return [tuple(int(x) for x in f) for f in self.faults]


class ReportList(cabc.Sequence):
    """The reports of a polled batch, gathered with two library calls; a
    Report is built when an item is accessed.  `records`, `launches_completed`
    and `tags` are arrays over the batch."""

    def __init__(self, lib, ptrs, n: int):
        self.n = n
        u64, u32 = np.uint64, np.uint32
        self.records = np.zeros(n, u64)
        self.launches_completed = np.zeros(n, u32)
        self.tags = np.zeros(n, u64)
        nr = np.zeros(n, u64)
        nf = np.zeros(n, u64)
        p = lambda a: a.ctypes.data if a.size else None
        st = lib.kc_reports_collect(ptrs, n, p(self.records), p(self.launches_completed), p(self.tags), p(nr), p(nf),
                                    None, None, None)
        if st != KC_OK:
            raise KcError(st, "kc_reports_collect")
        self._races = np.zeros(int(nr.sum()), RACE_DTYPE)
        self._faults = np.zeros(int(nf.sum()), FAULT_DTYPE)
        self._sites = np.zeros(int(nr.sum()), SITE_DTYPE)
        st = lib.kc_reports_collect(ptrs, n, None, None, None, None, None, p(self._races), p(self._faults),
                                    p(self._sites))
        lib.kc_reports_free(ptrs, n)
        if st != KC_OK:
            raise KcError(st, "kc_reports_collect")
        self._roff = np.concatenate([[0], np.cumsum(nr)]).astype(np.int64)
        self._foff = np.concatenate([[0], np.cumsum(nf)]).astype(np.int64)

    def __len__(self) -> int:
        return self.n

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[j] for j in range(*i.indices(self.n))]
        if i < 0:
            i += self.n
        if not 0 <= i < self.n:
            raise IndexError(i)
        return Report(int(self.records[i]), int(self.launches_completed[i]),
                      self._races[self._roff[i]:self._roff[i + 1]].copy(),
                      self._faults[self._foff[i]:self._foff[i + 1]].copy(), int(self.tags[i]),
                      self._sites[self._roff[i]:self._roff[i + 1]].copy())

    def total_records(self) -> int:
        return int(self.records.sum())


def _take_report(lib, ptr) -> Report:
    n = C.c_uint64()
    races = _copy(lib.kc_report_races(ptr, C.byref(n)), n.value, RACE_DTYPE)
    sites = _copy(lib.kc_report_race_sites(ptr, C.byref(n)), n.value, SITE_DTYPE)
    faults = _copy(lib.kc_report_faults(ptr, C.byref(n)), n.value, FAULT_DTYPE)
    rep = Report(int(lib.kc_report_records(ptr)), int(lib.kc_report_launches_completed(ptr)), races, faults,
                 int(lib.kc_report_tag(ptr)), sites)
    lib.kc_report_free(ptr)
    return rep


class Context:
    """A libkc context on one HIP device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, tune_cache: Optional[str] = None):
        self.lib = load_library()
        h = C.c_void_p()
        st = self.lib.kc_ctx_create(device, hbm_budget_bytes, tune_cache.encode() if tune_cache else None,
                                    C.byref(h))
        if st != KC_OK:
            raise KcError(st, f"kc_ctx_create(device={device})")
        self.h = h
        self.device = device
        self._progs: Dict[bytes, Program] = {}

    def _check(self, st: int, what: str):
        if st != KC_OK:
            raise KcError(st, f"{what}: {self.lib.kc_last_error(self.h).decode(errors='replace')}")

    def set_option(self, key: str, value: int):
        self._check(self.lib.kc_ctx_set_option(self.h, key.encode(), int(value)), f"set_option({key})")

    def stat(self, key: str) -> float:
        return float(self.lib.kc_ctx_get_stat(self.h, key.encode()))

    def reset_stats(self):
        self.set_option("reset", 1)

    def program(self, words) -> "Program":
        arr = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
        key = arr.tobytes()
        p = self._progs.get(key)
        if p is None:
            p = Program(self, arr)
            self._progs[key] = p
        return p

    def close(self):
        if getattr(self, "h", None):
            for p in self._progs.values():
                p.free()
            self._progs.clear()
            self.lib.kc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Program:
    def __init__(self, ctx: Context, words: np.ndarray):
        self.ctx = ctx
        self.words = words
        h = C.c_void_p()
        ctx._check(ctx.lib.kc_program_load(ctx.h, words.ctypes.data, len(words), C.byref(h)), "kc_program_load")
        self.h = h

    def free(self):
        if self.h:
            self.ctx.lib.kc_program_free(self.h)
            self.h = None


def _desc(prog: Program, grid, block, shmem_bytes: int, params: Sequence[int]) -> LaunchDesc:
    d = LaunchDesc()
    d.prog = prog.h
    g = tuple(grid) + (1,) * (3 - len(tuple(grid)))
    b = tuple(block) + (1,) * (3 - len(tuple(block)))
    d.grid = Dim3(*g)
    d.block = Dim3(*b)
    d.shmem_bytes = shmem_bytes
    ps = [int(np.int32(p)) for p in params]
    if len(ps) > 8:
        raise ValueError("at most 8 params")
    d.params[:] = ps + [0] * (8 - len(ps))
    d.n_params = len(ps)
    return d


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def launch(ctx: Context, prog: Program, grid, block, shmem_bytes: int, mem, params: Sequence[int] = (),
           stream=None) -> Report:
    """One synchronous launch on ``mem`` (an int32 CUDA tensor, updated in place)."""
    return PreparedLaunch(ctx, prog, grid, block, shmem_bytes, params).run(mem, stream)


class PreparedLaunch:
    """kc_launch with its descriptor (program, grid, block, shared memory,
    parameters) marshalled once, for callers that run the same launch on
    memories again and again."""

    def __init__(self, ctx: Context, prog: Program, grid, block, shmem_bytes: int, params: Sequence[int] = ()):
        self.ctx = ctx
        self.prog = prog                # keeps the program alive while the descriptor points at it
        self.desc = _desc(prog, grid, block, shmem_bytes, params)
        self._dref = C.byref(self.desc)

    def run(self, mem, stream=None) -> Report:
        """Run on ``mem`` (a contiguous int32 CUDA tensor, updated in place)."""
        import torch
        if mem.dtype != torch.int32 or not mem.is_cuda or not mem.is_contiguous():
            raise ValueError("mem must be a contiguous int32 tensor on the GPU")
        out = C.c_void_p()
        self.ctx._check(self.ctx.lib.kc_launch(self.ctx.h, self._dref, mem.data_ptr(), mem.numel(),
                                               _stream_handle(stream), C.byref(out)), "kc_launch")
        return _take_report(self.ctx.lib, out)


def launch_noalloc(ctx: Context, prog: Program, grid, block, shmem_bytes: int, mem, params: Sequence[int] = (),
                   stream=None) -> Report:
    """kc_launch_noalloc: the same launch as ``launch``, with every device
    buffer carved from the library's static scratch area (no allocation)."""
    import torch
    if mem.dtype != torch.int32 or not mem.is_cuda or not mem.is_contiguous():
        raise ValueError("mem must be a contiguous int32 tensor on the GPU")
    d = _desc(prog, grid, block, shmem_bytes, params)
    out = C.c_void_p()
    ctx._check(ctx.lib.kc_launch_noalloc(ctx.h, C.byref(d), mem.data_ptr(), mem.numel(), _stream_handle(stream),
                                         C.byref(out)), "kc_launch_noalloc")
    return _take_report(ctx.lib, out)


@dataclass
class Prepared:
    jd: object
    keep: list
    n: int
    mems: list


class Batch:
    """Asynchronous batches of jobs (each job = launches in order on one memory)."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self._keep: Dict[int, tuple] = {}

    def prepare(self, jobs) -> "Prepared":
        """Marshal jobs into C descriptors once (reusable by several submits)."""
        n = len(jobs)
        jd = (JobDesc * max(n, 1))()
        keep = []
        for i, item in enumerate(jobs):
            launches, mem, tag = item[:3]
            streams = item[3] if len(item) > 3 else None
            deps = item[4] if len(item) > 4 else ()
            allocs = item[5] if len(item) > 5 else None
            steps = item[6] if len(item) > 6 else None
            arr = (LaunchDesc * max(len(launches), 1))()
            for j, (p, g, b, sh, ps) in enumerate(launches):
                arr[j] = _desc(p, g, b, sh, ps)
            keep.append(arr)
            jd[i].launches = C.cast(arr, C.POINTER(LaunchDesc))
            jd[i].n_launches = len(launches)
            if isinstance(mem, int):           # a word count: no memory yet (kc_batch_footprint)
                jd[i].dev_mem, jd[i].n_words = None, mem
            else:
                jd[i].dev_mem = mem.data_ptr()
                jd[i].n_words = mem.numel()
            jd[i].tag = tag
            if streams is not None:
                if len(streams) != len(launches):
                    raise ValueError("one stream per launch")
                sarr = (C.c_uint32 * max(len(streams), 1))(*[int(x) for x in streams])
                keep.append(sarr)
                jd[i].streams = C.cast(sarr, C.POINTER(C.c_uint32))
            if len(deps):
                darr = (Dep * len(deps))(*[Dep(int(a), int(b)) for a, b in deps])
                keep.append(darr)
                jd[i].deps = C.cast(darr, C.POINTER(Dep))
                jd[i].n_deps = len(deps)
            if allocs is not None:
                rarr = (Region * max(len(allocs), 1))(*[Region(int(b), int(w)) for b, w in allocs])
                keep.append(rarr)
                jd[i].allocs = C.cast(rarr, C.POINTER(Region))
                jd[i].n_allocs = len(allocs)
            if steps is not None:
                iarr = (ItemDesc * max(len(steps), 1))(*[_item_desc(x) for x in steps])
                keep.append(iarr)
                jd[i].items = C.cast(iarr, C.POINTER(ItemDesc))
                jd[i].n_items = len(steps)
        return Prepared(jd, keep, n, [item[1] for item in jobs])

    def submit(self, jobs, stream=None) -> int:
        """jobs: a Prepared batch or a list of (launches, mem_tensor, tag) or
        (launches, mem_tensor, tag, streams, deps[, allocs[, items]]) with launches =
        [(prog, grid, block, shmem, params), ...], streams one stream id per
        launch (or None), deps (before, after) launch pairs, allocs the
        device allocations as (base, words) ranges (or None: no check) and
        items the host program (objects with workloads.Item's fields, or
        None: the launches in order)."""
        prep = jobs if isinstance(jobs, Prepared) else self.prepare(jobs)
        t = C.c_uint64()
        self.ctx._check(self.ctx.lib.kc_batch_submit(self.ctx.h, prep.jd, prep.n, _stream_handle(stream),
                                                     C.byref(t)), "kc_batch_submit")
        self._keep[t.value] = (prep.jd, prep.keep, prep.n, prep.mems)
        return t.value

    def footprint(self, jobs) -> int:
        """kc_batch_footprint: the device bytes the library would reserve to
        run ``jobs`` (a Prepared batch or items as for ``submit``; a memory
        may be given as its word count) as one batch."""
        prep = jobs if isinstance(jobs, Prepared) else self.prepare(jobs)
        b = C.c_uint64()
        self.ctx._check(self.ctx.lib.kc_batch_footprint(self.ctx.h, prep.jd, prep.n, C.byref(b)),
                        "kc_batch_footprint")
        return int(b.value)

    def poll(self, ticket: int, wait: bool = True) -> Optional[List[Report]]:
        n = self._keep[ticket][2]
        out = (C.c_void_p * max(n, 1))()
        st = self.ctx.lib.kc_poll(self.ctx.h, ticket, int(wait), out, n)
        if st == KC_E_PENDING:
            return None
        self._keep.pop(ticket, None)
        self.ctx._check(st, "kc_poll")
        return ReportList(self.ctx.lib, out, n)


# ---------------------------------------------------------------------------
# convenience over workload jobs (objects with .launches and .memory)
# ---------------------------------------------------------------------------
def job_launches(ctx: Context, job) -> list:
    return [(ctx.program(L.program), L.grid, L.block, L.shmem_bytes, L.params) for L in job.launches]


def job_item(ctx: Context, job, mem, tag):
    return (job_launches(ctx, job), mem, tag, getattr(job, "streams", None), getattr(job, "deps", None) or (),
            getattr(job, "allocs", None), getattr(job, "items", None))


def jobs_footprint(ctx: Context, jobs) -> int:
    """Device bytes the library would reserve to run workload ``jobs`` as one
    batch (their memories need not be on the GPU)."""
    return Batch(ctx).footprint([job_item(ctx, j, len(j.memory), i) for i, j in enumerate(jobs)])


def run_job(ctx: Context, job, mem=None, stream=None):
    """Run all launches of ``job`` as one job; returns (Report, final memory tensor)."""
    import torch
    if mem is None:
        mem = torch.from_numpy(np.ascontiguousarray(job.memory, dtype=np.int32)).to(f"cuda:{ctx.device}")
    b = Batch(ctx)
    t = b.submit([job_item(ctx, job, mem, 0)], stream=stream)
    return b.poll(t, wait=True)[0], mem


def run_jobs(ctx: Context, jobs, mems=None, stream=None):
    """Run many jobs as one batch; returns (reports, memories)."""
    import torch
    if mems is None:
        mems = [torch.from_numpy(np.ascontiguousarray(j.memory, dtype=np.int32)).to(f"cuda:{ctx.device}")
                for j in jobs]
    b = Batch(ctx)
    t = b.submit([job_item(ctx, j, m, i) for i, (j, m) in enumerate(zip(jobs, mems))], stream=stream)
    return b.poll(t, wait=True), mems
