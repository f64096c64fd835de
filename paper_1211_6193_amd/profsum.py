"""Summaries of rocprofv3 result databases (SQLite) as short text.

    python -m paper_1211_6193_amd.profsum kernels DB TITLE COMMAND
        markdown table of the kernel-trace statistics (calls, total, average)
    python -m paper_1211_6193_amd.profsum dispatches DB NAME[,NAME...]
        per kernel name and launch shape: dispatch count, mean/min/max duration
    python -m paper_1211_6193_amd.profsum counters DB
        per kernel name: dispatches and the mean of each PMC counter per dispatch
    python -m paper_1211_6193_amd.profsum counters_by_grid DB [NAME]
        the same per kernel name and launch shape (grid work-items, workgroup size)
    python -m paper_1211_6193_amd.profsum traffic FETCH_DB WRITE_DB COPY_FETCH_DB COPY_WRITE_DB KERNEL OUT.json
        HBM bytes per dispatch of KERNEL from FETCH_SIZE and WRITE_SIZE passes,
        each scaled by what the same counter reads for a device copy of a
        known 1 GiB (the copy-calibration mode of bench.py), written as JSON
        with a digest of the interpreter sources it was measured on.
    python -m paper_1211_6193_amd.profsum timeline DB ANCHOR [STEPS]
        the GPU timeline of the last STEPS (default 2) intervals that start at
        a dispatch of kernel ANCHOR: each kernel and memory copy with its start
        offset, duration and the idle gap before it (needs a trace taken with
        --kernel-trace --memory-copy-trace).
"""
from __future__ import annotations

import collections
import hashlib
import json
import os
import sqlite3
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
COPY_BYTES = 1 << 30


HOST_SECTION = b"#ifndef __HIPCC_RTC__\n// ---- host side"


def kernel_source_digest() -> str:
    """Digest of the sources of the free-run kernels (interpreter and
    program-specialised): the device code, and the shared header up to its
    host-only section (declarations the kernels never see)."""
    h = hashlib.sha256()
    for f in ("kc_internal.h", "kc_device.h", "kc_interp.hip", "kc_jit.hip"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            text = fh.read()
        if f == "kc_internal.h" and HOST_SECTION in text:
            text = text[:text.index(HOST_SECTION)]
        h.update(text)
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    return name.replace("kc::(anonymous namespace)::", "").replace("void ", "").split("(")[0][:100]


def kernels(db: str, title: str, cmd: str) -> str:
    c = sqlite3.connect(db)
    # top_kernels reports durations in microseconds
    rows = c.execute("select name,total_calls,total_duration,average,percentage from top_kernels").fetchall()
    out = [f"# {title}", "", "Command:", "", "```", cmd, "```", "",
           "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for n, calls, tot, avg, pct in rows:
        out.append(f"| `{_short(n)}` | {calls} | {tot / 1e3:.3f} | {avg:.2f} | {pct:.1f} |")
    return "\n".join(out)


def dispatches(db: str, like: str) -> str:
    c = sqlite3.connect(db)
    try:
        rows = c.execute("select name, duration, grid_x, workgroup_x from kernels where name like ?",
                         (f"%{like}%",)).fetchall()
    except sqlite3.Error as e:
        cols = [r[1] for r in c.execute("pragma table_info(kernels)")]
        return f"kernels view columns: {cols} ({e})"
    by = collections.defaultdict(list)
    for n, d, g, w in rows:
        by[(_short(n), g, w)].append(d / 1e3)
    out = []
    for (n, g, w), ds in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        ds.sort()
        out.append(f"{n} grid={g} wg={w} n={len(ds)} avg_us={sum(ds) / len(ds):.1f} "
                   f"min_us={ds[0]:.1f} max_us={ds[-1]:.1f}")
    return "\n".join(out)


def counter_means(db: str):
    """{kernel name: (dispatches, {counter: mean per dispatch})}"""
    c = sqlite3.connect(db)
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    nd = collections.defaultdict(set)
    for name, did, cn, cv in c.execute("select name, dispatch_id, counter_name, counter_value from pmc_events"):
        agg[name][cn] += cv
        nd[name].add(did)
    return {n: (len(nd[n]), {k: v / len(nd[n]) for k, v in agg[n].items()}) for n in agg}


def counter_means_by_grid(db: str):
    """{(kernel name, grid work-items, workgroup size): (dispatches, {counter: mean per dispatch})}"""
    c = sqlite3.connect(db)
    shape = {did: (g, w) for did, g, w in c.execute("select dispatch_id, grid_x, workgroup_x from kernels")}
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    nd = collections.defaultdict(set)
    for name, did, cn, cv in c.execute("select name, dispatch_id, counter_name, counter_value from pmc_events"):
        key = (name,) + shape.get(did, (0, 0))
        agg[key][cn] += cv
        nd[key].add(did)
    return {k: (len(nd[k]), {n: v / len(nd[k]) for n, v in agg[k].items()}) for k in agg}


def counters_by_grid(db: str, like: str = "") -> str:
    out = []
    for (n, g, w), (d, m) in sorted(counter_means_by_grid(db).items(), key=lambda kv: -sum(kv[1][1].values())):
        if like and like not in n:
            continue
        out.append(f"{_short(n)}\tgrid={g}\twg={w}\tdispatches={d}\t" +
                   "\t".join(f"{k}={v:.6g}" for k, v in sorted(m.items())))
    return "\n".join(out)


def counters(db: str) -> str:
    out = []
    for n, (d, m) in sorted(counter_means(db).items(), key=lambda kv: -sum(kv[1][1].values())):
        out.append(f"{_short(n)}\tdispatches={d}\t" + "\t".join(f"{k}={v:.6g}" for k, v in sorted(m.items())))
    return "\n".join(out)


def _pick(means, like: str, counter: str):
    hits = [(m[counter], n) for n, (d, m) in means.items() if like in n and counter in m]
    if not hits:
        raise SystemExit(f"no kernel matching {like!r} with counter {counter} in the database")
    return max(hits)


def traffic(fetch_db, write_db, copy_fetch_db, copy_write_db, kernel, out_path):
    f_kib, name = _pick(counter_means(fetch_db), kernel, "FETCH_SIZE")
    w_kib, _ = _pick(counter_means(write_db), kernel, "WRITE_SIZE")
    cf_kib, copy_name = _pick(counter_means(copy_fetch_db), "copy", "FETCH_SIZE")
    cw_kib, _ = _pick(counter_means(copy_write_db), "copy", "WRITE_SIZE")
    f_scale = COPY_BYTES / (cf_kib * 1024.0)
    w_scale = COPY_BYTES / (cw_kib * 1024.0)
    fetch_b = f_kib * 1024.0 * f_scale
    write_b = w_kib * 1024.0 * w_scale
    res = {"kernel": _short(name), "fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib,
           "copy_kernel": _short(copy_name), "copy_fetch_kib": cf_kib, "copy_write_kib": cw_kib,
           "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
           "bytes_per_launch": int(fetch_b + write_b), "fetch_bytes": int(fetch_b), "write_bytes": int(write_b),
           "source_digest": kernel_source_digest()}
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    return json.dumps(res)


def _events(c):
    """(start ns, end ns, label) of every kernel dispatch and memory copy."""
    ev = [(s, e, _short(n)) for s, e, n in c.execute("select start, end, name from kernels")]
    try:
        cols = [r[1] for r in c.execute("pragma table_info(memory_copies)")]
        label = "name" if "name" in cols else ("kind" if "kind" in cols else None)
        q = f"select start, end, {label or 'NULL'}, size from memory_copies" if "size" in cols else \
            f"select start, end, {label or 'NULL'}, 0 from memory_copies"
        for s, e, n, b in c.execute(q):
            ev.append((s, e, f"copy {n or ''} {b} B".replace("  ", " ")))
    except sqlite3.Error:
        pass
    return sorted(ev)


def timeline(db: str, anchor: str, steps: int = 2) -> str:
    c = sqlite3.connect(db)
    ev = _events(c)
    starts = [i for i, (_, _, n) in enumerate(ev) if anchor in n]
    if not starts:
        return f"no dispatch of {anchor!r}"
    out = []
    sel = starts[-steps - 1:]
    for a, b in zip(sel[:-1], sel[1:]):
        t0 = ev[a][0]
        busy = 0
        prev_end = t0
        out.append(f"-- interval of {(ev[b][0] - t0) / 1e3:.1f} us")
        out.append("offset_us  dur_us  gap_us  event")
        for s, e, n in ev[a:b]:
            gap = max(0, s - prev_end)
            busy += max(0, e - max(s, prev_end))
            out.append(f"{(s - t0) / 1e3:9.1f} {(e - s) / 1e3:7.1f} {gap / 1e3:7.1f}  {n}")
            prev_end = max(prev_end, e)
        out.append(f"busy {busy / 1e3:.1f} us, idle {(ev[b][0] - t0 - busy) / 1e3:.1f} us")
    return "\n".join(out)


def main(argv):
    mode = argv[1]
    if mode == "kernels":
        print(kernels(argv[2], argv[3], argv[4]))
    elif mode == "dispatches":
        for like in argv[3].split(","):
            print(dispatches(argv[2], like))
    elif mode == "counters":
        print(counters(argv[2]))
    elif mode == "counters_by_grid":
        print(counters_by_grid(argv[2], argv[3] if len(argv) > 3 else ""))
    elif mode == "timeline":
        print(timeline(argv[2], argv[3], int(argv[4]) if len(argv) > 4 else 2))
    elif mode == "traffic":
        print(traffic(*argv[2:8]))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv)
