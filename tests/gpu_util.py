"""Helpers of the GPU parity tests: run a job through the library and compare
it element by element with the CPU oracle."""
import sys

import numpy as np

from oracle import oracle as O
from paper_1211_6193_amd import kc


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def assert_same(rep, mem, orc, what=""):
    assert rep.records == orc.records, (what, "records", rep.records, orc.records)
    assert rep.launches_completed == orc.launches_completed, (what, "launches", rep.launches_completed,
                                                              orc.launches_completed)
    assert rep.race_tuples() == orc.race_tuples(), (what, "races", rep.race_tuples()[:8], orc.race_tuples()[:8])
    assert rep.fault_tuples() == orc.fault_tuples(), (what, "faults", rep.fault_tuples()[:8],
                                                      orc.fault_tuples()[:8])
    got = mem.cpu().numpy() if hasattr(mem, "cpu") else np.asarray(mem)
    if not np.array_equal(got, orc.memory):
        bad = np.nonzero(got != orc.memory)[0]
        raise AssertionError((what, "memory differs at", bad[:10].tolist(), got[bad[:10]].tolist(),
                              orc.memory[bad[:10]].tolist()))


def check_jobs(ctx, jobs, fuel=O.DEFAULT_FUEL, label="batch"):
    say(f"{label}: {len(jobs)} jobs batched")
    reps, mems = kc.run_jobs(ctx, jobs)
    for i, (j, r, m) in enumerate(zip(jobs, reps, mems)):
        orc = O.run_job(j, fuel=fuel)
        assert_same(r, m, orc, f"{label}[{i}] {j.meta}")
    return reps
