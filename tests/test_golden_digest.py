"""The stored digest of the oracle's result on workload 4 at 2^25 elements
(used by the GPU test, where the oracle would take minutes) still matches the
seeded input generator, and its race tuples equal the closed form: exactly
the two boundary words of every buggy block's range in the array each launch
reads, with the neighbouring halo loader as the other thread."""
import json
import os
import sys

from paper_1211_6193_amd import workloads as W

HERE = os.path.dirname(__file__)
sys.path.insert(0, os.path.join(HERE, "golden"))
from make_workload4_digest import memory_digest  # noqa: E402


def _closed_form(n, T, steps, bugs):
    nb = n // T
    want = []
    for s in range(steps):
        for b in sorted(bugs):
            g0 = b * T
            if b > 0:
                want.append([s, 1, 1, b, 0xFFFFFFFF, g0 + (n if s % 2 else 0), g0, (b - 1) * T + T - 1])
            if b < nb - 1:
                want.append([s, 1, 1, b, 0xFFFFFFFF, g0 + T - 1 + (n if s % 2 else 0), g0 + T - 1, (b + 1) * T])
    return sorted(want, key=lambda t: t[:6])


def test_workload4_digest_matches_generator_and_closed_form():
    with open(os.path.join(HERE, "golden", "workload4_2p25_oracle.json")) as f:
        d = json.load(f)
    job = W.stencil_pingpong_job(**d["spec"])
    assert memory_digest(job.memory) == d["input_sha256"]
    n, T, steps = job.meta["n"], job.meta["threads"], job.meta["steps"]
    assert d["launches_completed"] == steps and d["faults"] == []
    assert d["records"] == steps * (7 * n + 4 * (n // T) - 2)
    assert d["races"] == _closed_form(n, T, steps, [int(b) for b in job.meta["bug_blocks"]])
