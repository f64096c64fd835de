"""Writes workload4_2p25_oracle.json: the oracle's result on the ping-pong
stencil at 2^25 elements over two launches (blocks of 256 threads, bug
fraction 1e-4, seed 12116197) -- record count, completed launches, race and
finding tuples, and a SHA-256 of the final memory.  The oracle needs several
minutes for this job, longer than a GPU test may stay quiet, so the GPU test
compares against this file.  Calls nothing but the oracle and the seeded input
generator.  Run from the repository root:

    python tests/golden/make_workload4_digest.py
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O                     # noqa: E402
from paper_1211_6193_amd import workloads as W     # noqa: E402

SPEC = dict(n=1 << 25, threads=256, steps=2, bug_frac=0.0001, seed=12116197)


def memory_digest(mem):
    return hashlib.sha256(mem.astype("<i4").tobytes()).hexdigest()


def main():
    job = W.stencil_pingpong_job(**SPEC)
    orc = O.run_job(job)
    out = dict(spec=SPEC, input_sha256=memory_digest(job.memory), records=orc.records,
               launches_completed=orc.launches_completed,
               races=[list(t) for t in orc.race_tuples()], faults=[list(t) for t in orc.fault_tuples()],
               memory_sha256=memory_digest(orc.memory))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workload4_2p25_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(path, orc.records, len(out["races"]), len(out["faults"]))


if __name__ == "__main__":
    main()
