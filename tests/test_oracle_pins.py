"""Pins of the CPU oracle against what the paper and the mathematics fix.

* Figure 1 run (Section 3.2): inputs and OUTPUT 767, also for the variant
  without the second barrier (the paper reports the race and the same output).
* Hand derivation of the access records, races and findings of the three
  Figure-1 variants (worked out below from the kernel text).
* Closed form of the kernel's own sum for odd block sizes.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1211_6193_amd import workloads as W
from paper_1211_6193_amd.ir import pcs_of

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig1_paper_run.txt")


def _golden():
    vals = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split(":", 1)
        vals[k.strip()] = [int(x) for x in v.split()]
    return vals


def test_fig1_inputs_match_paper():
    assert W.PAPER_INPUT == _golden()["INPUT"]


def test_fig1_base_output_767():
    g = _golden()
    r = O.run_job(W.fig1_job("BASE"))
    assert int(r.memory[18]) == g["OUTPUT"][0] == 767
    assert r.launches_completed == 2
    assert len(r.races) == 0 and len(r.faults) == 0


def test_fig1_nobar14_output_and_races():
    g = _golden()
    r = O.run_job(W.fig1_job("NOBAR14"))
    assert int(r.memory[18]) == g["OUTPUT_NOBAR14"][0] == 767
    # Hand derivation: after the first barrier (epoch 1) threads 1..3 write
    # shared[tid] in the fold while thread 0's loop (line 17) reads shared[1..4];
    # no barrier separates them.  shared[4] is only read, shared[0] only touched
    # by thread 0.  Tuple: (launch, space, scope, block, epoch, addr, w, o).
    expect = [(0, 0, 0, b, 1, a, a, 0) for b in (0, 1) for a in (1, 2, 3)]
    assert r.race_tuples() == expect
    assert r.records == 97


def test_fig1_base_records_97():
    # per block of 9 threads: 9 LDG + 9 STS + 4 fold threads x 3 + 4 loop
    # iterations x 3 + final LDS + STG = 44; launch 0 has 2 blocks; launch 1
    # (2 threads): 2 + 2 + 1 x 3 + 0 + 2 = 9.  Total 97.
    r = O.run_job(W.fig1_job("BASE"))
    assert r.records == 2 * 44 + 9


def test_fig1_bar11_divergence_then_deadlock():
    p = W.sum_program("BAR11")
    bars = pcs_of(p, "BAR")
    inner, line14 = bars[1], bars[2]
    r = O.run_job(W.fig1_job("BAR11", out_init=(-5, -7)))
    # Both blocks of launch 0: threads 0..3 wait at the inserted barrier,
    # 4..8 at line 14 -> all wait at different sites (divergence, epoch 1);
    # then 4..8 exit while 0..3 wait at line 14 -> deadlock in epoch 2.
    expect = []
    for b in (0, 1):
        expect.append((0, O.F_DEADLOCK, b, 2, 4, 0, 4, 0))
        expect.append((0, O.F_DIVERGENCE, b, 1, inner, 0, line14, 4))
    expect.sort(key=lambda f: (f[0], f[2], f[3], f[1], f[4], f[5], f[6], f[7]))
    assert r.fault_tuples() == expect
    assert r.launches_completed == 0
    assert r.memory[18:20].tolist() == [-5, -7]     # out untouched, launch 1 never ran
    assert r.records == 2 * (18 + 12)
    assert len(r.races) == 0


@pytest.mark.parametrize("seed", range(5))
def test_fig1_closed_form_seeded(seed):
    # For odd bdim = 2h+1 the kernel folds s[t] += s[h+t] for t<h, then thread
    # 0 sums s[0..h]: the result is sum_{j<2h} s_j + s_h (s_{2h} is dropped and
    # s_h counted twice).  Launch 1 (2 threads) adds the two partials.
    rng = np.random.default_rng(1000 + seed)
    x = rng.integers(0, 100, 18)
    r = O.run_job(W.fig1_job("BASE", x.tolist()))
    parts = [int(x[9 * b:9 * b + 8].sum() + x[9 * b + 4]) for b in (0, 1)]
    assert r.memory[19] == parts[1]
    assert r.memory[18] == parts[0] + parts[1]
    assert r.memory[:18].tolist() == x.tolist()


def test_paper_partials():
    r = O.run_job(W.fig1_job("BASE"))
    assert r.memory[19] == 334
    # launch 0 partials before launch 1 combines them: run launch 0 alone
    j = W.fig1_job("BASE")
    j.launches = j.launches[:1]
    r0 = O.run_job(j)
    assert r0.memory[18:20].tolist() == [433, 334]
