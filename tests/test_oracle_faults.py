"""Pin the oracle with closed-form ground truth of injected faults and with the
plain outputs of race-free kernels (numpy sums, stencils, transposes).

Race tuples are (launch, space, scope, block, epoch, addr, w, o); space 0 is
shared memory, scope 0 intra-block.  Level k of a tree over P/2 = s_0 folds
s_k = s_0 >> k; level k runs in epoch k+1 (epoch 0 is the load phase).
"""
from collections import Counter

import numpy as np
import pytest

from oracle import oracle as O
from paper_1211_6193_amd import workloads as W
from paper_1211_6193_amd.ir import pcs_of


def _tree_tables_job(n_blocks, threads, drops=(), divs=(), seed=5):
    job = W.tree256_job(n_blocks=n_blocks, threads=threads, drop_frac=0.0, div_frac=0.0, seed=seed)
    n = job.meta["n"]
    for b, k in drops:
        job.memory[n + n_blocks + b] = k
    for b, j in divs:
        job.memory[n + 2 * n_blocks + b] = j
    return job


@pytest.mark.parametrize("threads", [32, 64, 256])
def test_tree_dropped_barrier_races_closed_form(threads):
    L = threads.bit_length() - 1
    nb = L + 1
    drops = [(k, k) for k in range(L)]            # block k drops the barrier after level k
    job = _tree_tables_job(nb, threads, drops=drops)
    r = O.run_job(job)
    s0 = threads // 2
    want = []
    for b, k in drops:
        sk = s0 >> k
        if sk >= 2:                               # the last level has no successor to race with
            want += [(0, 0, 0, b, k + 1, a, a, a - sk // 2) for a in range(sk // 2, sk)]
    assert r.race_tuples() == sorted(want, key=lambda t: (t[0], t[1], t[2], t[3], t[4], t[5]))
    n = job.meta["n"]
    sums = job.memory[:n].astype(np.int64).reshape(nb, threads).sum(1)
    # under lockstep the folding threads stay aligned, so the sum is still right
    assert r.memory[n:n + nb].tolist() == sums.tolist()
    assert len(r.faults) == 0 and r.launches_completed == 1


@pytest.mark.parametrize("j", [0, 2, 4])
def test_tree_tid_barrier_divergence_then_deadlock(j):
    threads, nb = 32, 3
    L = 5
    job = _tree_tables_job(nb, threads, divs=[(1, j)])
    r = O.run_job(job)
    prog = job.launches[0].program
    bars = pcs_of(prog, "BAR")
    extra, regular = bars[1], bars[2]
    sj = (threads // 2) >> j
    # threads < s_j wait at the extra barrier, the rest at the regular one
    # (epoch j+1); afterwards both groups meet at the same barrier instruction
    # one iteration apart, so no further divergence; after L+1 episodes the
    # leading group exits while the lagging one waits -> deadlock.
    want = [(0, O.F_DIVERGENCE, 1, j + 1, extra, 0, regular, sj),
            (0, O.F_DEADLOCK, 1, L + 1, sj, 0, sj, 0)]
    assert sorted(r.fault_tuples(), key=lambda f: (f[0], f[2], f[3], f[1])) == \
        sorted(want, key=lambda f: (f[0], f[2], f[3], f[1]))
    assert r.launches_completed == 0
    n = job.meta["n"]
    sums = job.memory[:n].astype(np.int64).reshape(nb, threads).sum(1)
    out = r.memory[n:n + nb]
    assert out[0] == sums[0] and out[2] == sums[2] and out[1] == 0
    assert len(r.races) == 0


def _stencil_ref(x):
    xp = np.concatenate([[0], x.astype(np.int64), [0]])
    return ((xp[:-2] + 2 * xp[1:-1] + xp[2:]) >> 2).astype(np.int32)


def _transpose_ref(x, nb):
    return x.reshape(32, 32 * nb).T.reshape(-1)


def _race_free_outputs(job, r):
    m = job.meta
    n, o = m["n"], m["out_base"]
    x = job.memory[:n]
    if m["family"] == "TREE":
        return r.memory[o:o + m["n_blocks"]].tolist() == \
            x.astype(np.int64).reshape(m["n_blocks"], m["threads"]).sum(1).tolist()
    if m["family"] == "STENCIL":
        return r.memory[o:o + n].tolist() == _stencil_ref(x).tolist()
    return r.memory[o:o + n].tolist() == _transpose_ref(x, m["n_blocks"]).tolist()


@pytest.mark.parametrize("family", W.FAMILIES)
@pytest.mark.parametrize("nb,threads", [(1, 32), (3, 96), (2, 256), (5, 64)])
def test_clean_families_equal_numpy(family, nb, threads):
    rng = np.random.default_rng(nb * 1000 + threads)
    job = W.family_job(family, nb, threads, rng)
    r = O.run_job(job)
    assert len(r.races) == 0 and len(r.faults) == 0 and r.launches_completed == 1
    assert _race_free_outputs(job, r)


def _key(t):
    return t[:6]


@pytest.mark.parametrize("threads", [32, 96, 1024])
def test_stencil_fault_ground_truth(threads):
    T = threads
    fb = 1
    rng = np.random.default_rng(T)
    cases = {
        "drop": [(0, 0, 0, fb, 0, 1, 0, 1)] + [(0, 0, 0, fb, 0, a, a - 1, a - 2) for a in range(2, T + 1)],
        "halo": [(0, 0, 0, fb, 0, T, T - 2, T - 1)],
        "double": [(0, 0, 0, fb, 0, 1, 0, 1)],
    }
    for fault, want in cases.items():
        job = W.family_job("STENCIL", 3, T, rng, fault, fb)
        r = O.run_job(job)
        assert r.race_tuples() == sorted(want, key=_key), fault
        assert len(r.faults) == 0


@pytest.mark.parametrize("threads", [32, 128, 1024])
def test_transpose_fault_ground_truth(threads):
    T = threads
    step = T // 32
    fb = 2
    rng = np.random.default_rng(T + 1)
    # dropped barrier: sh[R*33+C] is written by tid (R%step)*32+C and read by
    # tid (C%step)*32+R in the same epoch; equal only when R == C.
    drop = [(0, 0, 0, fb, 0, R * 33 + C, (R % step) * 32 + C, (C % step) * 32 + R)
            for R in range(32) for C in range(32) if R != C]
    # thread 1 stores its rows into column 0 (thread 0's column)
    double = [(0, 0, 0, fb, 0, R * 33, 0, 1) for R in range(0, 32, step)]
    for fault, want in (("drop", drop), ("double", double)):
        job = W.family_job("TRANSPOSE", 3, T, rng, fault, fb)
        r = O.run_job(job)
        assert r.race_tuples() == sorted(want, key=_key), fault
        assert len(r.faults) == 0


@pytest.mark.parametrize("family", W.FAMILIES)
def test_tidbar_first_divergence(family):
    T, nb, fb = 64, 3, 1
    job = W.family_job(family, nb, T, np.random.default_rng(3), "tidbar", fb)
    r = O.run_job(job)
    bars = pcs_of(job.launches[0].program, "BAR")
    divs = [f for f in r.fault_tuples() if f[1] == O.F_DIVERGENCE]
    dead = [f for f in r.fault_tuples() if f[1] == O.F_DEADLOCK]
    if family == "TREE":
        first = (0, O.F_DIVERGENCE, fb, 1, bars[1], 0, bars[2], T // 2)
    else:
        first = (0, O.F_DIVERGENCE, fb, 0, bars[0], 0, bars[1], T // 2)
    assert divs[0] == first
    assert len(dead) == 1 and dead[0][2] == fb and dead[0][4] == T // 2 and dead[0][5] == 0
    assert r.launches_completed == 0


def test_pingpong_inplace_bug_cross_block_races():
    job = W.stencil_pingpong_job(n=64 * 32, threads=32, steps=2, bug_frac=0.0, seed=1)
    n, T = job.meta["n"], 32
    bug = 5
    job.memory[2 * n + bug] = 1
    r = O.run_job(job)
    g0 = bug * T
    # step 0 reads A and the buggy block writes A[g0 .. g0+T): block bug-1's
    # right-halo loader (tid T-1) reads A[g0], block bug+1's left-halo loader
    # (tid 0) reads A[g0+T-1].
    want0 = [(0, 1, 1, bug, 0xFFFFFFFF, g0, g0, (bug - 1) * T + T - 1),
             (0, 1, 1, bug, 0xFFFFFFFF, g0 + T - 1, g0 + T - 1, (bug + 1) * T)]
    got0 = [t for t in r.race_tuples() if t[0] == 0]
    assert got0 == want0
    assert r.launches_completed == 2


def test_records_permutation_free_definition():
    """Races equal a pairwise evaluation of the definition over the oracle's own records."""
    rng = np.random.default_rng(9)
    jobs = [W.fig1_job("NOBAR14"), W.family_job("STENCIL", 2, 32, rng, "drop", 0),
            W.family_job("TRANSPOSE", 2, 64, rng, "double", 1),
            W.stencil_pingpong_job(n=8 * 32, threads=32, steps=1, bug_frac=0.0, seed=2)]
    jobs[-1].memory[2 * 256 + 3] = 1
    for job in jobs:
        r = O.run_job(job, keep_records=True)
        nt = job.launches[0].n_threads
        recs = r.record_log
        segs = {}
        for x in recs:
            L, sp, ad, bl, ep, ti, ki, pc = (int(v) for v in tuple(x)[:8])
            segs.setdefault((L, sp, 0, bl, ep, ad), []).append((ti, ki, pc))
            if sp == 1:
                segs.setdefault((L, sp, 1, ad), []).append((bl * nt + ti, ki, bl, pc))
        want, sites = [], {}
        for key, rs in segs.items():
            if key[2] == 0:
                pairs = [(a, b) for a in rs for b in rs if a[0] != b[0] and (a[1] or b[1])]
                if pairs:
                    w = min(t for t, k, _ in rs if k == 1)
                    o = min(t for t, k, _ in rs if t != w)      # every other tid conflicts with w
                    want.append(key + (w, o))
                    # source sites: w's first store site and o's first access site by pc
                    sites[want[-1]] = (min(p for t, k, p in rs if t == w and k == 1), min(p for t, _, p in rs if t == o))
            else:
                pairs = [(a, b) for a in rs for b in rs if a[2] != b[2] and (a[1] or b[1])]
                if pairs:
                    w, wb = min((g, b) for g, k, b, _ in rs if k == 1)
                    o = min(g for g, k, b, _ in rs if b != wb)
                    want.append((key[0], 1, 1, wb, 0xFFFFFFFF, key[3], w, o))
                    sites[want[-1]] = (min(p for g, k, _, p in rs if g == w and k == 1),
                                       min(p for g, _, _, p in rs if g == o))
        assert r.race_tuples() == sorted(want, key=_key)
        assert r.race_sites() == [sites[t] for t in r.race_tuples()]
