"""Pin the source sites of race tuples (w_pc: the smallest pc of the writer's
stores to the location, o_pc: the smallest pc of the other thread's accesses
to it).  For the racy variant of Figure 1 (the barrier of line 14 removed)
the paper's tool names line 17 of the figure as the place of the race
(Section 3.2): thread 0's read of shared[i] in the serial loop, against the
stores of line 12.  The recomputation of the sites from the
oracle's records is in test_oracle_faults.py."""
from oracle import oracle as O
from paper_1211_6193_amd import workloads as W


def _find(prog, op, a=None, b=None):
    hits = [pc for pc, w in enumerate(int(x) for x in prog)
            if w & 0xFF == op and (a is None or (w >> 16) & 0xFF == a) and (b is None or (w >> 24) & 0xFF == b)]
    assert len(hits) == 1, hits
    return hits[0]


def test_figure1_race_detected_at_line_17():
    job = W.fig1_job("NOBAR14")
    prog = job.launches[0].program
    line17_read = _find(prog, 0x50, a=13)           # LDS r11, [r13]: shared[i] in the loop of line 17
    line12_store = _find(prog, 0x51, a=0, b=10)      # STS [r0], r10: shared[tid] += ... of line 12
    res = O.run_job(job)
    assert len(res.races) == 6
    for t, (w_pc, o_pc) in zip(res.race_tuples(), res.race_sites()):
        assert t[6] in (1, 2, 3) and t[7] == 0
        assert (w_pc, o_pc) == (line12_store, line17_read), (t, w_pc, o_pc)


def test_race_free_and_between_launch_sites():
    assert len(O.run_job(W.fig1_job("BASE")).races) == 0
    import test_oracle_streams as S
    res = O.run_job(S._job([S._spec(S._writer(100), 1, 4), S._spec(S._reader_of(3), 2, 1)], streams=[0, 1]))
    assert res.race_sites() == [(0xFFFFFFFF, 0xFFFFFFFF)] * len(res.races) and len(res.races) == 2
