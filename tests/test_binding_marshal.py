"""The binding marshals jobs into the C descriptors (no GPU: fake program
handles and memories): launches, streams, event dependencies and allocations
reach the kc_job fields the header defines."""
import pytest

from paper_1211_6193_amd import kc


class _Prog:
    h = None


class _Mem:
    def __init__(self, n):
        self.n = n

    def data_ptr(self):
        return 0x1000

    def numel(self):
        return self.n


def _prepare(items):
    b = kc.Batch.__new__(kc.Batch)     # no context needed to marshal
    return b.prepare(items)


def test_plain_job_has_no_streams_deps_or_allocs():
    p = _prepare([([(_Prog(), (2, 1, 1), (9, 1, 1), 36, (0, 18))], _Mem(20), 7)])
    j = p.jd[0]
    assert j.n_launches == 1 and j.n_words == 20 and j.tag == 7
    assert not j.streams and not j.deps and j.n_deps == 0 and not j.allocs and j.n_allocs == 0
    assert j.launches[0].grid.x == 2 and j.launches[0].block.x == 9 and j.launches[0].shmem_bytes == 36
    assert list(j.launches[0].params)[:2] == [0, 18] and j.launches[0].n_params == 2


def test_streams_deps_and_allocs_are_marshalled():
    L = (_Prog(), (1, 1, 1), (4, 1, 1), 0, ())
    p = _prepare([([L, L, L], _Mem(32), 1, [0, 1, 0], [(0, 1), (1, 2)], [(0, 8), (16, 8)]),
                  ([L], _Mem(8), 2, None, (), [])])
    a, b = p.jd[0], p.jd[1]
    assert [a.streams[i] for i in range(3)] == [0, 1, 0]
    assert a.n_deps == 2 and [(a.deps[i].before, a.deps[i].after) for i in range(2)] == [(0, 1), (1, 2)]
    assert a.n_allocs == 2 and [(a.allocs[i].base, a.allocs[i].words) for i in range(2)] == [(0, 8), (16, 8)]
    # an empty allocation list is still a list (every access outside it), not "no check"
    assert bool(b.allocs) and b.n_allocs == 0 and not b.streams and b.n_deps == 0


def test_one_stream_per_launch_required():
    L = (_Prog(), (1, 1, 1), (4, 1, 1), 0, ())
    with pytest.raises(ValueError):
        _prepare([([L, L], _Mem(8), 0, [0], (), None)])
