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


def test_host_program_items_are_marshalled():
    from paper_1211_6193_amd import workloads as W
    L = (_Prog(), (1, 1, 1), (4, 1, 1), 0, ())
    steps = [W.copy_item(8, 0, 4, stream=2, sync=True), W.launch_item(0, stream=1), W.host_wait(1),
             W.host_write(0, 3, -5), W.host_read(8, 2), W.host_wait()]
    p = _prepare([([L], _Mem(16), 3, None, [(0, 1)], None, steps), ([L], _Mem(8), 4)])
    a, b = p.jd[0], p.jd[1]
    assert a.n_items == 6 and not a.streams and a.n_deps == 1
    got = [(a.items[i].kind, a.items[i].stream, a.items[i].ref, a.items[i].flags, a.items[i].dst, a.items[i].src,
            a.items[i].words, a.items[i].value) for i in range(6)]
    assert got == [(1, 2, 0, 1, 8, 0, 4, 0), (0, 1, 0, 0, 0, 0, 0, 0), (4, 0, 1, 0, 0, 0, 0, 0),
                   (3, 0, 0, 0, 0, 0, 3, -5), (2, 0, 0, 0, 8, 0, 2, 0), (4, 0, kc.WAIT_ALL, 0, 0, 0, 0, 0)]
    assert not b.items and b.n_items == 0
    with pytest.raises(ValueError):
        _prepare([([L], _Mem(8), 0, None, (), None, [W.Item("memset")])])
