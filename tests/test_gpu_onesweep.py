"""Sorts that take the single-pass digit scatters (option onesweep) against
the three-kernel passes and the oracle:

* a stencil ping-pong over 2^20 words whose logs (above 2^20 records each)
  take the sorted check: reports and memories equal the oracle's with the
  option on and off, for several digit widths and tile sizes;
* every look-back wait bounded to no poll at all (option sort_spin = 0): a
  tile that finds an earlier tile's counts not yet published stalls its pass,
  the host finishes the sort with three-kernel passes from that pass's input,
  and the results are still the oracle's;
* a log of representatives only sorted by location alone (option loc_sort)
  or by the whole key: the same results."""
import pytest

torch = pytest.importorskip("torch")

from gpu_util import assert_same, say
from oracle import oracle as O
from paper_1211_6193_amd import kc
from paper_1211_6193_amd import workloads as W

pytestmark = pytest.mark.gpu

N = 1 << 20


@pytest.fixture(scope="module")
def case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    job = W.stencil_pingpong_job(n=N, threads=256, steps=2, bug_frac=0.004, seed=12116197)
    say(f"oracle of the stencil ping-pong over {N} words")
    return job, O.run_job(job)


@pytest.fixture(scope="module")
def ctx():
    c = kc.Context(0)
    c.set_option("hash_check", 0)       # every log takes the sort
    yield c
    c.close()


def _run(ctx, case, label, **opts):
    job, ora = case
    for k, v in opts.items():
        ctx.set_option(k, v)
    try:
        ctx.reset_stats()
        say(f"{label}: {opts}")
        rep, mem = kc.run_job(ctx, job)
        assert_same(rep, mem, ora, label)
        assert ctx.stat("sort_keys") >= 2 * (1 << 20)
        return {k: ctx.stat(k) for k in ("sort_onesweep", "sort_stalls", "sorted_checks", "sort_ms", "loc_sorts")}
    finally:
        ctx.set_option("onesweep", 0)
        ctx.set_option("sort_spin", 1 << 16)
        ctx.set_option("sort_bits", 8)
        ctx.set_option("sort_tile", 2048)
        ctx.set_option("loc_sort", 1)


@pytest.mark.parametrize("onesweep", [1, 0], ids=["single-pass", "three-kernel"])
def test_same_results_either_way(ctx, case, onesweep):
    st = _run(ctx, case, "onesweep" if onesweep else "three-kernel", onesweep=onesweep)
    say(f"stats {st}")
    if onesweep:
        assert st["sort_onesweep"] >= 2 and st["sort_stalls"] == 0
    else:
        assert st["sort_onesweep"] == 0


@pytest.mark.parametrize("bits,tile", [(5, 2048), (8, 1024), (8, 4096), (6, 8192)])
def test_digit_widths_and_tiles(ctx, case, bits, tile):
    st = _run(ctx, case, f"bits={bits} tile={tile}", onesweep=1, sort_bits=bits, sort_tile=tile)
    assert st["sort_onesweep"] >= 2 and st["sort_stalls"] == 0


def test_stalled_passes_are_finished_by_the_three_kernel_passes(ctx, case):
    st = _run(ctx, case, "no waiting", onesweep=1, sort_spin=0)
    say(f"stats {st}")
    assert st["sort_onesweep"] >= 2


@pytest.mark.parametrize("loc", [1, 0], ids=["location-key", "whole-key"])
def test_location_key_or_whole_key(ctx, case, loc):
    st = _run(ctx, case, f"loc_sort={loc}", loc_sort=loc)
    say(f"stats {st}")
    if not loc:
        assert st["loc_sorts"] == 0
