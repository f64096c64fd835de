"""Autotuner: every setting it may pick gives the same results, the cache it
writes is applied by kc_ctx_create, and a bad cache is refused."""
import json

import pytest

from gpu_util import check_jobs

pytestmark = pytest.mark.gpu


def test_tune_writes_cache_that_context_applies(tmp_path):
    from paper_1211_6193_amd import kc, tune, workloads as W
    jobs = W.config3_jobs(n=120) + [W.tree256_job(n_blocks=64)]
    path = str(tmp_path / "tune.json")
    with kc.Context(0) as ctx:
        res = tune.tune(ctx, jobs, path=path, reps=1, sweeps=1)
        assert all(same for _, _, same in res["tried"]), "a tunable option changed results"
        assert tune.current(ctx) == res["setting"]
    saved = json.load(open(path))
    assert saved == res["setting"]
    with kc.Context(0, tune_cache=path) as ctx2:
        assert tune.current(ctx2) == saved
        check_jobs(ctx2, jobs[::10] + jobs[-1:])


def test_bad_tune_cache_is_refused(tmp_path):
    from paper_1211_6193_amd import kc
    bad = tmp_path / "bad.json"
    bad.write_text('{"sort_tile": 1234}')
    with pytest.raises(kc.KcError):
        kc.Context(0, tune_cache=str(bad))
    bad.write_text('{"no_such_option": 1}')
    with pytest.raises(kc.KcError):
        kc.Context(0, tune_cache=str(bad))
    with pytest.raises(kc.KcError):
        kc.Context(0, tune_cache=str(tmp_path / "missing.json"))
