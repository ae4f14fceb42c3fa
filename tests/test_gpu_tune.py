"""Autotuner: chooses the fastest qualifying (leaf, schedule); cache round trip."""
import numpy as np
import pytest

import spamm_inputs as si
from gpu_util import to_dev

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_1011_3534_amd")


@pytest.fixture(scope="module", autouse=True)
def _torch_alloc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sp.use_torch_allocator(True)
    yield


def test_cross_leaf_diff_norms_exact():
    a = si.exp_decay(300, 0.9, 1, np.float32)
    A32, A64 = sp.build(to_dev(a), 32), sp.build(to_dev(a), 64)
    d2, r2 = sp.diff_norms(A32, A64)
    assert d2 == 0.0 and abs(r2 - float(np.sum(a.astype(np.float64) ** 2))) < 1e-9 * r2


def test_autotune_picks_fastest_qualifying_and_caches(tmp_path):
    print("[case] autotune", flush=True)
    params = si.batch_params(count=8, seed=3, n_lo=256, n_hi=1536)
    dense = [to_dev(si.batch_matrix(n, lam, useed)) for n, lam, useed in params]
    taus = [1e-6] * len(dense)
    cache = str(tmp_path / "tune.txt")
    tune, rep = sp.autotune_batched(dense, taus, "f32", leaves=(32, 64), max_rel_err=1e-5, reps=2, cache_path=cache)
    print("  ", tune, rep, flush=True)
    assert not rep["from_cache"] and len(rep["trials"]) == 6   # 2 leaf sizes x 3 schedules
    assert {t["schedule"] for t in rep["trials"]} == {"static", "lpt", "list"}
    ok = [t for t in rep["trials"] if t["qualified"]]
    assert ok
    fastest = min(ok, key=lambda t: t["ms"])
    assert tune == {"leaf": fastest["leaf"], "schedule": fastest["schedule"]}
    assert all(t["max_rel_err"] < 1e-4 for t in rep["trials"])
    tune2, rep2 = sp.autotune_batched(dense, taus, "f32", leaves=(32, 64), max_rel_err=1e-5, reps=2, cache_path=cache)
    assert rep2["from_cache"] and tune2 == tune
    # the tuned configuration runs
    hs = [sp.build(d, tune["leaf"]) for d in dense]
    Cs = sp.multiply_batched(hs, hs, taus, "f32", schedule=tune["schedule"])
    assert len(Cs) == len(hs)


def test_autotune_rejects_unreachable_target():
    dense = [to_dev(si.batch_matrix(256, 0.9, 5))]
    with pytest.raises(sp.SpammError, match="EINVAL"):
        sp.autotune_batched(dense, [1e-2], "bf16", leaves=(64,), max_rel_err=1e-9, reps=1)
