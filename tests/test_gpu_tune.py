"""Autotuner: chooses the fastest qualifying (leaf, staging, schedule); cache keyed by batch buckets."""
import math

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
    assert tune == {"leaf": fastest["leaf"], "schedule": fastest["schedule"], "split": False}
    assert not any(t["split"] for t in rep["trials"])   # FP32 leaves: no staging axis
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


def _bucket(v, step):
    return math.floor(math.log2(v) / step + 0.5)


def _kept_fraction(dense, taus, leaf, prec):
    hs = [sp.build(d, leaf) for d in dense]
    _, sts = sp.multiply_batched(hs, hs, taus, prec, stats=True)
    return sum(s["tasks"] for s in sts) / sum(s["nb"] ** 3 for s in sts)


def test_autotune_split_axis_for_16_bit_leaves(tmp_path):
    print("[case] autotune bf16x3 split axis", flush=True)
    params = si.batch_params(count=6, seed=4, n_lo=256, n_hi=1024)
    dense = [to_dev(si.batch_matrix(n, lam, useed)) for n, lam, useed in params]
    taus = [1e-5] * len(dense)
    tune, rep = sp.autotune_batched(dense, taus, "bf16x3", leaves=(64,), max_rel_err=1e-3, reps=2,
                                    cache_path=str(tmp_path / "t.txt"))
    print("  ", tune, rep, flush=True)
    trials = rep["trials"]
    assert len(trials) == 6
    assert {(t["split"], t["schedule"]) for t in trials} == {(s, k) for s in (False, True)
                                                             for k in ("static", "lpt", "list")}
    # the same products either way: split and on-the-fly staging give the same bits
    for k in ("static", "lpt", "list"):
        pair = [t["max_rel_err"] for t in trials if t["schedule"] == k]
        assert pair[0] == pair[1]
    fastest = min((t for t in trials if t["qualified"]), key=lambda t: t["ms"])
    assert tune == {"leaf": 64, "schedule": fastest["schedule"], "split": fastest["split"]}
    # the tuned configuration runs with the operands it names
    hs = [sp.build(d, 64, prec="bf16x3" if tune["split"] else None) for d in dense]
    Cs = sp.multiply_batched(hs, hs, taus, "bf16x3", schedule=tune["schedule"])
    assert len(Cs) == len(hs)


def test_autotune_cache_is_keyed_by_batch_buckets(tmp_path):
    print("[case] autotune cache buckets", flush=True)
    cache = str(tmp_path / "tune.txt")
    params = si.batch_params(count=4, seed=7, n_lo=512, n_hi=768)
    dense = [to_dev(si.batch_matrix(n, lam, useed)) for n, lam, useed in params]
    taus = [1e-6] * 4
    tune, rep = sp.autotune_batched(dense, taus, "f32", leaves=(32,), max_rel_err=1e-4, reps=1, cache_path=cache)
    assert not rep["from_cache"]
    # another batch of the same shape: each matrix 64 rows smaller, same decay
    dense2 = [to_dev(si.batch_matrix(n - 64, lam, useed)) for n, lam, useed in params]
    mean1 = sum(d.shape[0] for d in dense) / 4
    mean2 = sum(d.shape[0] for d in dense2) / 4
    k1, k2 = _kept_fraction(dense, taus, 32, "f32"), _kept_fraction(dense2, taus, 32, "f32")
    same = _bucket(mean1, 0.5) == _bucket(mean2, 0.5) and _bucket(k1, 1.0) == _bucket(k2, 1.0)
    print(f"   mean n {mean1} / {mean2}, kept {k1:.4g} / {k2:.4g}, same buckets {same}", flush=True)
    tune2, rep2 = sp.autotune_batched(dense2, taus, "f32", leaves=(32,), max_rel_err=1e-4, reps=1, cache_path=cache)
    assert rep2["from_cache"] == same
    if same:
        assert tune2 == tune
    # tau = 0 keeps every triple: a different kept-fraction bucket, so new trials
    assert _bucket(_kept_fraction(dense, [0.0] * 4, 32, "f32"), 1.0) != _bucket(k1, 1.0)
    _, rep3 = sp.autotune_batched(dense, [0.0] * 4, "f32", leaves=(32,), max_rel_err=1e-4, reps=1, cache_path=cache)
    assert not rep3["from_cache"] and len(rep3["trials"]) == 3
    # and the first batch hits its own line
    _, rep4 = sp.autotune_batched(dense, taus, "f32", leaves=(32,), max_rel_err=1e-4, reps=1, cache_path=cache)
    assert rep4["from_cache"]
