"""Batched products (one cull pass, one leaf launch) against the oracle and
against one-at-a-time products."""
import numpy as np
import pytest

import oracle
import spamm_inputs as si
from gpu_util import elementwise_bound, to_dev

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_1011_3534_amd")

SIZES = [64, 200, 512, 1000, 130, 700, 33, 300, 1024]


@pytest.fixture(scope="module", autouse=True)
def _torch_alloc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sp.use_torch_allocator(True)
    yield


def _batch(leaf, seed=0):
    rng = np.random.default_rng(seed)
    mats, taus = [], []
    for i, n in enumerate(SIZES):
        lam = float(rng.uniform(0.8, 0.97))
        mats.append(si.exp_decay(n, lam, 300 + i, np.float32))
        taus.append(float(10 ** rng.uniform(-7, -3)))
    return mats, taus


@pytest.mark.parametrize("leaf,prec,schedule", [(64, "f32", "lpt"), (32, "f16x3", "lpt"), (64, "bf16x3", "static"),
                                                (64, "f32", "list"), (32, "f16x3", "list"), (128, "f32", "list")])
def test_batched_matches_oracle(leaf, prec, schedule):
    print(f"[case] batched leaf={leaf} prec={prec} schedule={schedule}", flush=True)
    mats, taus = _batch(leaf)
    hs = [sp.build(to_dev(a), leaf) for a in mats]
    Cs, sts = sp.multiply_batched(hs, hs, taus, prec, stats=True, schedule=schedule)
    for a, C, st, tau in zip(mats, Cs, sts, taus):
        a64 = a.astype(np.float64)
        S = oracle.tile_sqnorms(a64, leaf)
        keys, _ = oracle.tasks_flat(S, S, tau)
        assert np.array_equal(C.task_list(), keys)
        T, kept = oracle.count_hierarchical(S, S, tau)
        assert st["tasks"] == T and st["survivors"] == kept.tolist()
        ref, _ = oracle.spamm_flat(a64, a64, leaf, tau)
        out = C.to_dense().cpu().numpy().astype(np.float64)
        assert np.all(np.abs(out - ref) <= elementwise_bound(a64, a64, leaf, tau, prec))
        for lv, r in enumerate(oracle.norm_pyramid(out, leaf)):
            assert np.array_equal(C.norms(lv), r)


@pytest.mark.parametrize("leaf,prec,schedule", [(64, "f32", "list"), (32, "f16x3", "static"), (128, "f32", "lpt")])
def test_batched_direct_leaf_pass_matches_oracle(leaf, prec, schedule):
    # without statistics the batch tests every leaf triple in one pass (no
    # tier above the leaves is read or formed): kept triples equal the
    # oracle's, values stay within the bound, and the results equal the
    # batch with statistics (full descent) bit for bit
    print(f"[case] batched direct leaf={leaf} prec={prec} schedule={schedule}", flush=True)
    mats, taus = _batch(leaf, seed=2)
    hs = [sp.build(to_dev(a), leaf) for a in mats]
    Cs = sp.multiply_batched(hs, hs, taus, prec, schedule=schedule)
    Ds, _ = sp.multiply_batched(hs, hs, taus, prec, stats=True, schedule=schedule)
    for a, C, D, tau in zip(mats, Cs, Ds, taus):
        a64 = a.astype(np.float64)
        S = oracle.tile_sqnorms(a64, leaf)
        keys, _ = oracle.tasks_flat(S, S, tau)
        assert np.array_equal(C.task_list(), keys)
        ref, _ = oracle.spamm_flat(a64, a64, leaf, tau)
        out = C.to_dense().cpu().numpy()
        assert np.all(np.abs(out.astype(np.float64) - ref) <= elementwise_bound(a64, a64, leaf, tau, prec))
        assert np.array_equal(out.view(np.uint32), D.to_dense().cpu().numpy().view(np.uint32))


def test_batched_equals_single_products_bitwise():
    print("[case] batched == single", flush=True)
    mats, taus = _batch(64, seed=1)
    hs = [sp.build(to_dev(a), 64) for a in mats]
    lpt = sp.multiply_batched(hs, hs, taus, "f16x3", schedule="lpt")
    static = sp.multiply_batched(hs, hs, taus, "f16x3", schedule="static")
    lst = sp.multiply_batched(hs, hs, taus, "f16x3", schedule="list")
    for h, tau, c1, c2, c3 in zip(hs, taus, lpt, static, lst):
        single = sp.multiply(h, h, tau, "f16x3")
        a = single.to_dense().cpu().numpy()
        assert np.array_equal(c1.to_dense().cpu().numpy(), a)
        assert np.array_equal(c2.to_dense().cpu().numpy(), a)
        assert np.array_equal(c3.to_dense().cpu().numpy(), a)
        assert np.array_equal(c1.task_list(), single.task_list())
        assert np.array_equal(c3.norms(0), single.norms(0))


def test_list_schedule_reused_outputs_with_changing_kept_sets():
    # the list skips tiles with no kept product whose stored values are known
    # zero; a reused output whose kept set shrinks or grows must still equal
    # fresh products (tiles that became empty are listed and zeroed)
    print("[case] list schedule, reused outputs", flush=True)
    mats, _ = _batch(64, seed=4)
    hs = [sp.build(to_dev(a), 64) for a in mats]
    outs = None
    for tau in (1e-7, 1e-3, 1e-3, 1e-8, 0.0, 1e-5):
        taus = [tau] * len(hs)
        outs = sp.multiply_batched(hs, hs, taus, "f32", outs=outs, schedule="list")
        fresh = sp.multiply_batched(hs, hs, taus, "f32", schedule="static")
        for c, f in zip(outs, fresh):
            assert np.array_equal(c.to_dense().cpu().numpy(), f.to_dense().cpu().numpy())
            assert np.array_equal(c.norms(0), f.norms(0))
            assert np.array_equal(c.task_list(), f.task_list())


def test_batched_output_reuse_and_errors():
    print("[case] batched reuse/errors", flush=True)
    mats, taus = _batch(64, seed=2)
    hs = [sp.build(to_dev(a), 64) for a in mats]
    Cs = sp.multiply_batched(hs, hs, taus, "f32")
    first = [c.to_dense().cpu().numpy().copy() for c in Cs]
    Cs2 = sp.multiply_batched(hs, hs, taus, "f32", outs=Cs)
    assert all(a is b for a, b in zip(Cs, Cs2))
    assert all(np.array_equal(c.to_dense().cpu().numpy(), f) for c, f in zip(Cs2, first))
    h32 = sp.build(to_dev(mats[0]), 32)
    with pytest.raises(sp.SpammError, match="EINVAL"):
        sp.multiply_batched([hs[0], h32], [hs[0], h32], [1e-6, 1e-6])
    with pytest.raises(sp.SpammError, match="EINVAL"):
        sp.multiply_batched([hs[0]], [hs[0]], [1e-6], outs=[hs[0]])


@pytest.mark.parametrize("leaf,dtype", [(64, np.float32), (32, np.float64), (128, np.float32)])
def test_build_batched_equals_single_builds(leaf, dtype):
    # one pack launch and one launch per upper tier for the whole batch: the
    # same pyramids (bit-exact, also against the oracle), tiles and tile
    # exponents (through an FP16x3 product, which scales by them) as one
    # spamm_build per matrix; ragged sizes, one smaller than a tile
    print(f"[case] build_batched leaf={leaf} {np.dtype(dtype).name}", flush=True)
    sizes = [1, 31, leaf, leaf + 1, 200, 513, 1000, 130]
    mats = [si.exp_decay(n, 0.85, 400 + i, dtype) for i, n in enumerate(sizes)]
    Hs = sp.build_batched([to_dev(a) for a in mats], leaf)
    for a, H in zip(mats, Hs):
        S = sp.build(to_dev(a), leaf)
        assert H.levels == S.levels
        ref = oracle.norm_pyramid(a.astype(np.float64), leaf)
        for lv in range(S.levels + 1):
            assert np.array_equal(H.norms(lv), S.norms(lv)) and np.array_equal(H.norms(lv), ref[lv])
        assert np.array_equal(H.to_dense().cpu().numpy(), a)
        if dtype == np.float32:
            c1 = sp.multiply(H, H, 1e-6, "f16x3").to_dense().cpu().numpy()
            c2 = sp.multiply(S, S, 1e-6, "f16x3").to_dense().cpu().numpy()
            assert np.array_equal(c1, c2)
    # rebuilt in place from other values
    mats2 = [si.algebraic_decay(n, 2.0, 500 + i, dtype) for i, n in enumerate(sizes)]
    Hs2 = sp.build_batched([to_dev(a) for a in mats2], leaf, outs=Hs)
    assert all(x is y for x, y in zip(Hs, Hs2))
    for a, H in zip(mats2, Hs2):
        assert np.array_equal(H.norms(0), oracle.tile_sqnorms(a.astype(np.float64), leaf))
        assert np.array_equal(H.to_dense().cpu().numpy(), a)


def test_build_batched_errors():
    print("[case] build_batched errors", flush=True)
    a = to_dev(si.exp_decay(100, 0.85, 1, np.float32))
    b = to_dev(si.exp_decay(200, 0.85, 2, np.float32))
    with pytest.raises(sp.SpammError, match="EINVAL"):
        sp.build_batched([], 64)
    H = sp.build(a, 64)
    with pytest.raises(sp.SpammError, match="EINVAL"):
        sp.build_batched([a, b], 64, outs=[None, H])        # H has n = 100, not 200
    with pytest.raises(sp.SpammError, match="EINVAL"):
        sp.build_batched([a, a], 64, outs=[H, H])           # repeated handle
    with pytest.raises(sp.SpammError, match="EINVAL"):
        sp.build_batched([a, b], 48)                         # leaf size
    Hs = sp.build_batched([a, b], 64)
    assert [h.n for h in Hs] == [100, 200]
