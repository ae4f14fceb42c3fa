"""The allocation-free batched product (spamm_multiply_batched_noalloc) against
the allocating one (spamm_multiply_batched): same kernels and schedule, so the
same bits, on two calls in a row that share the static scratch, the second
with a smaller batch; the call draws nothing from the allocator."""
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


def _allocations():
    import torch
    return torch.cuda.memory_stats().get("allocation.all.allocated", 0)


def _dense(hs):
    return [h.to_dense().cpu().numpy() for h in hs]


def _targets(sizes, leaf, seed):
    # result handles that have received a product (of other operands), so
    # their product scratch is in place and their tiles hold other values
    others = sp.build_batched([to_dev(si.exp_decay(n, 0.7, seed + i, np.float32)) for i, n in enumerate(sizes)],
                              leaf)
    return sp.multiply_batched(others, others, [1e-2] * len(sizes), "f32")


@pytest.mark.parametrize("leaf,prec,schedule", [(64, "f32", "list"), (32, "f16x3", "lpt"), (64, "bf16x3", "static")])
def test_noalloc_equals_allocating_batched(leaf, prec, schedule):
    import torch
    calls = [([3072, 2048, 1000, 1536, 700], [1e-6, 1e-7, 1e-5, 1e-6, 0.0]),
             ([512, 900], [1e-6, 1e-4])]                                     # second call: smaller
    for c, (sizes, taus) in enumerate(calls):
        print(f"[case] noalloc call {c} leaf={leaf} prec={prec} schedule={schedule} sizes={sizes}", flush=True)
        mats = [si.algebraic_decay(n, 2.0, 80 + 10 * c + i, np.float32) for i, n in enumerate(sizes)]
        hs = sp.build_batched([to_dev(a) for a in mats], leaf)
        ref = _dense(sp.multiply_batched(hs, hs, taus, prec, schedule=schedule))
        outs = _targets(sizes, leaf, 500 + 10 * c)
        before = _dense(outs)
        torch.cuda.synchronize()
        n0 = _allocations()
        got = sp.multiply_batched_noalloc(hs, hs, taus, outs, prec, schedule=schedule)
        torch.cuda.synchronize()
        assert _allocations() == n0, "the allocation-free product drew memory from the allocator"
        assert all(g is o for g, o in zip(got, outs))
        for m, (g, r, b) in enumerate(zip(_dense(outs), ref, before)):
            assert np.array_equal(g, r), f"call {c} product {m} differs from the allocating path"
            assert not np.array_equal(b, r)   # the targets held other values before
        # the result is a valid operand: its norm pyramid matches a fresh build of its values
        chk = sp.build(outs[0].to_dense(), leaf)
        assert np.array_equal(outs[0].norms(0), chk.norms(0))


def test_noalloc_rejects_what_it_cannot_serve():
    print("[case] noalloc argument checks", flush=True)
    a = to_dev(si.algebraic_decay(1000, 2.0, 7, np.float32))
    A = sp.build(a, 64)
    with pytest.raises(sp.SpammError) as ei:            # a built handle holds no product scratch
        sp.multiply_batched_noalloc([A], [A], [1e-6], [sp.build(a, 64)], "f32")
    assert ei.value.code == 1
    C = sp.multiply(A, A, 1e-6, "f32")
    with pytest.raises(sp.SpammError) as ei:            # a result of another leaf size
        sp.multiply_batched_noalloc([A], [A], [1e-6], [sp.multiply(sp.build(a, 32), sp.build(a, 32), 1e-6)], "f32")
    assert ei.value.code == 1
    with pytest.raises(sp.SpammError) as ei:            # C aliases an operand
        sp.multiply_batched_noalloc([C], [A], [1e-6], [C], "f32")
    assert ei.value.code == 1


def test_noalloc_rejects_more_than_2_27_leaf_triples():
    # nb = 520 at leaf 32: 520^3 > 2^27 leaf triples need the descent's
    # frontiers, which the static scratch does not hold
    import torch
    print("[case] noalloc capacity limit n=16640 leaf 32", flush=True)
    n = 16640
    A = sp.build(sp.generate_decay(si.algebraic_table(n, 2.0), 9, 0.5, 1.5, False), 32)
    C = sp.multiply(A, A, 1e-2, "f32")
    before = C.to_dense().cpu().numpy()
    with pytest.raises(sp.SpammError) as ei:
        sp.multiply_batched_noalloc([A], [A], [1e-6], [C], "f32")
    assert ei.value.code == 4 and "2^27" in str(ei.value)
    torch.cuda.synchronize()
    assert np.array_equal(C.to_dense().cpu().numpy(), before)
