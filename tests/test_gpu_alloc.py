"""The allocator hook is stream-ordered: scratch the library releases right
after enqueueing the kernels that read it goes back to the pool of the
stream it was used on, so work on another stream cannot be handed that
memory while those kernels still run."""
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


def test_side_stream_products_survive_current_stream_allocations():
    # reference products on the current stream; then the same calls on a side
    # stream (the current one stays the default), the caller's input tensors
    # released as soon as they are enqueued, and the current stream at once
    # allocating and filling a lot of memory with NaN while the side stream
    # still works: the results must be the same bits
    import torch
    print("[case] side-stream batched product + builds + tau workspaces", flush=True)
    sizes = [1536, 2048, 1024, 3072]
    mats = [si.algebraic_decay(n, 2.0, 70 + i, np.float32) for i, n in enumerate(sizes)]
    ref_h = sp.build_batched([to_dev(a) for a in mats], 64)
    ref = [c.to_dense().cpu().numpy() for c in sp.multiply_batched(ref_h, ref_h, [1e-6] * 4, "f32", schedule="list")]
    ref_single = sp.multiply(ref_h[3], ref_h[3], 1e-6, "f16x3").to_dense().cpu().numpy()
    ref_err = sp.rel_err(sp.multiply(ref_h[1], ref_h[1], 1e-6, "f32"), sp.multiply(ref_h[1], ref_h[1], 0.0, "f64"))
    torch.cuda.synchronize()

    side = torch.cuda.Stream()
    cur = torch.cuda.current_stream()
    for rep in range(3):
        ins = [to_dev(a) for a in mats]
        side.wait_stream(cur)
        hs = sp.build_batched(ins, 64, stream=side)
        for t in ins:
            t.record_stream(side)
        del ins
        Cs = sp.multiply_batched(hs, hs, [1e-6] * 4, "f32", schedule="list", stream=side)
        C1 = sp.multiply(hs[3], hs[3], 1e-6, "f16x3", stream=side)
        E = sp.multiply(hs[1], hs[1], 0.0, "f64", stream=side)
        C2 = sp.multiply(hs[1], hs[1], 1e-6, "f32", stream=side)
        junk = [torch.full((1 << 22,), float("nan"), device="cuda") for _ in range(16)]   # on the current stream
        err = sp.rel_err(C2, E, stream=side)
        side.synchronize()
        del junk
        outs = [c.to_dense(stream=side) for c in Cs]
        single = C1.to_dense(stream=side)
        side.synchronize()
        for o, r in zip(outs, ref):
            assert np.array_equal(o.cpu().numpy(), r)
        assert np.array_equal(single.cpu().numpy(), ref_single)
        assert err == ref_err
    print(f"  rel_err {ref_err:.3e}", flush=True)


def test_tau_model_weights_follow_the_stream():
    # training on a side stream and reading the weights back: spamm_tau_model_params
    # orders its copy after the model's last stream (no device-wide synchronisation)
    import torch
    print("[case] tau model on a side stream", flush=True)
    from paper_1011_3534_amd import tau_data
    shapes = tau_data.SHAPES
    p0 = si.mlp_init(shapes, 3)
    m = sp.TauModel(p0)
    X = torch.randn((64, sp.TAU_NFEAT), device="cuda")
    y = torch.randn((64,), device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    m.train(X, y, 2, 16, 1e-3, stream=side)
    p_side = m.params()
    m2 = sp.TauModel(p0)
    m2.train(X, y, 2, 16, 1e-3)
    assert np.array_equal(p_side, m2.params())
    assert not np.array_equal(p_side, p0)
