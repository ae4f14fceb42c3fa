"""Views (spamm_build_view): handles whose tiles are the caller's row-major
array.  Their norm pyramids and products must be the same bits as those of
packed handles of the same array, which the other GPU tests hold to the
oracle; one case is also checked against the oracle directly."""
import numpy as np
import pytest

import oracle
import spamm_inputs as si
from gpu_util import elementwise_bound, to_dev

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_1011_3534_amd")


@pytest.fixture(scope="module", autouse=True)
def _torch_alloc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sp.use_torch_allocator(True)
    yield


def _dense(C):
    return C.to_dense().cpu().numpy()


def _same_bits(X, Y):
    x, y = _dense(X), _dense(Y)
    assert x.dtype == y.dtype
    assert np.array_equal(x.view(np.uint8), y.view(np.uint8))


def _padded(a, extra):
    """a stored with row pitch n + extra (a column slice of a wider array)."""
    import torch
    n = a.shape[0]
    wide = torch.full((n, n + extra), float("nan"), dtype=torch.float32 if a.dtype == np.float32 else torch.float64,
                      device="cuda")
    wide[:, :n] = to_dev(a)
    return wide[:, :n]


# leaf, n (a multiple of the leaf), extra row pitch (elements), dtype
CASES = [(32, 224, 0, np.float32), (64, 320, 0, np.float32), (64, 320, 16, np.float32),
         (128, 384, 4, np.float32), (64, 192, 2, np.float64)]


@pytest.mark.parametrize("leaf,n,extra,dt", CASES)
def test_view_norms_and_products_equal_packed(leaf, n, extra, dt):
    print(f"[case] view leaf={leaf} n={n} extra={extra} dt={np.dtype(dt).name}", flush=True)
    a = si.exp_decay(n, 0.9, 41, dt)
    b = si.exp_decay(n, 0.85, 42, dt)
    da = _padded(a, extra) if extra else to_dev(a)
    db = _padded(b, extra) if extra else to_dev(b)
    A, B = sp.build(da, leaf), sp.build(db, leaf)
    VA, VB = sp.build(da, leaf, view=True), sp.build(db, leaf, view=True)
    assert VA.source is da
    for lvl in range(A.levels + 1):
        assert np.array_equal(VA.norms(lvl), A.norms(lvl))
        assert np.array_equal(VB.norms(lvl), B.norms(lvl))
    assert np.array_equal(_dense(VA), a)
    d2, r2 = sp.diff_norms(VA, A)
    assert d2 == 0.0 and r2 == pytest.approx(float(np.sum(a.astype(np.float64) ** 2)), rel=1e-12)
    precs = ["f64"] if dt == np.float64 else ["f32", "f16x3", "bf16x3", "f16", "bf16", "f64"]
    for prec in precs:
        for tau in (0.0, 1e-4):
            C = sp.multiply(A, B, tau, prec)
            CV = sp.multiply(VA, VB, tau, prec)
            CM = sp.multiply(VA, B, tau, prec)
            _same_bits(CV, C)
            _same_bits(CM, C)
            assert np.array_equal(CV.task_list(), C.task_list())


def test_view_product_matches_oracle():
    print("[case] view oracle parity n=320 leaf 64 f32 tau=1e-5", flush=True)
    n, leaf, tau = 320, 64, 1e-5
    a = si.exp_decay(n, 0.9, 43, np.float32)
    da = _padded(a, 8)
    V = sp.build(da, leaf, view=True)
    C = sp.multiply(V, V, tau, "f32")
    a64 = a.astype(np.float64)
    ref, _ = oracle.spamm_flat(a64, a64, leaf, tau)
    bound = elementwise_bound(a64, a64, leaf, tau, "f32")
    assert np.all(np.abs(_dense(C).astype(np.float64) - ref) <= bound)
    SA = oracle.tile_sqnorms(a64, leaf)
    keys, _ = oracle.tasks_flat(SA, SA, tau)
    assert np.array_equal(C.task_list(), np.sort(keys))


def test_view_rebuild_repoints_and_rejects_mixing():
    print("[case] view rebuild / misuse", flush=True)
    n, leaf = 256, 64
    a = si.exp_decay(n, 0.9, 44, np.float32)
    b = si.exp_decay(n, 0.8, 45, np.float32)
    da, db = to_dev(a), to_dev(b)
    V = sp.build(da, leaf, view=True)
    h = V.handle.value
    V2 = sp.build(db, leaf, out=V, view=True)  # re-point at another array, no new handle
    assert V2 is V and V.handle.value == h and V.source is db
    P = sp.build(db, leaf)
    for lvl in range(P.levels + 1):
        assert np.array_equal(V.norms(lvl), P.norms(lvl))
    _same_bits(sp.multiply(V, V, 1e-6, "f16x3"), sp.multiply(P, P, 1e-6, "f16x3"))
    with pytest.raises(sp.SpammError) as e:
        sp.build(da, leaf, out=V)  # packing into a view
    assert e.value.status == "EINVAL"
    with pytest.raises(sp.SpammError) as e:
        sp.build(da, leaf, out=P, view=True)  # a view into a packed handle
    assert e.value.status == "EINVAL"
    with pytest.raises(sp.SpammError) as e:
        sp.multiply(P, P, 1e-6, "f32", out=V)  # a view cannot hold a product
    assert e.value.status == "EINVAL"
    with pytest.raises(sp.SpammError) as e:
        sp.multiply_batched([P], [P], [1e-6], "f32", outs=[V])
    assert e.value.status == "EINVAL"
    with pytest.raises(sp.SpammError) as e:
        sp.sp2(V, n // 2, 1e-6, max_iter=2)
    assert e.value.status == "EUNSUPPORTED"
    # the handle still works after the rejected calls
    _same_bits(sp.multiply(V, V, 1e-6, "f32"), sp.multiply(P, P, 1e-6, "f32"))


@pytest.mark.parametrize("schedule", ["list", "lpt"])
def test_view_batched_equals_packed(schedule):
    print(f"[case] view batched schedule={schedule}", flush=True)
    rng = np.random.default_rng(7)
    sizes = [64, 512, 128, 1024, 320, 64 * 11]
    mats = [si.exp_decay(n, float(rng.uniform(0.8, 0.97)), 500 + i, np.float32) for i, n in enumerate(sizes)]
    taus = [float(10 ** rng.uniform(-7, -3)) for _ in sizes]
    dev = [to_dev(a) for a in mats]
    P = sp.build_batched(dev, 64)
    V = sp.build_batched(dev, 64, view=True)
    for p, v in zip(P, V):
        for lvl in range(p.levels + 1):
            assert np.array_equal(v.norms(lvl), p.norms(lvl))
    for prec in ("f32", "f16x3"):
        CP = sp.multiply_batched(P, P, taus, prec, schedule=schedule)
        CV = sp.multiply_batched(V, V, taus, prec, schedule=schedule)
        for cp, cv in zip(CP, CV):
            _same_bits(cv, cp)
    # rebuild the views in place on other arrays
    dev2 = [to_dev(si.exp_decay(n, 0.9, 600 + i, np.float32)) for i, n in enumerate(sizes)]
    V2 = sp.build_batched(dev2, 64, outs=V, view=True)
    P2 = sp.build_batched(dev2, 64)
    for v, p, d in zip(V2, P2, dev2):
        assert v.source is d
        assert np.array_equal(v.norms(0), p.norms(0))


def test_view_full_size_product_equals_packed():
    """The bench workload (algebraic decay, n = 8192, leaf 64) at tau = 1e-6."""
    print("[case] view full size n=8192 f16x3/f32 tau=1e-6", flush=True)
    a = si.algebraic_workload(8192)
    da = to_dev(a)
    P = sp.build(da, 64)
    V = sp.build(da, 64, view=True)
    assert np.array_equal(V.norms(0), P.norms(0))
    for prec in ("f16x3", "f32"):
        C, st = sp.multiply(P, P, 1e-6, prec, stats=True)
        CV, stv = sp.multiply(V, V, 1e-6, prec, stats=True)
        assert stv["tasks"] == st["tasks"] == 104137
        d2, _ = sp.diff_norms(CV, C)
        assert d2 == 0.0


@pytest.mark.parametrize("leaf,n,extra", [(64, 320, 0), (64, 384, 16), (32, 224, 0), (128, 384, 4)])
def test_split_view_products_equal_view(leaf, n, extra):
    # views with split tiles (spamm_build_view_ex): the 16-bit leaves read the
    # split tiles (at leaf 64 straight into LDS) instead of splitting the
    # array on the fly; the products are the same bits
    print(f"[case] split view leaf={leaf} n={n} extra={extra}", flush=True)
    a = si.algebraic_decay(n, 2.0, 44, np.float32)
    b = si.exp_decay(n, 0.85, 45, np.float32)
    da = _padded(a, extra) if extra else to_dev(a)
    db = _padded(b, extra) if extra else to_dev(b)
    VA, VB = sp.build(da, leaf, view=True), sp.build(db, leaf, view=True)
    for prec in ("f16x3", "bf16x3", "f16", "bf16"):
        SA, SB = sp.build(da, leaf, view=True, prec=prec), sp.build(db, leaf, view=True, prec=prec)
        assert np.array_equal(SA.norms(0), VA.norms(0))
        for tau in (0.0, 1e-5):
            _same_bits(sp.multiply(SA, SB, tau, prec), sp.multiply(VA, VB, tau, prec))
            _same_bits(sp.multiply(SA, SA, tau, prec), sp.multiply(VA, VA, tau, prec))
        # one split operand and one without: split on the fly (same bits)
        _same_bits(sp.multiply(SA, VB, 1e-5, prec), sp.multiply(VA, VB, 1e-5, prec))
    # a rebuild of a split view on other values refreshes its split tiles
    S = sp.build(da, leaf, view=True, prec="f16x3")
    sp.build(db, leaf, out=S, view=True, prec="f16x3")
    _same_bits(sp.multiply(S, S, 1e-5, "f16x3"), sp.multiply(VB, VB, 1e-5, "f16x3"))


@pytest.mark.parametrize("n", [64, 100, 130, 190])
def test_split_packed_small_and_ragged_equal_on_the_fly(n):
    # packed builds with split tiles (spamm_build_ex) at one tile (nb = 1) and
    # ragged sizes (zero-padded tiles, odd nb): a single product of split
    # operands (leaf 64: 2 x 2 super-tiles, some of them cut by the edge) is
    # the same bits as the product that splits the packed tiles on the fly
    print(f"[case] split packed leaf=64 n={n}", flush=True)
    a = si.algebraic_decay(n, 2.0, 46, np.float32)
    b = si.exp_decay(n, 0.8, 47, np.float32)
    da, db = to_dev(a), to_dev(b)
    PA, PB = sp.build(da, 64), sp.build(db, 64)
    for prec in ("f16x3", "bf16x3", "f16", "bf16"):
        SA, SB = sp.build(da, 64, prec=prec), sp.build(db, 64, prec=prec)
        for tau in (0.0, 1e-4):
            _same_bits(sp.multiply(SA, SB, tau, prec), sp.multiply(PA, PB, tau, prec))
            _same_bits(sp.multiply(SB, SA, tau, prec), sp.multiply(PB, PA, tau, prec))


@pytest.mark.parametrize("schedule", ["list", "lpt", "static"])
def test_split_view_batched_equals_view(schedule):
    print(f"[case] split view batched schedule={schedule}", flush=True)
    rng = np.random.default_rng(9)
    sizes = [64, 512, 128, 1024, 320, 64 * 11]
    mats = [si.exp_decay(n, float(rng.uniform(0.8, 0.97)), 700 + i, np.float32) for i, n in enumerate(sizes)]
    taus = [float(10 ** rng.uniform(-7, -3)) for _ in sizes]
    dev = [to_dev(a) for a in mats]
    V = [sp.build(d, 64, view=True) for d in dev]
    for prec in ("f16x3", "bf16"):
        S = [sp.build(d, 64, view=True, prec=prec) for d in dev]
        CS = sp.multiply_batched(S, S, taus, prec, schedule=schedule)
        CV = sp.multiply_batched(V, V, taus, prec, schedule=schedule)
        for cs, cv in zip(CS, CV):
            _same_bits(cs, cv)


@pytest.mark.parametrize("n,tau", [(8192, 1e-6), (16448, 1e-7)])
def test_split_view_full_size_equals_view(n, tau):
    """The bench workload (n = 8192, leaf 64, FP16x3) and nb = 257 (tiles whose
    kept K span two 256-K segments), split view against view."""
    print(f"[case] split view full size n={n} f16x3 tau={tau}", flush=True)
    a = si.algebraic_workload(8192) if n == 8192 else None
    da = to_dev(a) if a is not None else sp.generate_decay(si.algebraic_table(n, 1.5), 61, 0.5, 1.5, False)
    V = sp.build(da, 64, view=True)
    S = sp.build(da, 64, view=True, prec="f16x3")
    CV = sp.multiply(V, V, tau, "f16x3")
    CS = sp.multiply(S, S, tau, "f16x3")
    d2, r2 = sp.diff_norms(CS, CV)
    assert d2 == 0.0 and r2 > 0.0
    assert np.array_equal(CS.task_list(), CV.task_list())
