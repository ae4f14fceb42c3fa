"""GPU parity at the full sizes of the workloads, on what the oracle can
compute there: complete kept-triple lists (bit-exact), sampled leaf norms
against the host generator, and sampled C tile rows."""
import numpy as np
import pytest

import oracle
import spamm_inputs as si
from gpu_util import check_row_many
from oracle import sp2 as osp2

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_1011_3534_amd")


@pytest.fixture(scope="module", autouse=True)
def _torch_alloc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sp.use_torch_allocator(True)
    yield


def _host_block(table, seed, lo, hi, symmetric, r0, c0, b):
    """Rows r0..r0+b, columns c0..c0+b of the decay matrix drawn by the device
    generator (same counter-based draw, FP64 then FP32)."""
    i = np.arange(r0, r0 + b, dtype=np.int64)[:, None]
    j = np.arange(c0, c0 + b, dtype=np.int64)[None, :]
    ci, cj = (np.minimum(i, j), np.maximum(i, j)) if symmetric else (np.broadcast_to(i, (b, b)), np.broadcast_to(j, (b, b)))
    u = lo + (hi - lo) * si.uniform01(seed, ci, cj)
    return (table[np.abs(i - j)] * u).astype(np.float32)


def test_workload_32768_task_list():
    # algebraic decay p = 1.5, n = 32768, leaf 64 (nb = 512, 1.3e8 candidate
    # triples), tau = 1e-8: the complete kept-triple list bit-exact against the
    # oracle's flat enumeration of the stored leaf norms, with and without
    # statistics (full descent / flat-start cull); sampled leaf norms against
    # the host generator
    n, b, tau = 32768, 64, 1e-8
    print(f"[case] n={n} b={b} tau={tau} task list", flush=True)
    table = si.algebraic_table(n, 1.5)
    Ad = sp.generate_decay(table, 5, 0.5, 1.5, False)
    A = sp.build(Ad, b)
    del Ad
    S = A.norms(0)
    for I, K in ((0, 0), (511, 0), (300, 301), (17, 400)):
        blk = _host_block(table, 5, 0.5, 1.5, False, I * b, K * b, b)
        assert S[I, K] == oracle.tile_sqnorms(blk.astype(np.float64), b)[0, 0]
    keys, _ = oracle.tasks_flat(S, S, tau)
    C, st = sp.multiply(A, A, tau, "f32", stats=True)
    assert st["tasks"] == len(keys)
    assert np.array_equal(C.task_list(), keys)
    C2 = sp.multiply(A, A, tau, "f32")
    assert np.array_equal(C2.task_list(), keys)
    print(f"  T={len(keys)}", flush=True)


def test_workload_32768_sampled_rows():
    # the same operand at tau = 1e-8: C tile row 300 (kept K of its tiles
    # spread over both 256-K segments of the 512-K mask) with FP32 and FP16x3
    # leaves against one oracle evaluation of that row
    n, b, tau, I = 32768, 64, 1e-8, 300
    print(f"[case] n={n} b={b} tau={tau} tile row {I}", flush=True)
    Ad = sp.generate_decay(si.algebraic_table(n, 1.5), 5, 0.5, 1.5, False)
    A = sp.build(Ad, b)
    rs = slice(I * b, (I + 1) * b)
    outs = {}
    for prec in ("f32", "f16x3"):
        C = sp.multiply(A, A, tau, prec)
        outs[prec] = C.to_dense()[rs].cpu().numpy().copy()
        if prec == "f32":
            keys = C.task_list()
        del C
    Ii, Jj, Kk = oracle.unpack_keys(keys)
    row = Ii == I
    assert any(np.any(Kk[row & (Jj == j)] < 256) and np.any(Kk[row & (Jj == j)] >= 256) for j in range(512))
    a64 = Ad.cpu().numpy().astype(np.float64)
    del Ad, A
    full = {p: np.zeros((n, n), np.float32) for p in outs}   # lazily touched: only row I is written
    for p, o in outs.items():
        full[p][rs] = o
    worst = check_row_many(full, a64, b, tau, I)
    print(f"  worst/bound {worst}", flush=True)


def test_sp2_full_size_first_step():
    # SP2 at n = 16384, leaf 64, tau = 1e-6: step 0 from X_0 = (eps_max I - H) /
    # (eps_max - eps_min) built by the oracle (FP64, rounded to FP32): same task
    # count, branch and trace; three tile rows of X_1 against the oracle
    n, b, n_occ, tau = 16384, 64, 8192, 1e-6
    print(f"[case] sp2 n={n} first step", flush=True)
    for sym in (False, True):
        Hd = sp.generate_decay(-si.exp_table(n, 0.85), 0, 1.0, 1.0, False, "f32", si.sp2_diagonal(n, 4))
        H = sp.build(Hd, b)
        P1, log = sp.sp2(H, n_occ, tau, max_iter=1, idem_tol=0.0, symmetric=sym)
        h = Hd.cpu().numpy().astype(np.float64)
        del Hd
        x0 = osp2.initial_x(h).astype(np.float32).astype(np.float64)
        del h
        S = oracle.tile_sqnorms(x0, b)
        keys, _ = oracle.tasks_flat(S, S, tau)
        I, J, _ = oracle.unpack_keys(keys)
        T = int(np.sum(I <= J)) if sym else len(keys)
        assert log["tasks"][0] == T
        tr = float(np.trace(x0))
        assert abs(log["trace"][0] - tr) < 1e-9 * n
        br = 0 if tr > n_occ else 1
        assert log["branch"][0] == br
        x1 = P1.to_dense().cpu().numpy()
        for row in (0, 100, 255):
            y, _ = oracle.spamm_flat(x0, x0, b, tau, rows=(row, row + 1))
            rs = slice(row * b, (row + 1) * b)
            ref = y[rs] if br == 0 else 2.0 * x0[rs] - y[rs]
            assert np.max(np.abs(x1[rs].astype(np.float64) - ref)) < 1e-5
        del x0, x1
        print(f"  symmetric={sym} T={T} branch={br}", flush=True)


def test_sp2_full_size_gapped_converges():
    # the SP2 workload's H with its diagonal shifted by -10 on the first n/2
    # indices and +10 on the rest: the two halves' spectra (each about 13
    # wide) separate, a gap of about 3.5 opens at N_occ, and TC2 must drive
    # ||X^2 - X||_F below the tolerance at full size (n = 16384, leaf 64) with
    # trace N_occ; the energy at tau = 1e-6 matches the tau = 0 solve
    n, b, n_occ = 16384, 64, 8192
    print(f"[case] sp2 n={n} gapped convergence", flush=True)
    Hd = sp.generate_decay(-si.exp_table(n, 0.85), 0, 1.0, 1.0, False, "f32",
                           si.sp2_diagonal(n, 4, gap=20.0, n_occ=n_occ))
    H = sp.build(Hd, b)
    del Hd
    _, ref = sp.sp2(H, n_occ, 0.0, max_iter=60, idem_tol=1e-5, prec="f32")
    assert ref["converged"] and ref["status"] == "OK"
    for prec in ("f32", "f16x3"):
        P, lg = sp.sp2(H, n_occ, 1e-6, max_iter=60, idem_tol=1e-5, prec=prec)
        print(f"  {prec}: {lg['iterations']} steps, idem {lg['idem'][-1]:.3e}, trace {lg['final_trace']:.6f}, "
              f"E {lg['energy']:.10g} (tau = 0: {ref['energy']:.10g}), products/step {np.mean(lg['tasks']):.0f}",
              flush=True)
        assert lg["converged"] and not lg["stagnated"] and lg["status"] == "OK"
        assert lg["iterations"] < 60
        assert lg["idem"][-1] <= 1e-5
        assert abs(lg["final_trace"] - n_occ) < 1e-3
        assert abs(lg["energy"] - ref["energy"]) < 1e-7 * abs(ref["energy"])
        assert max(lg["tasks"]) < 0.01 * (n // b) ** 3
        del P


def test_batched_full_64_task_lists():
    # the 64-matrix batch (n ~ U{512..8192}, exponential decay, tau = 1e-6): one
    # batched build and one batched product with the list schedule; every
    # product's kept-triple list against the oracle's flat enumeration of its
    # stored norms, and a leaf norm of each matrix against the host generator
    params = si.batch_params()
    print(f"[case] batched 64 full, sum n^2 = {sum(n * n for n, _, _ in params):.3e}", flush=True)
    dense = [sp.generate_decay(si.exp_table(n, lam), useed, -1.0, 1.0, True) for n, lam, useed in params]
    hs = sp.build_batched(dense, 64)
    # values: one C tile row of the largest, the smallest and two middle products
    order = np.argsort([n for n, _, _ in params])
    sample = [int(order[-1]), int(order[0]), int(order[20]), int(order[40])]
    kept_dense = {m: dense[m].cpu().numpy().astype(np.float64) for m in sample}
    del dense
    Cs, sts = sp.multiply_batched(hs, hs, [1e-6] * len(hs), "f32", stats=True, schedule="list")
    for m in sample:
        a64 = kept_dense[m]
        I = (a64.shape[0] // 64) // 2
        w = check_row_many({"f32": Cs[m].to_dense().cpu().numpy()}, a64, 64, 1e-6, I)
        print(f"  product {m} n={a64.shape[0]} row {I} worst/bound {w['f32']:.2e}", flush=True)
    del kept_dense
    total = 0
    for (n, lam, useed), h, C, st in zip(params, hs, Cs, sts):
        S = h.norms(0)
        nb = S.shape[0]
        I = nb // 2
        blk = _host_block(si.exp_table(n, lam), useed, -1.0, 1.0, True, I * 64, I * 64, 64)
        assert S[I, I] == oracle.tile_sqnorms(blk.astype(np.float64), 64)[0, 0]
        keys, _ = oracle.tasks_flat(S, S, 1e-6)
        assert st["tasks"] == len(keys)
        assert np.array_equal(C.task_list(), keys)
        total += len(keys)
    print(f"  T={total}", flush=True)
