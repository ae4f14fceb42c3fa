"""GPU TC2/SP2 purification (hipGraph) against the FP64 oracle and LAPACK."""
import numpy as np
import pytest

import oracle
import spamm_inputs as si
from gpu_util import to_dev
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


@pytest.mark.parametrize("prec", ["f32", "f16x3", "bf16x3"])
def test_sp2_projector_matches_eigh(prec):
    print(f"[case] sp2 vs eigh prec={prec}", flush=True)
    n, b, n_occ = 512, 32, 256
    h = si.sp2_hamiltonian(n, 0.85, 4, np.float32, gap=4.0)
    H = sp.build(to_dev(h), b)
    P, log = sp.sp2(H, n_occ, 0.0, max_iter=100, idem_tol=1e-6, prec=prec)
    assert log["status"] == "OK" and (log["converged"] or log["stagnated"])
    w, v = np.linalg.eigh(h.astype(np.float64))
    pe = v[:, :n_occ] @ v[:, :n_occ].T
    pd = P.to_dense().cpu().numpy().astype(np.float64)
    # FP32 purification: the converged projector carries ~10 u sqrt(n) (1.4e-5) elementwise;
    # BF16x3 leaves add 3 * 2^-16 (4.6e-5) per product term, and the iteration stops
    # (stagnates) about five of those units from the projector
    tol = 1e-3 if prec == "bf16x3" else 5e-5
    assert np.max(np.abs(pd - pe)) < tol
    assert abs(np.trace(pd) - n_occ) < 1e-3
    assert abs(log["final_trace"] - np.trace(pd)) < 1e-6 * n
    assert abs(log["energy"] - w[:n_occ].sum()) < 1e-5 * abs(w[:n_occ].sum())
    assert abs(log["eps_min"] - osp2.gershgorin(h)[0]) < 1e-12
    assert abs(log["eps_max"] - osp2.gershgorin(h)[1]) < 1e-12
    assert 10 <= log["iterations"] <= 100


def test_sp2_step_replay_matches_oracle():
    # feed the GPU's stored X_k into one oracle step: same norms -> same kept
    # triples (count), same branch; trace, idempotency and X_{k+1} agree
    n, b, n_occ, tau = 384, 32, 192, 1e-5
    h = si.sp2_hamiltonian(n, 0.85, 7, np.float32)
    H = sp.build(to_dev(h), b)
    for k in (1, 6, 15):
        print(f"[case] sp2 replay k={k}", flush=True)
        Pk, logk = sp.sp2(H, n_occ, tau, max_iter=k, idem_tol=0.0)
        assert logk["status"] == "ENOCONV" and logk["result_step"] == k
        xk = Pk.to_dense().cpu().numpy().astype(np.float64)
        Pk1, logk1 = sp.sp2(H, n_occ, tau, max_iter=k + 1, idem_tol=0.0)
        x_next, tr, idem, br, T = osp2.step(xk, n_occ, b, tau)
        assert logk1["tasks"][k] == T
        assert logk1["branch"][k] == br
        assert abs(logk1["trace"][k] - tr) < 1e-9 * n
        assert abs(logk1["idem"][k] - idem) < 1e-5 * max(idem, 1.0)
        got = Pk1.to_dense().cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - x_next)) < 1e-5
        # the k-step prefix of the log is reproduced exactly
        assert logk1["tasks"][:k] == logk["tasks"][:k]
        assert logk1["idem"][:k] == logk["idem"][:k]


def test_sp2_first_step_from_gershgorin():
    # step 0 from X_0 = (eps_max I - H)/(eps_max - eps_min), built by the oracle in FP64
    n, b, n_occ, tau = 256, 32, 128, 1e-6
    h = si.sp2_hamiltonian(n, 0.85, 9, np.float32)
    H = sp.build(to_dev(h), b)
    P1, log = sp.sp2(H, n_occ, tau, max_iter=1, idem_tol=0.0)
    x0 = osp2.initial_x(h.astype(np.float64)).astype(np.float32).astype(np.float64)
    x1, tr, idem, br, T = osp2.step(x0, n_occ, b, tau)
    assert log["tasks"][0] == T and log["branch"][0] == br
    assert abs(log["trace"][0] - tr) < 1e-9 * n
    assert np.max(np.abs(P1.to_dense().cpu().numpy() - x1)) < 1e-5


def test_sp2_invalid_arguments():
    h = si.sp2_hamiltonian(128, 0.85, 4, np.float32)
    H = sp.build(to_dev(h), 32)
    for kw in ({"n_occ": 129}, {"n_occ": -1}, {"max_iter": 0}, {"max_iter": 257}):
        args = {"n_occ": 64, "tau": 1e-6, "max_iter": 10}
        args.update(kw)
        with pytest.raises(sp.SpammError, match="EINVAL"):
            sp.sp2(H, **args)
    H64 = sp.build(to_dev(h.astype(np.float64)), 32)
    with pytest.raises(sp.SpammError, match="EUNSUPPORTED"):
        sp.sp2(H64, 64, 1e-6)


def test_sp2_truncated_energy_close_to_exact():
    # tau > 0 inside TC2: energy error small and leaf work well below tau = 0
    n, b, n_occ = 1024, 64, 512
    h = si.sp2_hamiltonian(n, 0.85, 4, np.float32)
    H = sp.build(to_dev(h), b)
    _, log0 = sp.sp2(H, n_occ, 0.0, max_iter=80, idem_tol=1e-6)
    _, log1 = sp.sp2(H, n_occ, 1e-5, max_iter=80, idem_tol=1e-6)
    rel = abs(log1["energy"] - log0["energy"]) / abs(log0["energy"])
    print(f"[case] sp2 tau=1e-5 dE={rel:.2e} iters={log1['iterations']} vs {log0['iterations']}", flush=True)
    assert rel < 1e-5
    assert sum(log1["tasks"]) < 0.7 * sum(log0["tasks"])


# ------------------------------------------------------------------ symmetric squarings

def test_sp2_symmetric_step_replay_matches_oracle():
    # symmetric squarings: tiles I <= J formed, the others mirrored.  The GPU's
    # stored X_k fed to the oracle's symmetric step gives the same task count
    # and branch; trace, idempotency and X_{k+1} agree
    n, b, n_occ, tau = 384, 32, 192, 1e-5
    h = si.sp2_hamiltonian(n, 0.85, 7, np.float32)
    H = sp.build(to_dev(h), b)
    for k in (1, 6, 15):
        print(f"[case] symmetric sp2 replay k={k}", flush=True)
        Pk, logk = sp.sp2(H, n_occ, tau, max_iter=k, idem_tol=0.0, symmetric=True)
        assert logk["status"] == "ENOCONV" and logk["result_step"] == k
        xk = Pk.to_dense().cpu().numpy().astype(np.float64)
        Pk1, logk1 = sp.sp2(H, n_occ, tau, max_iter=k + 1, idem_tol=0.0, symmetric=True)
        x_next, tr, idem, br, T = osp2.step(xk, n_occ, b, tau, symmetric=True)
        assert logk1["tasks"][k] == T
        assert logk1["branch"][k] == br
        assert abs(logk1["trace"][k] - tr) < 1e-9 * n
        assert abs(logk1["idem"][k] - idem) < 1e-5 * max(idem, 1.0)
        x1 = Pk1.to_dense().cpu().numpy().astype(np.float64)
        assert np.max(np.abs(x1 - x_next)) < 1e-5


@pytest.mark.parametrize("prec", ["f32", "f16x3"])
def test_sp2_symmetric_projector_exact_mirror(prec):
    print(f"[case] symmetric sp2 vs eigh prec={prec}", flush=True)
    n, b, n_occ = 512, 32, 256
    h = si.sp2_hamiltonian(n, 0.85, 4, np.float32, gap=4.0)
    H = sp.build(to_dev(h), b)
    P, log = sp.sp2(H, n_occ, 1e-7, max_iter=100, idem_tol=1e-6, prec=prec, symmetric=True)
    _, log_g = sp.sp2(H, n_occ, 1e-7, max_iter=100, idem_tol=1e-6, prec=prec)
    assert log["status"] == "OK" and (log["converged"] or log["stagnated"])
    w, v = np.linalg.eigh(h.astype(np.float64))
    pe = v[:, :n_occ] @ v[:, :n_occ].T
    pd = P.to_dense().cpu().numpy()
    assert np.max(np.abs(pd.astype(np.float64) - pe)) < 5e-5
    assert abs(log["energy"] - w[:n_occ].sum()) < 1e-5 * abs(w[:n_occ].sum())
    i = np.arange(n)
    lower = (i[:, None] // b) > (i[None, :] // b)
    assert np.array_equal(pd[lower], pd.T[lower])          # mirrored tiles, bit for bit
    # the stored pyramid is that of the stored values, mirrored tiles included
    for lv, r in enumerate(oracle.norm_pyramid(pd.astype(np.float64), b)):
        assert np.array_equal(P.norms(lv), r)
    assert log["tasks"][0] < 0.6 * log_g["tasks"][0]       # about half the products


def test_sp2_symmetric_rejects_unsymmetric_h():
    print("[case] symmetric sp2 EINVAL", flush=True)
    h = si.sp2_hamiltonian(256, 0.85, 4, np.float32)
    h[3, 70] += 1e-3
    H = sp.build(to_dev(h), 32)
    with pytest.raises(sp.SpammError, match="EINVAL"):
        sp.sp2(H, 128, 1e-6, max_iter=5, symmetric=True)
    P, log = sp.sp2(H, 128, 1e-6, max_iter=5)              # the general squaring still runs
    assert log["iterations"] == 5


@pytest.mark.parametrize("tau_d", [1e-3, 1e-5])
def test_sp2_dropping_step_replay_matches_oracle(tau_d):
    # the dropping scheme (section 3, scheme I): feed the GPU's stored X_k
    # into one oracle dropping step; the pairs of present tiles are the same
    # (exact count), as are the branch, trace and idempotency, and the tiles
    # dropped from X_{k+1} (those whose norm is not within rounding of tau)
    n, b, n_occ = 512, 32, 256
    h = si.sp2_hamiltonian(n, 0.85, 7, np.float32)
    H = sp.build(to_dev(h), b)
    for k in (1, 5, 12):
        print(f"[case] sp2 dropping replay tau_d={tau_d} k={k}", flush=True)
        Pk, logk = sp.sp2(H, n_occ, tau_d, max_iter=k, idem_tol=0.0, dropping=True)
        assert logk["status"] == "ENOCONV" and logk["result_step"] == k
        xk = Pk.to_dense().cpu().numpy().astype(np.float64)
        Pk1, logk1 = sp.sp2(H, n_occ, tau_d, max_iter=k + 1, idem_tol=0.0, dropping=True)
        x_next, tr, idem, br, T = osp2.step_dropping(xk, n_occ, b, tau_d)
        assert logk1["tasks"][k] == T
        assert logk1["branch"][k] == br
        assert abs(logk1["trace"][k] - tr) < 1e-9 * n
        assert abs(logk1["idem"][k] - idem) < 1e-5 * max(idem, 1.0)
        got = Pk1.to_dense().cpu().numpy().astype(np.float64)
        S_or = oracle.tile_sqnorms(x_next, b)
        S_gpu = Pk1.norms(0)
        clear = np.abs(np.sqrt(oracle.tile_sqnorms(osp2.step(xk, n_occ, b, 0.0)[0], b)) - tau_d) > 1e-3 * tau_d
        assert np.array_equal((S_gpu == 0.0)[clear], (S_or == 0.0)[clear])
        assert np.all(S_gpu[S_or == 0.0][clear[S_or == 0.0]] == 0.0)
        elem_clear = np.kron(clear, np.ones((b, b), dtype=bool))[:n, :n]
        assert np.max(np.abs(got - x_next)[elem_clear]) < 1e-5


def test_sp2_dropping_solve_matches_oracle():
    # a whole dropping-scheme solve against the oracle's; at tau = 0 no tile
    # is dropped and every squaring counts all nb^3 pairs, as exact TC2
    n, b, n_occ = 512, 32, 256
    h = si.sp2_hamiltonian(n, 0.85, 4, np.float32, gap=2.0, n_occ=n_occ)
    H = sp.build(to_dev(h), b)
    h64 = h.astype(np.float64)
    print("[case] sp2 dropping solve tau_d=0", flush=True)
    P0, log0 = sp.sp2(H, n_occ, 0.0, max_iter=100, idem_tol=1e-6, dropping=True)
    assert log0["status"] == "OK"
    assert all(t == (n // b) ** 3 for t in log0["tasks"][:log0["iterations"]])
    _, logx = sp.sp2(H, n_occ, 0.0, max_iter=100, idem_tol=1e-6)
    assert abs(log0["energy"] - logx["energy"]) < 1e-6 * abs(logx["energy"])
    for tau_d in (1e-2, 1e-4):
        print(f"[case] sp2 dropping solve tau_d={tau_d}", flush=True)
        P, log = sp.sp2(H, n_occ, tau_d, max_iter=100, idem_tol=1e-6, dropping=True)
        _, lo = osp2.sp2_dropping(h64, n_occ, b, tau_d, max_iter=100, tol=1e-6)
        assert log["status"] == "OK"
        assert abs(log["energy"] - lo["energy"]) < 1e-5 * abs(lo["energy"])
        k = min(log["iterations"], lo["iterations"])
        assert abs(np.mean(log["tasks"][:k]) - np.mean(lo["tasks"][:k])) <= 0.01 * np.mean(lo["tasks"][:k])
    with pytest.raises(sp.SpammError) as e:
        sp.sp2(H, n_occ, 1e-4, max_iter=4, symmetric=True, dropping=True)
    assert e.value.status == "EUNSUPPORTED"
