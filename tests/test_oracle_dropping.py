"""Pins of the oracle's block-dropping TC2 (section 3, scheme I): leaf
products counted over present blocks only, the filter of the iterate by
block Frobenius norm, equality with exact TC2 at tau = 0, and block-diagonal
Hamiltonians whose counts and energies are known in closed form."""
import itertools

import numpy as np
import pytest

import oracle
import spamm_inputs as si
from oracle import sp2


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_present_count_is_the_number_of_present_pairs(seed):
    rng = np.random.default_rng(seed)
    nb = 7
    S = rng.random((nb, nb)) * (rng.random((nb, nb)) < 0.45)
    S[3, :] = 0.0          # an empty block row and column
    S[:, 5] = 0.0
    brute = sum(1 for I, J, K in itertools.product(range(nb), repeat=3) if S[I, K] > 0 and S[K, J] > 0)
    assert sp2.present_count(S) == brute
    assert sp2.present_count(np.ones((nb, nb))) == nb ** 3
    assert sp2.present_count(np.zeros((nb, nb))) == 0
    assert sp2.present_count(np.eye(nb)) == nb


@pytest.mark.parametrize("n,b", [(96, 16), (100, 16)])
def test_drop_filter_zeroes_exactly_the_small_blocks(n, b):
    # block (I, J) scaled by 10^-(I+J); tau halfway (in log) between scales,
    # so the dropped set is the blocks with I + J >= 4, by numpy's own norm
    rng = np.random.default_rng(3)
    nb = -(-n // b)
    x = rng.uniform(-1, 1, (n, n))
    for I in range(nb):
        for J in range(nb):
            x[I * b:(I + 1) * b, J * b:(J + 1) * b] *= 10.0 ** -(I + J)
    tau = 10.0 ** -3.5 * b / 2
    y, drop = sp2.drop_filter(x, b, tau)
    for I in range(nb):
        for J in range(nb):
            blk = (slice(I * b, min((I + 1) * b, n)), slice(J * b, min((J + 1) * b, n)))
            small = np.linalg.norm(x[blk]) < tau
            assert drop[I, J] == small
            if small:
                assert np.all(y[blk] == 0.0)
            else:
                assert np.array_equal(y[blk], x[blk])
    assert drop.any() and not drop.all()


def test_dropping_at_zero_threshold_is_exact_tc2():
    # tau = 0 drops nothing: the same iterates, logs and energy as exact TC2;
    # a dense H keeps every block, so each multiply counts nb^3 products
    n, b, n_occ = 128, 16, 64
    h = si.sp2_hamiltonian(n, 0.85, 4, np.float64, gap=2.0, n_occ=n_occ)
    P0, log0 = sp2.sp2(h, n_occ, b, 0.0, max_iter=80, tol=1e-9)
    Pd, logd = sp2.sp2_dropping(h, n_occ, b, 0.0, max_iter=80, tol=1e-9)
    assert np.array_equal(P0, Pd)
    for key in ("trace", "idem", "branch", "iterations", "energy"):
        assert log0[key] == logd[key]
    assert all(t == (n // b) ** 3 for t in logd["tasks"])


def _block_diagonal_h(nblk, b, seed):
    rng = np.random.default_rng(seed)
    n = nblk * b
    h = np.zeros((n, n))
    for I in range(nblk):
        m = rng.normal(size=(b, b))
        h[I * b:(I + 1) * b, I * b:(I + 1) * b] = (m + m.T) / 2 + np.diag(np.linspace(-3, 3, b))
    return h


@pytest.mark.parametrize("tau", [0.0, 1e-6, 1e-3])
def test_block_diagonal_h_keeps_its_blocks(tau):
    # H with zero blocks off the diagonal: every iterate stays block diagonal,
    # so each multiply counts exactly nb products (one per diagonal block) and
    # no diagonal block is ever small; TC2 converges to the spectral
    # projector, E = the sum of the n_occ lowest eigenvalues
    nblk, b = 6, 16
    h = _block_diagonal_h(nblk, b, 7)
    w, v = np.linalg.eigh(h)
    n_occ = int(np.searchsorted(w, 0.5 * (w[47] + w[48]))) if w[48] - w[47] > 1e-3 else 48
    P, log = sp2.sp2_dropping(h, n_occ, b, tau, max_iter=120, tol=1e-9)
    assert log["converged"]
    assert all(t == nblk for t in log["tasks"])
    pe = v[:, :n_occ] @ v[:, :n_occ].T
    assert np.max(np.abs(P - pe)) < 1e-7
    assert abs(log["energy"] - w[:n_occ].sum()) < 1e-8 * abs(w[:n_occ].sum())


def test_dropping_error_and_work_fall_and_rise_with_tau():
    # larger drop thresholds remove more blocks: fewer leaf products on
    # average, a larger energy error (against exact TC2)
    n, b, n_occ = 256, 16, 128
    h = si.sp2_hamiltonian(n, 0.85, 4, np.float64, gap=1.0, n_occ=n_occ)
    _, log0 = sp2.sp2(h, n_occ, b, 0.0, max_iter=100, tol=1e-9)
    errs, work = [], []
    for tau in (1e-2, 1e-4, 1e-6):
        _, lg = sp2.sp2_dropping(h, n_occ, b, tau, max_iter=100, tol=1e-9)
        errs.append(abs(lg["energy"] - log0["energy"]) / abs(log0["energy"]))
        work.append(np.mean(lg["tasks"]))
    assert work[0] < work[1] < work[2] <= (n // b) ** 3
    assert errs[0] > errs[2]
