"""Pins of the oracle's TC2/SP2 purification against LAPACK's spectral projector."""
import numpy as np
import pytest

import spamm_inputs as si
from oracle import sp2


@pytest.mark.parametrize("n,gap", [(256, 4.0), (192, 0.0)])
def test_sp2_matches_eigh_projector(n, gap):
    # P = theta[mu I - H] with n_occ states occupied: the projector onto the
    # n_occ lowest eigenvectors (section 3; TC2 drives eigenvalues to 0 or 1).
    n_occ = n // 2
    h = si.sp2_hamiltonian(n, 0.85, 4, np.float64, gap=gap)
    P, log = sp2.sp2(h, n_occ, 16, 0.0, max_iter=100, tol=1e-9)
    w, v = np.linalg.eigh(h)
    pe = v[:, :n_occ] @ v[:, :n_occ].T
    assert log["converged"]
    assert np.max(np.abs(P - pe)) < 1e-8
    assert abs(np.trace(P) - n_occ) < 1e-8
    assert np.linalg.norm(P @ P - P) < 1e-8
    assert np.linalg.norm(P @ h - h @ P) < 1e-7
    assert abs(log["energy"] - w[:n_occ].sum()) < 1e-8 * abs(w[:n_occ].sum())


def test_sp2_iteration_count_in_paper_range():
    # 40-60 multiplies per solve for realistic problems (section 3)
    h = si.sp2_hamiltonian(256, 0.85, 4, np.float64)
    _, log = sp2.sp2(h, 128, 16, 0.0, max_iter=100, tol=1e-9)
    assert 30 <= log["iterations"] <= 70


def test_sp2_initial_spectrum_in_unit_interval():
    h = si.sp2_hamiltonian(128, 0.85, 5, np.float64)
    lo, hi = sp2.gershgorin(h)
    w = np.linalg.eigvalsh(h)
    assert lo <= w[0] and w[-1] <= hi
    wx = np.linalg.eigvalsh(sp2.initial_x(h))
    assert wx[0] >= -1e-12 and wx[-1] <= 1 + 1e-12


def test_sp2_branch_rule():
    # the trace above n_occ takes X^2 (trace decreases), otherwise 2X - X^2
    h = si.sp2_hamiltonian(128, 0.85, 6, np.float64)
    x = sp2.initial_x(h)
    for _ in range(6):
        x2, tr, _, br, _ = sp2.step(x, 64, 16, 0.0)
        assert br == (0 if tr > 64 else 1)
        if br == 0:
            assert np.trace(x2) <= tr + 1e-9
        else:
            assert np.trace(x2) >= tr - 1e-9
        x = x2


def test_sp2_with_truncation_energy_error_small():
    # SpAMM at tau > 0 inside TC2: the energy error is controlled and shrinks
    # with tau, while the leaf work drops well below the tau = 0 run (section 3)
    h = si.sp2_hamiltonian(256, 0.85, 4, np.float64)
    _, log0 = sp2.sp2(h, 128, 16, 0.0, 80, 1e-9)
    errs = []
    for tau in (1e-4, 1e-6, 1e-8):
        _, log1 = sp2.sp2(h, 128, 16, tau, 80, 1e-9)
        assert log1["stagnated"] and not log1["converged"]
        assert abs(log1["final_trace"] - 128) < 1e-3
        errs.append(abs(log1["energy"] - log0["energy"]) / abs(log0["energy"]))
        assert sum(log1["tasks"]) < 0.5 * sum(log0["tasks"])
    assert errs[0] < 1e-5 and errs[1] < 1e-7 and errs[2] < 1e-9
    assert errs[2] < errs[1] < errs[0]


def test_sp2_stagnation_stops_divergence():
    # without the stagnation stop the trace rule keeps squaring and the
    # idempotency error doubles each step; with it the result stays idempotent
    h = si.sp2_hamiltonian(256, 0.85, 4, np.float64)
    P, log = sp2.sp2(h, 128, 16, 1e-6, 80, 1e-12)
    assert log["stagnated"] and log["iterations"] < 80
    assert np.linalg.norm(P @ P - P) < 1e-4


# ---------------------------------------------------------------- symmetric squaring
# For X = X^T the squaring can form the tiles I <= J by the flat rule and
# mirror the rest (C_JI = C_IJ^T).  These pins do not use that code path.

def _int_sym(n, seed):
    # small-integer symmetric decaying matrix: every tile norm and every product
    # is an exact FP64 integer, so keep sets and products are exactly symmetric
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    base = np.round(40.0 * 0.8 ** np.abs(i[:, None] - i[None, :]))
    u = rng.integers(1, 4, (n, n)).astype(np.float64)
    u = np.triu(u) + np.triu(u, 1).T
    return base * u


@pytest.mark.parametrize("n,b,tau", [(96, 8, 50.0), (130, 16, 300.0), (64, 16, 0.0)])
def test_sym_square_equals_general_rule_on_exact_inputs(n, b, tau):
    # catches: lower tiles formed instead of mirrored (T too big), a missed
    # upper tile or the diagonal tiles left out, the transpose of the mirror
    # taken the wrong way round (wrong values below the diagonal)
    from oracle import spamm_flat, tasks_flat, tile_sqnorms, unpack_keys
    x = _int_sym(n, 7)
    c_sym, t_sym = spamm_flat(x, x, b, tau, sym_upper=True)
    c_gen, t_gen = spamm_flat(x, x, b, tau)
    assert np.array_equal(c_sym, c_gen)
    S = tile_sqnorms(x, b)
    keys, _ = tasks_flat(S, S, tau)
    I, J, _ = unpack_keys(keys)
    assert t_sym == int(np.sum(I <= J)) and t_gen == len(keys)
    if tau == 0.0:
        assert np.array_equal(c_sym, x @ x)        # integers: exact either way


def test_sym_square_result_is_symmetric_and_near_the_general_rule():
    from oracle import spamm_flat
    x = si.exp_decay(300, 0.9, 3)                   # symmetric FP64
    for tau in (1e-3, 1e-6):
        c_sym, _ = spamm_flat(x, x, 32, tau, sym_upper=True)
        c_gen, _ = spamm_flat(x, x, 32, tau)
        i = np.arange(300)
        lower = (i[:, None] // 32) > (i[None, :] // 32)      # elements of tiles I > J
        assert np.array_equal(c_sym[lower], c_sym.T[lower])
        absx = np.abs(x)
        assert np.all(np.abs(c_sym - c_gen) <= 64 * 2.0 ** -53 * (absx @ absx) + 1e-300)


def test_sp2_symmetric_squarings_match_eigh_projector():
    n, n_occ = 256, 128
    h = si.sp2_hamiltonian(n, 0.85, 4, np.float64, gap=4.0)
    P, log = sp2.sp2(h, n_occ, 16, 0.0, max_iter=100, tol=1e-9, symmetric=True)
    w, v = np.linalg.eigh(h)
    pe = v[:, :n_occ] @ v[:, :n_occ].T
    assert log["converged"]
    assert np.max(np.abs(P - pe)) < 1e-8
    assert abs(log["energy"] - w[:n_occ].sum()) < 1e-8 * abs(w[:n_occ].sum())
    assert log["tasks"][0] < (n // 16) ** 3        # only the upper tiles are formed
