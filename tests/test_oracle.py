"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names the plausible oracle mistake it would catch.  None of them
re-types the oracle's own formula: they use numpy/closed forms/exact cases.
"""
import numpy as np
import pytest

import oracle
import spamm_inputs as si

U64 = 2.0 ** -53


def _rand(n, seed, sym=False):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, (n, n))
    return (a + a.T) / 2 if sym else a


# ---------------------------------------------------------------- norms (Eq. 1, section 3)

@pytest.mark.parametrize("n,b", [(64, 16), (100, 16), (128, 32), (96, 64), (5, 4)])
def test_tile_sqnorms_match_numpy(n, b):
    # catches: wrong tile indexing (I,K swapped), a missed row/column, padding leaking in
    a = _rand(n, n + b)
    a[0, -1] = 7.0                      # make the matrix clearly non-symmetric
    S = oracle.tile_sqnorms(a, b)
    nb = -(-n // b)
    assert S.shape == (nb, nb)
    for I in range(nb):
        for K in range(nb):
            ref = float(np.sum(a[I * b:(I + 1) * b, K * b:(K + 1) * b] ** 2))
            assert abs(S[I, K] - ref) <= 2 * b * b * U64 * ref


def test_tile_sqnorm_exact_cases():
    b = 32
    ones = np.ones((b, b))
    assert oracle.tile_sqnorms(ones, b)[0, 0] == b * b
    single = np.zeros((b, b))
    single[5, 17] = -3.0
    assert oracle.tile_sqnorms(single, b)[0, 0] == 9.0
    # powers of two on distinct columns sum exactly
    p2 = np.zeros((b, b))
    p2[0, :] = 2.0 ** -np.arange(b)
    assert oracle.tile_sqnorms(p2, b)[0, 0] == float(np.sum(4.0 ** -np.arange(b)))


def test_norm_parent_and_root():
    # catches: a dropped child, wrong child index, odd-size (absent child) handling
    rng = np.random.default_rng(3)
    S = rng.integers(0, 1000, (7, 7)).astype(np.float64)   # integers: all sums exact
    P = oracle.norm_parent(S)
    assert P.shape == (4, 4)
    Sp = np.zeros((8, 8))
    Sp[:7, :7] = S
    ref = Sp.reshape(4, 2, 4, 2).sum(axis=(1, 3))
    assert np.array_equal(P, ref)
    levels = oracle.norm_pyramid(_rand(200, 1), 16)
    assert [lv.shape[0] for lv in levels] == [13, 7, 4, 2, 1]
    total = float(np.sum(_rand(200, 1) ** 2))
    assert abs(levels[-1][0, 0] - total) <= 1e-12 * total
    for lo, hi in zip(levels, levels[1:]):             # monotone up the tree
        m = hi.shape[0]
        for I in range(lo.shape[0]):
            for K in range(lo.shape[0]):
                assert hi[I // 2, K // 2] >= lo[I, K]
        assert m == -(-lo.shape[0] // 2)


# ---------------------------------------------------------------- tau = 0: the dense product

@pytest.mark.parametrize("n,b", [(64, 16), (100, 16), (130, 32)])
def test_tau0_is_dense_product(n, b):
    # catches: transposed operand, wrong K range, dropped tile, padded garbage
    a, bm = _rand(n, 10), _rand(n, 11)
    c, T, _, _ = oracle.spamm_recursive(a, bm, b, 0.0)
    nb = -(-n // b)
    assert T == nb ** 3                      # tau = 0 keeps every triple (section 3)
    ref = a @ bm
    gamma = n * U64 / (1 - n * U64)
    bound = 2 * gamma * (np.abs(a) @ np.abs(bm))
    assert np.all(np.abs(c - ref) <= bound)


def test_tau0_keeps_zero_tiles():
    # 0 < 0 is false: zero-norm tiles are still multiplied at tau = 0
    a = np.zeros((64, 64))
    a[:16, :16] = 1.0
    _, T, _, _ = oracle.spamm_recursive(a, a, 16, 0.0)
    assert T == 4 ** 3
    _, T, _, _ = oracle.spamm_recursive(a, a, 16, 1e-300 ** 0.5)
    assert T == 1


def _kms_product(n, r1, r2):
    """Closed form of (A B)_ij for A_ij = r1^|i-j|, B_ij = r2^|i-j| (geometric sums)."""
    def geo(q, lo, hi):                      # sum_{m=lo}^{hi} q^m, empty if hi < lo
        if hi < lo:
            return 0.0
        if abs(q - 1.0) < 1e-15:
            return float(hi - lo + 1)
        return (q ** lo - q ** (hi + 1)) / (1.0 - q)
    c = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            if i <= j:
                # k <= i: r1^(i-k) r2^(j-k);  i < k < j: r1^(k-i) r2^(j-k);  k >= j: r1^(k-i) r2^(k-j)
                s = r2 ** (j - i) * geo(r1 * r2, 0, i)
                s += r2 ** (j - i) * geo(r1 / r2, 1, j - i - 1) if j - i >= 2 else 0.0
                if j > i:
                    s += r1 ** (j - i) * geo(r1 * r2, 0, n - 1 - j)
                else:
                    s += geo(r1 * r2, 1, n - 1 - j)
            else:
                # k <= j: r1^(i-k) r2^(j-k);  j < k < i: r1^(i-k) r2^(k-j);  k >= i: r1^(k-i) r2^(k-j)
                s = r1 ** (i - j) * geo(r1 * r2, 0, j)
                s += r1 ** (i - j) * geo(r2 / r1, 1, i - j - 1) if i - j >= 2 else 0.0
                s += r2 ** (i - j) * geo(r1 * r2, 0, n - 1 - i)
            c[i, j] = s
    return c


def test_figure1_case_a_closed_form():
    # Figure 1 (A): A = exp(-|i-j|), B = exp(-2|i-j|); at tau = 0 the product is
    # the closed-form geometric sum.  Catches operand swaps (A B != B A here).
    n = 96
    a, bm = si.figure1_pair(n, "A")
    c, _, _, _ = oracle.spamm_recursive(a, bm, 16, 0.0)
    ref = _kms_product(n, np.exp(-1.0), np.exp(-2.0))
    assert np.max(np.abs(c - ref)) < 1e-14
    assert np.max(np.abs(ref - _kms_product(n, np.exp(-2.0), np.exp(-1.0)).T)) < 1e-14


def test_figure1_truncation_counts_shrink():
    # Figure 1 setting: n = 512, tau = 1e-8.  Both pairs prune most of the
    # product space; the fast exponential pair prunes more than 1/|i-j|^3.
    counts = {}
    for case in "AB":
        a, bm = si.figure1_pair(512, case)
        sa, sb = oracle.tile_sqnorms(a, 16), oracle.tile_sqnorms(bm, 16)
        T, kept = oracle.count_hierarchical(sa, sb, 1e-8)
        counts[case] = T
        assert kept[-1] == 1 and T < 32 ** 3
    assert counts["A"] < counts["B"]


# ---------------------------------------------------------------- the keep rule (Eq. 4)

def test_identity_operand_exact():
    # A = I: only diagonal leaves have norm (S = b); C~_IJ = B_IJ iff b*S_B[I,J] >= tau^2.
    # Catches: S_A/S_B index mix-ups (S_B[J,K] instead of S_B[K,J]) and sign errors.
    n, b = 128, 16
    rng = np.random.default_rng(4)
    bm = rng.uniform(-1, 1, (n, n)) * (10.0 ** rng.integers(-6, 1, (n // b, n // b))).repeat(b, 0).repeat(b, 1)
    a = np.eye(n)
    tau = 1e-3
    c, T, _, _ = oracle.spamm_recursive(a, bm, b, tau)
    expect = np.zeros_like(bm)
    t_expect = 0
    for I in range(n // b):
        for J in range(n // b):
            tile = bm[I * b:(I + 1) * b, J * b:(J + 1) * b]
            if b * np.sum(tile ** 2) >= tau ** 2 * (1 + 1e-9):
                expect[I * b:(I + 1) * b, J * b:(J + 1) * b] = tile
                t_expect += 1
    assert T == t_expect
    assert np.array_equal(c, expect)


def test_tie_is_kept():
    # ||A|| ||B|| == tau exactly: the strict "<" of Eq. (4) keeps the product.
    b = 4
    a = np.zeros((8, 8))
    bm = np.zeros((8, 8))
    a[0, 0] = 2.0        # S_A[0,0] = 4
    bm[0, 0] = 4.0       # S_B[0,0] = 16  ->  S_A S_B = 64 = 8^2
    _, T, _, _ = oracle.spamm_recursive(a, bm, b, 8.0)
    assert T == 1
    _, T, _, _ = oracle.spamm_recursive(a, bm, b, 8.0 * (1 + 2 ** -50))
    assert T == 0


def test_keep_set_matches_independent_norms():
    # keep(I,J,K) <=> ||A_IK||_F ||B_KJ||_F >= tau, with the norms from numpy;
    # tau chosen away from every product value so rounding cannot decide.
    n, b = 160, 16
    a = si.exp_decay(n, 0.8, 21, np.float64, symmetric=False)
    bm = si.algebraic_decay(n, 2.0, 22, np.float64)
    nb = n // b
    na = np.array([[np.linalg.norm(a[I*b:(I+1)*b, K*b:(K+1)*b]) for K in range(nb)] for I in range(nb)])
    nbm = np.array([[np.linalg.norm(bm[K*b:(K+1)*b, J*b:(J+1)*b]) for J in range(nb)] for K in range(nb)])
    prods = np.einsum("ik,kj->ijk", na, nbm)
    vals = np.sort(prods.ravel())
    mid = len(vals) // 3
    tau = float(np.sqrt(vals[mid] * vals[mid + 1]))
    assert vals[mid + 1] / vals[mid] > 1 + 1e-9
    want = {(I, J, K) for I, J, K in zip(*np.nonzero(prods >= tau))}
    _, _, keys, _ = oracle.spamm_recursive(a, bm, b, tau, want_keys=True)
    got = set(zip(*oracle.unpack_keys(keys)))
    assert got == want


@pytest.mark.parametrize("n,b,tau", [(1024, 32, 1e-6), (300, 16, 1e-5), (256, 64, 1e-3)])
def test_recursive_equals_flat_bitexact(n, b, tau):
    a = si.exp_decay(n, 0.9, 1)
    bm = si.algebraic_decay(n, 2.0, 3, np.float64)
    c1, t1, keys, kept = oracle.spamm_recursive(a, bm, b, tau, want_keys=True)
    c2, t2 = oracle.spamm_flat(a, bm, b, tau)
    assert t1 == t2 and np.array_equal(c1, c2)
    flat_keys, _ = oracle.tasks_flat(oracle.tile_sqnorms(a, b), oracle.tile_sqnorms(bm, b), tau)
    assert np.array_equal(np.sort(keys), flat_keys)
    t3, kept3 = oracle.count_hierarchical(oracle.tile_sqnorms(a, b), oracle.tile_sqnorms(bm, b), tau)
    assert t3 == t1 and np.array_equal(kept3, kept)


def test_flat_row_ranges_compose():
    a = si.exp_decay(256, 0.85, 7)
    c_all, t_all = oracle.spamm_flat(a, a, 32, 1e-5)
    c1, t1 = oracle.spamm_flat(a, a, 32, 1e-5, rows=(0, 3))
    c2, t2 = oracle.spamm_flat(a, a, 32, 1e-5, rows=(3, 8))
    assert t1 + t2 == t_all and np.array_equal(c1 + c2, c_all)


def test_exp_decay_workload_counts():
    # exponential decay, n = 1024, leaf 32, tau = 1e-6: the cull keeps a small
    # fraction of the 32^3 product space; tau = 0 keeps all of it.
    a = si.exp_decay_workload()
    c, T, _, kept = oracle.spamm_recursive(a, a, 32, 1e-6)
    assert T == 2400 and kept[-1] == 1
    err = oracle.rel_err(c, a @ a)
    assert 1e-9 < err < 1e-7


# ---------------------------------------------------------------- error, nesting, symmetry, scaling

@pytest.mark.parametrize("tau", [1e-2, 1e-4, 1e-6])
def test_error_below_culled_norm_bound(tau):
    # Eq. (3): each omitted product has norm <= ||A_IK|| ||B_KJ||, so the error is
    # at most the sum of the culled norm products (plus rounding).
    n, b = 256, 16
    a = si.algebraic_decay(n, 2.0, 5, np.float64)
    c, _, _, _ = oracle.spamm_recursive(a, a, b, tau)
    _, bound = oracle.tasks_flat(oracle.tile_sqnorms(a, b), oracle.tile_sqnorms(a, b), tau, want_keys=False)
    ref = a @ a
    err = np.linalg.norm(c - ref)
    assert err <= bound + 1e-12 * np.linalg.norm(ref)
    assert err > 0


def _block_constant(alpha, b):
    """Matrix whose b x b tile (I, K) is alpha[I, K] * ones: its squared tile
    norm is alpha^2 b^2, exact for powers of two."""
    return np.kron(alpha, np.ones((b, b)))


def test_flat_culled_bound_exact_on_block_constant_operands():
    # Eq. (3) summed over culled leaf triples: sum |alpha_IK| |beta_KJ| b^2 over
    # the triples with alpha^2 beta^2 b^4 < tau^2.  Powers of two make every norm,
    # square root and sum exact.  Catches: the bound summing S_A S_B (squared)
    # or sqrt(S_A + S_B), an (I,K)/(K,J) index mix-up, kept triples counted in.
    rng = np.random.default_rng(21)
    nb, b = 9, 16
    alpha = 2.0 ** rng.integers(-10, 1, (nb, nb)) * rng.choice([-1.0, 1.0], (nb, nb))
    beta = 2.0 ** rng.integers(-10, 1, (nb, nb)) * rng.choice([-1.0, 1.0], (nb, nb))
    alpha[rng.random((nb, nb)) < 0.2] = 0.0
    a, bm = _block_constant(alpha, b), _block_constant(beta, b)
    for tau in (2.0 ** -3, 2.0 ** -7, 2.0 ** -12):
        prod = (alpha[:, :, None] ** 2) * (beta[None, :, :] ** 2) * b ** 4      # [I, K, J]
        culled = prod < tau * tau
        ref = float(np.sum((np.abs(alpha)[:, :, None] * np.abs(beta)[None, :, :] * b * b)[culled]))
        keys, bound = oracle.tasks_flat(oracle.tile_sqnorms(a, b), oracle.tile_sqnorms(bm, b), tau)
        assert bound == ref
        assert len(keys) == int(np.sum(~culled))


def test_culled_bounds_hand_computed_block_case():
    # nb = 4 tiles of 16: a big 2x2-tile block of ones and a small one of
    # 2^-6 on the diagonal, zeros elsewhere (A = B).  At tau = 1 the recursion
    # culls the tier-1 node of the small block whole (its norm product is
    # 0.25 * 0.25 < 1) while every leaf triple of the big block passes
    # (2^8 * 2^8 >= 1).  Omitted product: (2^-6 J_32)^2 = 2^-7 J_32, Frobenius
    # norm 2^-7 * 32 = 0.25.  Culled-node bound = sqrt(0.25) sqrt(0.25) = 0.25
    # (tight); culled-triple bound = 8 triples * 2^-4 = 0.5.
    b = 16
    alpha = np.zeros((4, 4))
    alpha[:2, :2] = 1.0
    alpha[2:, 2:] = 2.0 ** -6
    a = _block_constant(alpha, b)
    S = oracle.tile_sqnorms(a, b)
    T, kept, hbound = oracle.count_hierarchical(S, S, 1.0, want_bound=True)
    assert hbound == 0.25
    assert T == 8 and kept.tolist() == [8, 1, 1]
    _, fbound = oracle.tasks_flat(S, S, 1.0)
    assert fbound == 0.5
    c, _, _, _ = oracle.spamm_recursive(a, a, b, 1.0)
    assert np.linalg.norm(c - a @ a) == 0.25


def test_culled_node_bound_limits():
    # root culled: the bound is ||A||_F ||B||_F; no node above the leaves
    # culled: the node bound is the triple bound (the same culled triples).
    # Catches: the root test skipped, culled upper nodes not added, a leaf
    # triple under a culled node counted again.
    n, b = 256, 16
    a = si.algebraic_decay(n, 2.0, 5, np.float64)
    bm = si.algebraic_decay(n, 1.5, 6, np.float64)
    SA, SB = oracle.tile_sqnorms(a, b), oracle.tile_sqnorms(bm, b)
    T, kept, hb = oracle.count_hierarchical(SA, SB, 1e6, want_bound=True)
    assert T == 0 and kept.sum() == 0
    ref = np.linalg.norm(a) * np.linalg.norm(bm)
    assert abs(hb - ref) <= 1e-13 * ref
    # the smallest norm product of any node above the leaves (from numpy block sums)
    upper = []
    m = SA
    mb = SB
    while m.shape[0] > 1:
        k = m.shape[0]
        pad = -(-k // 2) * 2
        ma, mbb = np.zeros((pad, pad)), np.zeros((pad, pad))
        ma[:k, :k], mbb[:k, :k] = m, mb
        m = ma.reshape(pad // 2, 2, pad // 2, 2).sum(axis=(1, 3))
        mb = mbb.reshape(pad // 2, 2, pad // 2, 2).sum(axis=(1, 3))
        upper.append(np.min(m[:, :, None] * mb[None, :, :]))
    leaf_min = np.min(SA[:, :, None] * SB[None, :, :])
    tau2 = 0.5 * (min(upper) + leaf_min) if min(upper) > leaf_min else None
    assert tau2 is not None
    tau = float(np.sqrt(tau2))
    T, kept, hb = oracle.count_hierarchical(SA, SB, tau, want_bound=True)
    assert all(kept[l] == (-(-SA.shape[0] // 2 ** l)) ** 3 for l in range(1, len(kept)))
    keys, fb = oracle.tasks_flat(SA, SB, tau)
    assert T == len(keys) < SA.shape[0] ** 3
    assert abs(hb - fb) <= 1e-13 * fb


def test_nested_in_tau_and_monotone_error():
    n, b = 256, 16
    a = si.algebraic_decay(n, 2.0, 6, np.float64)
    ref = a @ a
    prev_keys, prev_err = None, -1.0
    for tau in [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6]:
        c, _, keys, _ = oracle.spamm_recursive(a, a, b, tau, want_keys=True)
        ks = set(keys.tolist())
        if prev_keys is not None:
            assert prev_keys <= ks            # smaller tau keeps a superset
            err = np.linalg.norm(c - ref)
            assert err <= prev_err            # non-negative operands: monotone error
            prev_err = err
        else:
            prev_err = np.linalg.norm(c - ref)
        prev_keys = ks


def test_symmetric_operand_symmetric_result():
    n, b = 320, 32
    a = si.exp_decay(n, 0.9, 8)
    c, _, keys, _ = oracle.spamm_recursive(a, a, b, 1e-4, want_keys=True)
    I, J, K = oracle.unpack_keys(keys)
    s = set(zip(I.tolist(), J.tolist(), K.tolist()))
    # (A A)^T = A A: triple (I,J,K) pairs with (J,I,K); allow rare last-bit ties
    mism = sum((j, i, k) not in s for i, j, k in s)
    assert mism <= 0.001 * len(s)
    assert np.max(np.abs(c - c.T)) < 1e-3 * np.abs(c).max()


def test_power_of_two_scaling_is_exact():
    # A -> 2A, B -> 4B, tau -> 8 tau: every norm product scales by 64 = 8^2 exactly.
    a = si.exp_decay(200, 0.9, 9)
    bm = si.algebraic_decay(200, 2.0, 10, np.float64)
    c1, t1, k1, _ = oracle.spamm_recursive(a, bm, 16, 1e-5, want_keys=True)
    c2, t2, k2, _ = oracle.spamm_recursive(2 * a, 4 * bm, 16, 8e-5, want_keys=True)
    assert t1 == t2 and np.array_equal(k1, k2) and np.array_equal(8 * c1, c2)


def test_huge_tau_gives_zero():
    a = si.exp_decay(128, 0.9, 1)
    c, T, _, kept = oracle.spamm_recursive(a, a, 16, 1e6)
    assert T == 0 and not np.any(c) and kept.sum() == 0


def test_ragged_sizes_flat_equals_recursive():
    for n in (33, 47, 129, 255):
        a = _rand(n, n)
        c1, t1, _, _ = oracle.spamm_recursive(a, a.T.copy(), 16, 0.05)
        c2, t2 = oracle.spamm_flat(a, a.T.copy(), 16, 0.05)
        assert t1 == t2 and np.array_equal(c1, c2)


# ---------------------------------------------------------------- depth-scaled threshold (section 2)
# The paper's rigorous variant lowers tau by a factor 8 per level below the
# root: a node at depth k is tested against tau / 8^k and kept only if every
# ancestor was kept.  These pins do not use the recursion's code.

def _ancestor_chain_keys(a, bm, b, tau):
    """Brute force: a leaf triple is kept iff, at every depth k from the root,
    its ancestor (I >> l, J >> l, K >> l) on tier l = L - k passes against
    tau / 8^k, with tier norms summed directly from the matrix (numpy)."""
    n = a.shape[0]
    nb = -(-n // b)
    L = oracle.num_levels(nb)
    keys = set()
    for I in range(nb):
        for J in range(nb):
            for K in range(nb):
                ok = True
                for l in range(L, -1, -1):
                    s = b << l                     # side of a tier-l block
                    i, j, k = (I >> l) * s, (J >> l) * s, (K >> l) * s
                    na = float(np.sum(a[i:i + s, k:k + s] ** 2))
                    nbm = float(np.sum(bm[k:k + s, j:j + s] ** 2))
                    t = tau / 8.0 ** (L - l)
                    if na * nbm < t * t:
                        ok = False
                        break
                if ok:
                    keys.add((I, J, K))
    return keys


@pytest.mark.parametrize("n,b,tau", [(32, 4, 3e-2), (40, 4, 1e-2), (64, 8, 1e-3)])
def test_depth_scaled_matches_ancestor_brute_force(n, b, tau):
    # catches: the wrong depth for the divisor (tier instead of depth), dividing
    # by 4 or 64 instead of 8 per level, a child tested against its parent's
    # threshold, padding blocks kept or lost
    a = si.exp_decay(n, 0.7, 5)
    bm = si.algebraic_decay(n, 2.0, 6, np.float64)
    want = _ancestor_chain_keys(a, bm, b, tau)
    _, T, keys, _ = oracle.spamm_recursive(a, bm, b, tau, want_keys=True, depth_scaled=True)
    got = set(zip(*oracle.unpack_keys(keys)))
    # the norms of numpy's sums and the canonical ones differ by rounding: only
    # triples whose decisive test is within 1e-12 of its threshold may differ
    assert T == len(got)
    assert len(got ^ want) <= max(1, len(want) // 1000)
    assert len(got) > 0


@pytest.mark.parametrize("tau", [1e-2, 1e-4, 1e-6])
def test_depth_scaled_sandwich(tau):
    # every test is looser than tau (tau / 8^k <= tau) and at least as strict as
    # the leaf's tau / 8^L, and tier norms dominate their leaves', so
    # flat(tau) <= depth(tau) <= flat(tau / 8^L) as sets of leaf triples
    a = si.exp_decay(512, 0.9, 8)
    b = 16
    S = oracle.tile_sqnorms(a, b)
    L = oracle.num_levels(S.shape[0])
    d, _ = oracle.tasks_hierarchical(S, S, tau, depth_scaled=True)
    lo, _ = oracle.tasks_flat(S, S, tau)
    hi, _ = oracle.tasks_flat(S, S, tau / 8.0 ** L)
    ds, los, his = set(d.tolist()), set(lo.tolist()), set(hi.tolist())
    assert los <= ds <= his
    assert len(los) < len(ds) < len(his)       # the schedules really differ here


@pytest.mark.parametrize("tau", [3e-3, 1e-4, 1e-6])
def test_depth_scaled_error_bound(tau):
    # each culled node at depth k omits a product of norm < tau / 8^k, and depth
    # k has at most 8^k nodes, so ||C~ - C||_F < (L + 1) tau (the rigorous bound)
    a = si.exp_decay(384, 0.92, 9)
    bm = si.exp_decay(384, 0.88, 10)
    b = 16
    c, T, _, _ = oracle.spamm_recursive(a, bm, b, tau, depth_scaled=True)
    L = oracle.num_levels(-(-384 // b))
    err = np.linalg.norm(c - a @ bm)
    assert 0 < err < (L + 1) * tau
    assert T < (384 // b) ** 3                  # something was culled


def test_depth_scaled_single_tile_and_zero_tau():
    # one tile (L = 0): the only test is at the root, with tau itself; tau = 0
    # keeps every triple under either schedule
    a = _rand(16, 3)
    for tau in (0.0, 1.0, 1e3):
        _, t1, _, _ = oracle.spamm_recursive(a, a, 16, tau)
        _, t2, _, _ = oracle.spamm_recursive(a, a, 16, tau, depth_scaled=True)
        assert t1 == t2
    a = si.exp_decay(200, 0.8, 11)
    c, T, _, _ = oracle.spamm_recursive(a, a, 8, 0.0, depth_scaled=True)
    assert T == 25 ** 3 and np.allclose(c, a @ a, rtol=0, atol=1e-12)
