"""Pins of the learned-tau oracle pieces: histogram bins, MLP gradient by
finite differences, Adam's first-step property and convergence, bisection."""
import numpy as np
import pytest

import oracle
import spamm_inputs as si
from oracle import tau_model as tm


def test_feature_layout_and_param_count():
    assert tm.NFEAT == 515
    assert tm.n_params() == 515 * 128 + 128 + 2 * (128 * 128 + 128) + 128 + 1


def test_histogram_bins_exact_cases():
    # root S = 1: S in [0.1, 1] -> bin 0, [0.01, 0.1) -> bin 1, tiny and 0 -> bin 31
    tier0 = np.array([[1.0, 0.5], [0.05, 0.0]])
    tier1 = np.array([[1.0]])
    h = tm.tier_histograms([tier0, tier1]).reshape(tm.NTIERS, tm.NBINS)
    assert h[0, 0] == 0.5 and h[0, 1] == 0.25 and h[0, 31] == 0.25
    assert h[1, 0] == 1.0 and np.all(h[2:] == 0)
    # exactly at a threshold: S == root * 1e-3 is not below it -> bin 2
    h = tm.tier_histograms([np.array([[1e-3]]), np.array([[1.0]])]).reshape(tm.NTIERS, tm.NBINS)
    assert h[0, 2] == 1.0


def test_histogram_fractions_on_real_pyramid():
    a = si.algebraic_decay(1000, 2.0, 3, np.float64)
    pyr = oracle.norm_pyramid(a, 64)
    h = tm.tier_histograms(pyr).reshape(tm.NTIERS, tm.NBINS)
    for l in range(len(pyr)):
        assert abs(h[l].sum() - 1.0) < 1e-12
    assert h[len(pyr) - 1, 0] == 1.0          # the root tier holds the root only
    # scale free: 3 * A gives the same features
    pyr3 = oracle.norm_pyramid(3 * a, 64)
    f1 = tm.features(pyr, pyr, 1000, 64, 1e-6)
    f3 = tm.features(pyr3, pyr3, 1000, 64, 1e-6)
    assert np.array_equal(f1, f3)


def test_label_scale_covariance():
    # A -> 2A, B -> 2B multiplies S_root by 4 each and the equivalent tau by 4
    assert abs(tm.label(4e-6, 4.0 * 9.0, 4.0 * 25.0) - tm.label(1e-6, 9.0, 25.0)) < 1e-15


def test_forward_pass_through_network():
    # hand-set weights route feature 0 through the ReLUs: y = 2 relu(x0) + 0.5
    shapes = tm.layer_shapes()
    params = [(np.zeros(s), np.zeros(s[1])) for s in shapes]
    for li in range(3):
        params[li][0][0, 0] = 1.0
    params[3][0][0, 0] = 2.0
    params[3][1][0] = 0.5
    X = np.zeros((3, tm.NFEAT))
    X[:, 0] = [-1.0, 0.0, 3.0]
    yhat, _ = tm.forward(params, X)
    assert np.array_equal(yhat, [0.5, 0.5, 6.5])


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    params = tm.unflatten(si.mlp_init(tm.layer_shapes(), 7))
    X = rng.uniform(0, 0.3, (9, tm.NFEAT))
    y = rng.normal(-8, 1, 9)
    _, grads = tm.loss_and_grad(params, X, y)
    flat = tm.flatten(params)
    g = tm.flatten(grads)
    idx = rng.choice(flat.size, 60, replace=False)
    idx = np.concatenate([idx, [flat.size - 1, flat.size - 2, 515 * 128 + 5]])
    h = 1e-6
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        lp, _ = tm.loss_and_grad(tm.unflatten(fp), X, y)
        lm, _ = tm.loss_and_grad(tm.unflatten(fm), X, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_first_step_and_convergence():
    # first step: bias correction makes |dp| = lr * |g| / (|g| + eps) ~ lr
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.3, -5.0, 1e-3])
    p1, m, v = tm.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(np.abs(p1 - p), 0.01 * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.all(np.sign(p - p1) == np.sign(g))
    # minimises a convex quadratic
    c = np.array([0.5, -1.5, 2.0])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        p, m, v = tm.adam_step(p, 2 * (p - c), m, v, t, 0.01)
    assert np.max(np.abs(p - c)) < 1e-3


def test_bisection_finds_threshold():
    # err(tau) = tau / 7 meets target 1e-6 up to tau* = 7e-6
    tau, err, evals = tm.bisect_tau(lambda t: t / 7.0, 1e-6, 1.0, resolution_decades=0.01)
    assert tau <= 7e-6 and tau >= 7e-6 * 10 ** -0.01 and err <= 1e-6
    # the start, six decade steps (1e-6 meets), seven halvings of [1e-6, 1e-5]
    assert evals == 1 + 6 + 7
    # already met at the start
    assert tm.bisect_tau(lambda t: 0.0, 1e-6, 1e-3)[2] == 1
