"""Learned tau selector: features, MLP, Adam and the bisection check in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper tunes tau by hand to match energy errors (section 3); the selector
learns the map from the norm structure of A and B and a target relative
error to a threshold.  Definitions used on both sides:

features(A, B, target) -- 2 * 8 * 32 histogram fractions + 3 scalars:
  for operand X in (A, B) and tier l = 0..7 counted from the leaves (tiers
  above the root are empty), the fraction of tier-l nodes falling in bin
  k = #{j in 1..31 : S < S_root * 1e-j}, i.e. bin k holds squared norms
  between 10^-(k+1) and 10^-k of the whole matrix's (bin 31 also takes
  zeros); 1e-j are the correctly rounded decimal constants.  Scalars:
  log10(target), log2(nb) / 10, log2(b) / 7.
label -- y = log10(tau / (||A||_F ||B||_F)), scale free (A -> aA, tau -> a^2
  tau keeps the kept set; see the scaling test of the oracle).
MLP -- 515 -> 128 -> 128 -> 128 -> 1, ReLU on the hidden layers, weights as
  W (in x out) row-major followed by b, layer after layer; loss = mean
  squared error of y.
Adam -- Kingma & Ba (2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
  p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

NBINS = 32
NTIERS = 8
NSCALAR = 3
NFEAT = 2 * NTIERS * NBINS + NSCALAR
HIDDEN = 128
NLAYERS = 3
THRESH = np.array([float(f"1e-{j}") for j in range(1, NBINS)], dtype=np.float64)


def layer_shapes(nin: int = NFEAT, hidden: int = HIDDEN, layers: int = NLAYERS):
    dims = [nin] + [hidden] * layers + [1]
    return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]


def n_params(nin: int = NFEAT) -> int:
    return sum(i * o + o for i, o in layer_shapes(nin))


def unflatten(flat, nin: int = NFEAT):
    flat = np.asarray(flat, dtype=np.float64)
    out, k = [], 0
    for i, o in layer_shapes(nin):
        W = flat[k:k + i * o].reshape(i, o)
        k += i * o
        b = flat[k:k + o]
        k += o
        out.append((W, b))
    assert k == flat.size
    return out


def flatten(params) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def tier_histograms(pyramid) -> np.ndarray:
    """8 x 32 bin fractions of the squared norms of tiers 0..7 (0 = leaves)."""
    root = float(pyramid[-1].ravel()[0])
    out = np.zeros((NTIERS, NBINS))
    for l in range(min(NTIERS, len(pyramid))):
        S = np.asarray(pyramid[l], dtype=np.float64).ravel()
        k = (S[:, None] < root * THRESH[None, :]).sum(axis=1)
        out[l] = np.bincount(k, minlength=NBINS)[:NBINS] / S.size
    return out.ravel()


def features(pyr_a, pyr_b, n: int, b: int, target: float) -> np.ndarray:
    nb = -(-n // b)
    scal = [np.log10(target), np.log2(nb) / 10.0, np.log2(b) / 7.0]
    return np.concatenate([tier_histograms(pyr_a), tier_histograms(pyr_b), scal])


def label(tau: float, sa_root: float, sb_root: float) -> float:
    return float(np.log10(tau) - 0.5 * np.log10(sa_root) - 0.5 * np.log10(sb_root))


def forward(params, X):
    """Returns (yhat (N,), activations list) in FP64."""
    h = np.asarray(X, dtype=np.float64)
    acts = [h]
    for li, (W, b) in enumerate(params):
        z = h @ W + b
        h = np.maximum(z, 0.0) if li < len(params) - 1 else z
        acts.append(h)
    return h[:, 0], acts


def loss_and_grad(params, X, y):
    """MSE loss and its gradient (list of (dW, db)) by the chain rule."""
    yhat, acts = forward(params, X)
    y = np.asarray(y, dtype=np.float64)
    N = y.size
    r = yhat - y
    loss = float(np.mean(r * r))
    g = (2.0 / N) * r[:, None]
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        a_in = acts[li]
        grads[li] = (a_in.T @ g, g.sum(axis=0))
        if li > 0:
            g = (g @ W.T) * (acts[li] > 0.0)
    return loss, grads


def adam_step(flat_p, flat_g, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * flat_g
    v = b2 * v + (1 - b2) * flat_g * flat_g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return flat_p - lr * mh / (np.sqrt(vh) + eps), m, v


def bisect_tau(err_of_tau, target: float, tau_hi: float, resolution_decades: float = 0.05,
               max_down: int = 12):
    """Largest tau (within the resolution) with err_of_tau(tau) <= target.

    Starts from tau_hi; steps down a decade at a time to a tau that meets the
    target, then bisects in log10(tau) between it and the last tau that missed.
    Returns (tau, err, evaluations)."""
    evals = 0
    e = err_of_tau(tau_hi)
    evals += 1
    if e <= target:
        return tau_hi, e, evals
    hi = np.log10(tau_hi)
    lo = hi
    e_lo = e
    for _ in range(max_down):
        hi = lo
        lo -= 1.0
        e_lo = err_of_tau(10 ** lo)
        evals += 1
        if e_lo <= target:
            break
    else:
        return 10 ** lo, e_lo, evals
    while hi - lo > resolution_decades:
        mid = 0.5 * (lo + hi)
        e_mid = err_of_tau(10 ** mid)
        evals += 1
        if e_mid <= target:
            lo, e_lo = mid, e_mid
        else:
            hi = mid
    return 10 ** lo, e_lo, evals
