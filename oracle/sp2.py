"""TC2 / SP2 density-matrix purification on the FP64 oracle SpAMM.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3 of the paper builds the Heaviside function P = theta[F - mu I] by
the TC2 trace-correcting purification (Niklasson, Phys. Rev. B 66, 155115,
2002), 40-60 multiplies per solve, and measures the accumulated error by the
electronic energy E = Tr(P F).  The iteration itself is only cited; the
reading used here:

  1. Gershgorin bounds eps_min, eps_max of H (FP64);
  2. X_0 = (eps_max I - H) / (eps_max - eps_min), eigenvalues in [0, 1],
     the lowest eigenvalues of H mapped nearest 1;
  3. at step m: Y = SpAMM(X_m, X_m, tau); t_m = tr(X_m);
     X_{m+1} = Y if t_m > n_occ else 2 X_m - Y  (the branch is decided from the
     trace before the product; a tie takes 2X - Y);
     e_m = ||Y - X_m||_F (idempotency of X_m);
  4. stop after the step whose e_m <= tol (P = X_{m+1}); or stop when the
     iteration stagnates, e_m >= e_{m-2} while e_{m-2} < STAG_BELOW
     (P = X_m: under truncation the idempotency error stops falling and the
     trace rule would then amplify the truncation error every step); or after
     max_iter steps (P = X_max_iter);
  5. E = tr(P H) in FP64.
"""
from __future__ import annotations

import numpy as np

from . import spamm_flat

STAG_BELOW = 0.1


def gershgorin(h) -> tuple[float, float]:
    h = np.asarray(h, dtype=np.float64)
    d = np.diag(h)
    r = np.abs(h).sum(axis=1) - np.abs(d)
    return float(np.min(d - r)), float(np.max(d + r))


def initial_x(h) -> np.ndarray:
    h = np.asarray(h, dtype=np.float64)
    lo, hi = gershgorin(h)
    x = -h.copy()
    x[np.diag_indices_from(x)] += hi
    return x / (hi - lo)


def step(x, n_occ: int, b: int, tau: float, symmetric: bool = False):
    """One TC2 step from X (FP64).  Returns (X_next, trace, idem, branch, T).

    symmetric: the squaring forms the tiles I <= J and mirrors the others."""
    x = np.asarray(x, dtype=np.float64)
    y, t_count = spamm_flat(x, x, b, tau, sym_upper=symmetric)
    tr = float(np.trace(x))
    idem = float(np.linalg.norm(y - x))
    branch = 0 if tr > n_occ else 1          # 0: X <- X^2 ; 1: X <- 2X - X^2
    x_next = y if branch == 0 else 2.0 * x - y
    return x_next, tr, idem, branch, t_count


def sp2(h, n_occ: int, b: int, tau: float, max_iter: int = 60, tol: float = 1e-8, symmetric: bool = False):
    """TC2 purification; returns (P, log dict).  symmetric: symmetric squarings."""
    x = initial_x(h)
    log = {"trace": [], "idem": [], "branch": [], "tasks": [], "converged": False,
           "stagnated": False}
    for m in range(max_iter):
        x_next, tr, idem, br, t = step(x, n_occ, b, tau, symmetric)
        log["trace"].append(tr)
        log["idem"].append(idem)
        log["branch"].append(br)
        log["tasks"].append(t)
        e = log["idem"]
        if idem <= tol:
            log["converged"] = True
            x = x_next
            break
        if m >= 2 and e[m - 2] < STAG_BELOW and idem >= e[m - 2]:
            log["stagnated"] = True
            break
        x = x_next
    log["iterations"] = len(log["trace"])
    log["final_trace"] = float(np.trace(x))
    log["energy"] = energy(x, h)
    return x, log


def energy(p, h) -> float:
    """E = tr(P H) = sum_ij P_ij H_ji in FP64."""
    p = np.asarray(p, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    return float(np.sum(p * h.T))


# --------------------------------------------------------------------------
# The block-dropping comparison of section 3 (scheme I): every multiply is
# exact over the blocks present, and after each purification step the
# iterate is filtered, its leaf blocks with Frobenius norm below tau dropped.
# Readings: a dropped block is absent from the matrix, so no product reads
# it (the multiply counts only pairs of present blocks); the filter acts on
# the new iterate X_{m+1} (after the TC2 update), so the trace that decides
# the next branch is that of the filtered iterate.  X_0 is not filtered.

def present_count(S) -> int:
    """Leaf products of a multiply X X over present blocks (S > 0): the pairs
    (I,K), (K,J) with both blocks present, sum over K of (present blocks in
    block column K) x (present blocks in block row K)."""
    p = np.asarray(S) > 0.0
    return int(np.sum(p.sum(axis=0).astype(np.int64) * p.sum(axis=1).astype(np.int64)))


def drop_filter(x, b: int, tau: float):
    """Zero the b x b blocks of x whose squared Frobenius norm S (the fixed
    summation order) is below tau^2.  Returns (filtered copy, dropped mask)."""
    from . import tile_sqnorms
    x = np.array(x, dtype=np.float64, copy=True)
    S = tile_sqnorms(x, b)
    drop = S < tau * tau
    n = x.shape[0]
    for I, J in zip(*np.nonzero(drop)):
        x[I * b:min((I + 1) * b, n), J * b:min((J + 1) * b, n)] = 0.0
    return x, drop


def step_dropping(x, n_occ: int, b: int, tau_drop: float):
    """One TC2 step of the dropping scheme from X (FP64).  Returns
    (X_next, trace, idem, branch, T): the product is exact (absent blocks are
    zero and add exact zeros), T counts the pairs of present blocks, X_next is
    the filtered iterate."""
    from . import tile_sqnorms
    x = np.asarray(x, dtype=np.float64)
    y, _ = spamm_flat(x, x, b, 0.0)
    t_count = present_count(tile_sqnorms(x, b))
    tr = float(np.trace(x))
    idem = float(np.linalg.norm(y - x))
    branch = 0 if tr > n_occ else 1
    x_next = y if branch == 0 else 2.0 * x - y
    x_next, _ = drop_filter(x_next, b, tau_drop)
    return x_next, tr, idem, branch, t_count


def sp2_dropping(h, n_occ: int, b: int, tau_drop: float, max_iter: int = 60, tol: float = 1e-8):
    """TC2 purification with the dropping scheme; stop rules and log as sp2."""
    x = initial_x(h)
    log = {"trace": [], "idem": [], "branch": [], "tasks": [], "converged": False,
           "stagnated": False}
    for m in range(max_iter):
        x_next, tr, idem, br, t = step_dropping(x, n_occ, b, tau_drop)
        log["trace"].append(tr)
        log["idem"].append(idem)
        log["branch"].append(br)
        log["tasks"].append(t)
        e = log["idem"]
        if idem <= tol:
            log["converged"] = True
            x = x_next
            break
        if m >= 2 and e[m - 2] < STAG_BELOW and idem >= e[m - 2]:
            log["stagnated"] = True
            break
        x = x_next
    log["iterations"] = len(log["trace"])
    log["final_trace"] = float(np.trace(x))
    log["energy"] = energy(x, h)
    return x, log
