"""Helpers of the GPU parity tests: upload, oracle comparisons, tolerances."""
import numpy as np

import oracle

U32 = 2.0 ** -24

# Per-term relative error of one leaf product term a*b, beyond FP32 accumulation
# (operands are the stored FP32 values; see the leaf-precision definitions):
#   f32    : exact operands
#   bf16   : a, b rounded to 8 significant bits (unit roundoff 2^-8) each
#   bf16x3 : hi/lo split leaves |a - hi - lo| <= 2^-16|a|; lo*lo dropped -> 3 * 2^-16
#   f16    : 11 significant bits -> 2 * 2^-11 (+ square)
#   f16x3  : 3 * 2^-22 (power-of-two tile scaling keeps both halves normal
#            except for entries 2^-17 below their tile maximum, covered by
#            the absolute slack)
INPUT_REL = {"f64": 0.0, "f32": 0.0, "bf16": 2 * 2 ** -8 + 2 ** -16, "bf16x3": 3 * 2 ** -16 + 2 ** -24,
             "f16": 2 * 2 ** -11 + 2 ** -22, "f16x3": 3 * 2 ** -22 + 2 ** -33}
ACC_U = {"f64": 2.0 ** -53}


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gamma(k, u):
    return k * u / (1 - k * u)


def elementwise_bound(a64, b64, leaf, tau, prec, depth_scaled=False, rows=None):
    """Bound on |C_gpu - C_oracle| for the same kept triples.

    (|A||B|)_kept is the oracle SpAMM of |A|, |B| (same squares -> same norms
    -> same kept set).  Terms: operand representation error, accumulation in
    the leaf's accumulator over at most n terms, rounding of the stored result.
    rows = (I0, I1): only C tile rows [I0, I1) are formed (the others are 0)."""
    n = a64.shape[0]
    if depth_scaled:
        absprod, _, _, _ = oracle.spamm_recursive(np.abs(a64), np.abs(b64), leaf, tau, depth_scaled=True)
    else:
        absprod, _ = oracle.spamm_flat(np.abs(a64), np.abs(b64), leaf, tau, rows=rows)
    return bound_from_abs(absprod, n, prec, np.max(np.abs(a64)), np.max(np.abs(b64)))


def bound_from_abs(absprod, n, prec, amax, bmax):
    """elementwise_bound from (|A||B|)_kept and the operands' largest |entries|."""
    u = ACC_U.get(prec, U32)
    rel = INPUT_REL[prec] * (1 + gamma(n, u)) + gamma(n + 2, u) + (U32 if prec != "f64" else 2 ** -53)
    slack = 2.0 ** -36 * amax * bmax * n if prec.startswith("f16") else 0.0
    return rel * absprod + slack


def check_rows(out, a64, b64, leaf, tau, prec, rows):
    """Tile rows `rows` of the GPU result `out` (dense, n x n) against the
    oracle's flat SpAMM of the same rows, within elementwise_bound.  Returns
    the largest |difference| / bound."""
    worst = 0.0
    for I in rows:
        ref, _ = oracle.spamm_flat(a64, b64, leaf, tau, rows=(I, I + 1))
        bound = elementwise_bound(a64, b64, leaf, tau, prec, rows=(I, I + 1))
        sl = slice(I * leaf, min((I + 1) * leaf, a64.shape[0]))
        diff = np.abs(np.asarray(out[sl], dtype=np.float64) - ref[sl])
        excess = diff - bound[sl]
        assert np.all(excess <= 0), f"tile row {I}: max excess {excess.max():.3e}"
        nz = bound[sl] > 0
        if np.any(nz):
            worst = max(worst, float(np.max(diff[nz] / bound[sl][nz])))
    return worst


def check_row_many(outs, a64, leaf, tau, I):
    """Tile row I of several GPU results of A A (outs: {prec: dense n x n
    result}) against one oracle evaluation of that row.  Returns
    {prec: largest |difference| / bound}."""
    n = a64.shape[0]
    ref, _ = oracle.spamm_flat(a64, a64, leaf, tau, rows=(I, I + 1))
    aa = np.abs(a64)
    absprod, _ = oracle.spamm_flat(aa, aa, leaf, tau, rows=(I, I + 1))
    amax = float(np.max(aa))
    del aa
    sl = slice(I * leaf, min((I + 1) * leaf, n))
    worst = {}
    for prec, out in outs.items():
        bound = bound_from_abs(absprod[sl], n, prec, amax, amax)
        diff = np.abs(np.asarray(out[sl], dtype=np.float64) - ref[sl])
        excess = diff - bound
        assert np.all(excess <= 0), f"{prec} tile row {I}: max excess {excess.max():.3e}"
        nz = bound > 0
        worst[prec] = float(np.max(diff[nz] / bound[nz])) if np.any(nz) else 0.0
    return worst
