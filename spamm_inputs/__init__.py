"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only draws numbers: it holds none of the multiply's arithmetic
(no norms, no culling, no products).  Both sides take their inputs from here,
so the oracle and the HIP library see bit-identical matrices.

Uniform draws come from a counter-based hash, SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):

    mix(z):  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9
             z ^= z >> 27; z *= 0x94D049BB133111EB
             z ^= z >> 31
    sm64(x) = mix(x + 0x9E3779B97F4A7C15)           (mod 2^64)

    h(seed, i, j) = sm64(sm64(seed) ^ (i << 32 | j))
    u(seed, i, j) = (h >> 11) * 2^-53                 in [0, 1)

For a symmetric matrix the counter is (min(i,j), max(i,j)), i.e. one draw for
i <= j copied to the mirror element (not (U + U^T)/2, which would change the
distribution).  The decay factor f(|i-j|) is tabulated on the host in FP64
and each element is round_to_storage(f(|i-j|) * (lo + (hi-lo) * u)).

Decay families follow the paper's definition of decay (introduction,
footnote 1: |a_ij| < c*lambda^|i-j| exponential, c/(|i-j|^lambda+1)
algebraic) and the Figure 1 test matrices of section 2.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_ROW_CHUNK_ELEMS = 1 << 24      # elements generated per chunk (bounds host memory)


def _sm64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser of x + golden, elementwise on uint64 (wrapping)."""
    with np.errstate(over="ignore"):
        z = x + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def seed_key(seed: int) -> np.uint64:
    return _sm64(np.array([seed], dtype=np.uint64))[0]


def uniform01(seed: int, i: np.ndarray, j: np.ndarray) -> np.ndarray:
    """u(seed, i, j) in [0, 1) as FP64 (53 random bits)."""
    i = np.asarray(i, dtype=np.uint64)
    j = np.asarray(j, dtype=np.uint64)
    h = _sm64(seed_key(seed) ^ ((i << np.uint64(32)) | j))
    return (h >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _decay_matrix(n: int, table: np.ndarray, seed: int, lo: float, hi: float,
                  symmetric: bool, dtype, out: np.ndarray | None = None) -> np.ndarray:
    """a_ij = round(table[|i-j|] * (lo + (hi-lo) * u(seed, i, j)))."""
    dtype = np.dtype(dtype)
    if out is None:
        out = np.empty((n, n), dtype=dtype)
    rows = max(1, _ROW_CHUNK_ELEMS // max(n, 1))
    cols = np.arange(n, dtype=np.int64)
    for r0 in range(0, n, rows):
        r1 = min(n, r0 + rows)
        ii = np.arange(r0, r1, dtype=np.int64)[:, None]
        jj = cols[None, :]
        if symmetric:
            ci, cj = np.minimum(ii, jj), np.maximum(ii, jj)
        else:
            ci, cj = np.broadcast_to(ii, (r1 - r0, n)), np.broadcast_to(jj, (r1 - r0, n))
        u = uniform01(seed, ci, cj)
        u = lo + (hi - lo) * u
        f = table[np.abs(ii - jj)]
        out[r0:r1] = (f * u).astype(dtype)
    return out


def exp_table(n: int, lam: float) -> np.ndarray:
    """f(d) = lam^d, d = 0..n-1, FP64."""
    return np.power(float(lam), np.arange(n, dtype=np.float64))


def algebraic_table(n: int, p: float) -> np.ndarray:
    """f(d) = 1 / (d^p + 1), d = 0..n-1, FP64."""
    d = np.arange(n, dtype=np.float64)
    return 1.0 / (np.power(d, float(p)) + 1.0)


def exp_decay(n: int, lam: float, seed: int, dtype=np.float64, lo=-1.0, hi=1.0,
              symmetric=True) -> np.ndarray:
    """Exponential decay a_ij = lam^|i-j| * u_ij, u ~ U(lo, hi)."""
    return _decay_matrix(n, exp_table(n, lam), seed, lo, hi, symmetric, dtype)


def algebraic_decay(n: int, p: float, seed: int, dtype=np.float32, lo=0.5, hi=1.5,
                    symmetric=False) -> np.ndarray:
    """Algebraic decay a_ij = u_ij / (|i-j|^p + 1), u ~ U(lo, hi)."""
    return _decay_matrix(n, algebraic_table(n, p), seed, lo, hi, symmetric, dtype)


def sp2_diagonal(n: int, seed: int = 4, gap: float = 0.0, n_occ: int | None = None) -> np.ndarray:
    """The N(0,1) diagonal of sp2_hamiltonian (PCG64 stream of seed), FP64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    diag = rng.standard_normal(n)
    if gap:
        k = n // 2 if n_occ is None else n_occ
        diag = diag.copy()
        diag[:k] -= gap / 2.0
        diag[k:] += gap / 2.0
    return diag


def sp2_hamiltonian(n: int, lam: float = 0.85, seed: int = 4, dtype=np.float32,
                    gap: float = 0.0, n_occ: int | None = None) -> np.ndarray:
    """Symmetric banded-decay model Hamiltonian.

    h_ii ~ N(0,1) (numpy PCG64 stream of ``seed``, drawn on the host),
    h_ij = -lam^|i-j| for i != j.  With gap > 0 the n_occ lowest-indexed
    diagonal entries are shifted by -gap/2 and the rest by +gap/2, which opens
    a spectral gap at the occupation boundary (used for small exact checks).
    """
    diag = sp2_diagonal(n, seed, gap, n_occ)
    table = -np.power(float(lam), np.arange(n, dtype=np.float64))
    h = np.empty((n, n), dtype=np.float64)
    rows = max(1, _ROW_CHUNK_ELEMS // max(n, 1))
    cols = np.arange(n)
    for r0 in range(0, n, rows):
        r1 = min(n, r0 + rows)
        ii = np.arange(r0, r1)[:, None]
        h[r0:r1] = table[np.abs(ii - cols[None, :])]
    h[np.arange(n), np.arange(n)] = diag
    return h.astype(dtype)


def figure1_pair(n: int = 512, case: str = "A"):
    """The two synthetic pairs of the paper's Figure 1 (section 2).

    Case A: A_ij = exp(-|i-j|), B_ij = exp(-2|i-j|).
    Case B: A_ij = B_ij = 1/|i-j|^3 off the diagonal, 0 on it.
    """
    d = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :]).astype(np.float64)
    if case == "A":
        return np.exp(-d), np.exp(-2.0 * d)
    if case == "B":
        with np.errstate(divide="ignore"):
            a = np.where(d > 0, 1.0 / d ** 3, 0.0)
        return a, a.copy()
    raise ValueError(case)


def tau_training_params(count: int, seed: int = 10000, n_lo: int = 512, n_hi: int = 8192,
                        leaves=(32, 64, 128), taus_per_matrix: int = 20, log_tau_rel=(-13.0, -3.0)):
    """Recipes of the matrices of a tau training set, drawn from PCG64(seed).

    Each entry: family "exp" (lam ~ U(0.8, 0.97), u ~ U(-1, 1), symmetric, as the
    exponential workloads) or "alg" (p ~ U(1.25, 3), u ~ U(0.5, 1.5), as the
    algebraic ones), n ~ U{n_lo..n_hi step 64}, leaf from `leaves`, u-seed
    seed + i, and taus_per_matrix values of log10(tau / ||A||_F^2) ~ U(log_tau_rel)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        fam = "exp" if rng.integers(2) == 0 else "alg"
        n = int(rng.integers(n_lo // 64, n_hi // 64 + 1)) * 64
        leaf = int(leaves[int(rng.integers(len(leaves)))])
        if fam == "exp":
            par, lo, hi, sym = float(rng.uniform(0.8, 0.97)), -1.0, 1.0, True
        else:
            par, lo, hi, sym = float(rng.uniform(1.25, 3.0)), 0.5, 1.5, False
        taus = rng.uniform(log_tau_rel[0], log_tau_rel[1], taus_per_matrix)
        out.append({"family": fam, "n": n, "leaf": leaf, "param": par, "lo": lo, "hi": hi, "symmetric": sym,
                    "seed": seed + i, "log_tau_rel": taus})
    return out


def recipe_table(r) -> np.ndarray:
    return exp_table(r["n"], r["param"]) if r["family"] == "exp" else algebraic_table(r["n"], r["param"])


def mlp_init(shapes, seed: int) -> np.ndarray:
    """Initial weights of a ReLU network: He-normal W (std sqrt(2/in)), zero b.

    shapes: list of (in, out) per layer; returns the flat FP64 vector
    W1 (row-major, in x out), b1, W2, b2, ... drawn from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for i, o in shapes:
        parts.append(rng.standard_normal(i * o) * np.sqrt(2.0 / i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


# --- workload recipes -------------------------------------------------------

def exp_decay_workload(n=1024, lam=0.9, seed=1):
    """Exponential decay, lam = 0.9, u ~ U(-1,1) symmetric, FP64, C = A*A (leaf 32)."""
    return exp_decay(n, lam, seed, np.float64, -1.0, 1.0, True)


def algebraic_workload(n=8192, p=2.0, seed=2, dtype=np.float32):
    """Algebraic decay u/(|i-j|^p + 1), u ~ U(0.5,1.5), FP32 storage, C = A*A (leaf 64)."""
    return algebraic_decay(n, p, seed, dtype, 0.5, 1.5, False)


def batch_params(count=64, seed=3, n_lo=512, n_hi=8192, step=64, lam_lo=0.8, lam_hi=0.97):
    """Sizes n_m ~ U{n_lo..n_hi step} and lam_m ~ U(lam_lo, lam_hi) from PCG64(seed).

    Matrix m uses u-seed 300 + m."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(n_lo // step, n_hi // step + 1, size=count) * step
    lams = rng.uniform(lam_lo, lam_hi, size=count)
    return [(int(s), float(l), 300 + m) for m, (s, l) in enumerate(zip(sizes, lams))]


def batch_matrix(n, lam, useed, dtype=np.float32):
    return exp_decay(n, lam, useed, dtype, -1.0, 1.0, True)
