"""FP64 CPU oracle for SpAMM (Challacombe & Bock, section 2, Eqs. 1 and 4).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline of the benchmark may import this package; the product path (the HIP
library and its Python binding) never does and shares no code with it.

The heavy loops live in ``spamm_oracle.c`` (plain C, FP64, built with gcc and
-ffp-contract=off); this module marshals numpy arrays to it.  The TC2
purification driver and the tau-model pieces are in ``sp2.py`` and
``tau_model.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spamm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-O3", "-mavx2", "-mfma", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-Wall"]

_lib = None
_DP = ctypes.POINTER(ctypes.c_double)
_U64P = ctypes.POINTER(ctypes.c_uint64)
_I64P = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (always when force, else only if missing)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.orc_tile_sqnorms.argtypes = [_DP, i64, i64, i32, _DP]
    lib.orc_tile_sqnorms.restype = ctypes.c_int
    lib.orc_norm_parent.argtypes = [_DP, i64, _DP]
    lib.orc_norm_parent.restype = None
    lib.orc_num_levels.argtypes = [i64]
    lib.orc_num_levels.restype = i32
    lib.orc_spamm_recursive.argtypes = [_DP, _DP, i64, i32, dbl, i32, _DP, _U64P, i64, _I64P]
    lib.orc_spamm_recursive.restype = i64
    lib.orc_spamm_flat.argtypes = [_DP, _DP, i64, i32, dbl, i64, i64, i32, _DP]
    lib.orc_spamm_flat.restype = i64
    lib.orc_tasks_flat.argtypes = [_DP, _DP, i64, dbl, _U64P, i64, _DP]
    lib.orc_tasks_flat.restype = i64
    lib.orc_tasks_hierarchical.argtypes = [_DP, _DP, i64, dbl, i32, _U64P, i64, _I64P, _DP]
    lib.orc_tasks_hierarchical.restype = i64
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = i32
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=_DP):
    return a.ctypes.data_as(t)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def num_levels(nb: int) -> int:
    """Tiers above the leaves: m_0 = nb, m_{l+1} = ceil(m_l / 2), m_L = 1."""
    return int(_load().orc_num_levels(nb))


def tile_sqnorms(a, b: int) -> np.ndarray:
    """Canonical FP64 squared Frobenius norms of the b x b leaves, shape (nb, nb)."""
    a = _f64(a)
    n = a.shape[0]
    nb = -(-n // b)
    out = np.empty((nb, nb), dtype=np.float64)
    rc = _load().orc_tile_sqnorms(_p(a), n, a.shape[1], b, _p(out))
    if rc:
        raise ValueError(f"orc_tile_sqnorms failed ({rc})")
    return out


def norm_parent(S) -> np.ndarray:
    S = _f64(S)
    m = S.shape[0]
    mp = -(-m // 2)
    out = np.empty((mp, mp), dtype=np.float64)
    _load().orc_norm_parent(_p(S), m, _p(out))
    return out


def norm_pyramid(a, b: int) -> list[np.ndarray]:
    """[S_0 (leaves), S_1, ..., S_L (root, 1x1)] of the quadtree (Eq. 1)."""
    levels = [tile_sqnorms(a, b)]
    while levels[-1].shape[0] > 1:
        levels.append(norm_parent(levels[-1]))
    return levels


def spamm_recursive(a, bm, b: int, tau: float, want_keys: bool = False, depth_scaled: bool = False):
    """Eq. (4) literally.  Returns (C, T, keys-or-None, kept-per-tier).

    depth_scaled: the threshold of a sub-product is its parent's divided by 8
    (tau at the root), the rigorous variant discussed in section 2."""
    a, bm = _f64(a), _f64(bm)
    n = a.shape[0]
    nb = -(-n // b)
    L = num_levels(nb)
    c = np.empty((n, n), dtype=np.float64)
    kept = np.zeros(L + 1, dtype=np.int64)
    cap = nb ** 3 if want_keys else 0
    keys = np.empty(max(cap, 1), dtype=np.uint64)
    t = _load().orc_spamm_recursive(_p(a), _p(bm), n, b, float(tau), int(bool(depth_scaled)), _p(c),
                                    _p(keys, _U64P) if want_keys else None, cap, _p(kept, _I64P))
    if t < 0:
        raise ValueError(f"orc_spamm_recursive failed ({t})")
    return c, int(t), (keys[:t].copy() if want_keys else None), kept


def spamm_flat(a, bm, b: int, tau: float, rows: tuple[int, int] | None = None, sym_upper: bool = False):
    """Flat enumeration of kept leaf triples; returns (C, T).

    rows = (I0, I1) restricts the work to C tile rows [I0, I1); the other rows
    of the returned C are zero.  sym_upper: symmetric squaring (A = B
    symmetric): tiles I <= J by the rule, C_JI = C_IJ^T; T counts those."""
    a, bm = _f64(a), _f64(bm)
    n = a.shape[0]
    nb = -(-n // b)
    I0, I1 = rows if rows is not None else (0, nb)
    c = np.zeros((n, n), dtype=np.float64)
    t = _load().orc_spamm_flat(_p(a), _p(bm), n, b, float(tau), I0, I1, int(bool(sym_upper)), _p(c))
    if t < 0:
        raise ValueError(f"orc_spamm_flat failed ({t})")
    return c, int(t)


def tasks_flat(SA, SB, tau: float, want_keys: bool = True):
    """Brute-force kept triples from leaf norms.  Returns (keys sorted, bound)."""
    SA, SB = _f64(SA), _f64(SB)
    nb = SA.shape[0]
    cap = nb ** 3 if want_keys else 0
    keys = np.empty(max(cap, 1), dtype=np.uint64)
    bound = ctypes.c_double(0.0)
    t = _load().orc_tasks_flat(_p(SA), _p(SB), nb, float(tau),
                               _p(keys, _U64P) if want_keys else None, cap, ctypes.byref(bound))
    return (keys[:t].copy() if want_keys else int(t)), float(bound.value)


def count_hierarchical(SA, SB, tau: float, depth_scaled: bool = False, want_bound: bool = False):
    """Kept octree nodes per tier (tier 0 = leaf triples) from leaf norms.

    want_bound: also return the culled-node bound (sum over the octree nodes
    the recursion culls, at any tier, of ||A^k||_F ||B^k||_F; Eq. 3)."""
    SA, SB = _f64(SA), _f64(SB)
    nb = SA.shape[0]
    kept = np.zeros(num_levels(nb) + 1, dtype=np.int64)
    bound = ctypes.c_double(0.0)
    t = _load().orc_tasks_hierarchical(_p(SA), _p(SB), nb, float(tau), int(bool(depth_scaled)), None, 0,
                                       _p(kept, _I64P), ctypes.byref(bound))
    return (int(t), kept, float(bound.value)) if want_bound else (int(t), kept)


def tasks_hierarchical(SA, SB, tau: float, depth_scaled: bool = False):
    """Kept leaf triples of the recursion (Eq. 4, products left out) from leaf
    norms, as sorted keys, with the kept nodes per tier."""
    SA, SB = _f64(SA), _f64(SB)
    nb = SA.shape[0]
    kept = np.zeros(num_levels(nb) + 1, dtype=np.int64)
    lib = _load()
    t = lib.orc_tasks_hierarchical(_p(SA), _p(SB), nb, float(tau), int(bool(depth_scaled)), None, 0,
                                   _p(kept, _I64P), None)
    keys = np.empty(max(t, 1), dtype=np.uint64)
    t2 = lib.orc_tasks_hierarchical(_p(SA), _p(SB), nb, float(tau), int(bool(depth_scaled)), _p(keys, _U64P), t,
                                    _p(kept, _I64P), None)
    assert t2 == t
    return np.sort(keys[:t]), kept


def unpack_keys(keys):
    keys = np.asarray(keys, dtype=np.uint64)
    m21 = np.uint64((1 << 21) - 1)
    return ((keys >> np.uint64(42)) & m21).astype(np.int64), \
        ((keys >> np.uint64(21)) & m21).astype(np.int64), (keys & m21).astype(np.int64)


def pack_keys(I, J, K):
    I, J, K = (np.asarray(x, dtype=np.uint64) for x in (I, J, K))
    return (I << np.uint64(42)) | (J << np.uint64(21)) | K


def rel_err(c_approx, c_exact) -> float:
    """||C~ - C||_F / ||C||_F in FP64."""
    d = np.asarray(c_approx, dtype=np.float64) - np.asarray(c_exact, dtype=np.float64)
    den = np.linalg.norm(np.asarray(c_exact, dtype=np.float64))
    return float(np.linalg.norm(d) / den) if den > 0 else float(np.linalg.norm(d))
