"""Python binding of libspamm: the MI355X SpAMM (Challacombe & Bock, section 2).

Argument marshalling only: every step of the multiply runs in the HIP
library; PyTorch provides device memory (its caching allocator backs the
library's allocations) and the stream.  The binding refuses to work without
the built library -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspamm.so")

LEAF = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3, "f16": 4, "f16x3": 5}
LEAF_NAMES = {v: k for k, v in LEAF.items()}
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ECAPACITY", 5: "ENONFINITE",
          6: "ENOCONV", 7: "EUNSUPPORTED"}
MAX_LEVELS = 24
SP2_MAX_ITER = 256


class SpammError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("leaf", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("nb", ctypes.c_int64), ("survivors", ctypes.c_int64 * MAX_LEVELS),
                ("tasks", ctypes.c_int64), ("nonempty_tiles", ctypes.c_int64),
                ("flops", ctypes.c_double), ("culled_bound", ctypes.c_double)]

    def to_dict(self):
        return {"n": self.n, "leaf": self.leaf, "levels": self.levels, "nb": self.nb,
                "survivors": [int(self.survivors[i]) for i in range(self.levels + 1)],
                "tasks": int(self.tasks), "nonempty_tiles": int(self.nonempty_tiles),
                "flops": float(self.flops), "culled_bound": float(self.culled_bound)}


SCHEDULE = {"static": 0, "lpt": 1, "list": 2}


class Tune(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int32), ("schedule", ctypes.c_int32), ("split", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 5)]


TUNE_MAX_TRIALS = 18


class TuneReport(ctypes.Structure):
    _fields_ = [("trials", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("leaf", ctypes.c_int32 * TUNE_MAX_TRIALS), ("schedule", ctypes.c_int32 * TUNE_MAX_TRIALS),
                ("split", ctypes.c_int32 * TUNE_MAX_TRIALS), ("qualified", ctypes.c_int32 * TUNE_MAX_TRIALS),
                ("ms", ctypes.c_double * TUNE_MAX_TRIALS), ("max_rel_err", ctypes.c_double * TUNE_MAX_TRIALS),
                ("best_ms", ctypes.c_double)]

    def to_dict(self):
        sched = {v: k for k, v in SCHEDULE.items()}
        return {"from_cache": bool(self.from_cache), "best_ms": self.best_ms,
                "trials": [{"leaf": self.leaf[i], "schedule": sched[self.schedule[i]], "split": bool(self.split[i]),
                            "ms": self.ms[i], "max_rel_err": self.max_rel_err[i],
                            "qualified": bool(self.qualified[i])}
                           for i in range(self.trials)]}


TAU_NFEAT = 515
TAU_NPARAM = 515 * 128 + 128 + 2 * (128 * 128 + 128) + 128 + 1


class TauInfo(ctypes.Structure):
    _fields_ = [("tau_pred", ctypes.c_double), ("err_pred", ctypes.c_double), ("tau", ctypes.c_double),
                ("rel_err", ctypes.c_double), ("tasks", ctypes.c_int64), ("evaluations", ctypes.c_int32),
                ("fallback", ctypes.c_int32)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Timing(ctypes.Structure):
    _fields_ = [("ms_cull", ctypes.c_double), ("ms_leaf", ctypes.c_double), ("ms_norms", ctypes.c_double),
                ("ms_total", ctypes.c_double)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Sp2Log(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("stagnated", ctypes.c_int32), ("result_step", ctypes.c_int32),
                ("trace", ctypes.c_double * SP2_MAX_ITER), ("idem", ctypes.c_double * SP2_MAX_ITER),
                ("branch", ctypes.c_int32 * SP2_MAX_ITER), ("tasks", ctypes.c_int64 * SP2_MAX_ITER),
                ("final_trace", ctypes.c_double), ("energy", ctypes.c_double),
                ("eps_min", ctypes.c_double), ("eps_max", ctypes.c_double)]

    def to_dict(self):
        k = self.iterations
        return {"iterations": k, "converged": bool(self.converged), "stagnated": bool(self.stagnated),
                "result_step": int(self.result_step),
                "trace": [self.trace[i] for i in range(k)], "idem": [self.idem[i] for i in range(k)],
                "branch": [int(self.branch[i]) for i in range(k)],
                "tasks": [int(self.tasks[i]) for i in range(k)],
                "final_trace": self.final_trace, "energy": self.energy,
                "eps_min": self.eps_min, "eps_max": self.eps_max}


_lib = None
_alloc_cb = None
_dealloc_cb = None
_VP = ctypes.c_void_p
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_DEALLOC_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def lib():
    """Load libspamm.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1011_3534_amd.hipbuild`")
    L = ctypes.CDLL(LIB_PATH)
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    PP = ctypes.POINTER(_VP)
    sig = {
        "spamm_build": ([_VP, i64, i64, i32, i32, _VP, PP], i32),
        "spamm_build_ex": ([_VP, i64, i64, i32, i32, i32, _VP, PP], i32),
        "spamm_build_batched": ([i32, _VP, _VP, _VP, i32, i32, _VP, _VP], i32),
        "spamm_build_view": ([_VP, i64, i64, i32, i32, _VP, PP], i32),
        "spamm_build_view_ex": ([_VP, i64, i64, i32, i32, i32, _VP, PP], i32),
        "spamm_build_view_batched": ([i32, _VP, _VP, _VP, i32, i32, _VP, _VP], i32),
        "spamm_multiply": ([_VP, _VP, dbl, i32, _VP, PP, ctypes.POINTER(Stats)], i32),
        "spamm_multiply_ex": ([_VP, _VP, dbl, i32, i32, _VP, PP, ctypes.POINTER(Stats)], i32),
        "spamm_multiply_timed": ([_VP, _VP, dbl, i32, _VP, PP, ctypes.POINTER(Timing)], i32),
        "spamm_multiply_timed_ex": ([_VP, _VP, dbl, i32, i32, _VP, PP, ctypes.POINTER(Timing)], i32),
        "spamm_multiply_batched": ([i32, PP, PP, ctypes.POINTER(dbl), i32, ctypes.POINTER(Tune), _VP, PP,
                                    ctypes.POINTER(Stats)], i32),
        "spamm_multiply_batched_noalloc": ([i32, PP, PP, ctypes.POINTER(dbl), i32, ctypes.POINTER(Tune), _VP,
                                            PP], i32),
        "spamm_sp2_ex": ([_VP, i64, dbl, i32, dbl, i32, i32, _VP, PP, ctypes.POINTER(Sp2Log)], i32),
        "spamm_sp2": ([_VP, i64, dbl, i32, dbl, i32, _VP, PP, ctypes.POINTER(Sp2Log)], i32),
        "spamm_autotune_batched": ([i32, PP, ctypes.POINTER(i64), i32, ctypes.POINTER(dbl), i32,
                                    ctypes.POINTER(i32), i32, dbl, i32, ctypes.c_char_p, _VP,
                                    ctypes.POINTER(Tune), ctypes.POINTER(TuneReport)], i32),
        "spamm_to_dense": ([_VP, _VP, i64, _VP], i32),
        "spamm_info": ([_VP, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32),
                        ctypes.POINTER(i32)], i32),
        "spamm_norms": ([_VP, i32, ctypes.POINTER(dbl), i64, _VP], i32),
        "spamm_task_list": ([_VP, ctypes.POINTER(ctypes.c_uint64), i64, ctypes.POINTER(i64), _VP], i32),
        "spamm_diff_norms": ([_VP, _VP, ctypes.POINTER(dbl), ctypes.POINTER(dbl), _VP], i32),
        "spamm_set_allocator": ([_ALLOC_FN, _DEALLOC_FN, _VP], i32),
        "spamm_tau_model_create": ([ctypes.POINTER(ctypes.c_float), PP], i32),
        "spamm_tau_model_params": ([_VP, ctypes.POINTER(ctypes.c_float)], i32),
        "spamm_tau_model_free": ([_VP], None),
        "spamm_tau_features": ([_VP, _VP, dbl, _VP, _VP], i32),
        "spamm_tau_forward": ([_VP, _VP, i64, _VP, _VP], i32),
        "spamm_tau_grad": ([_VP, _VP, _VP, i64, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                            _VP], i32),
        "spamm_tau_train": ([_VP, _VP, _VP, i64, i32, i32, ctypes.c_float, _VP, ctypes.POINTER(ctypes.c_float)],
                            i32),
        "spamm_tau_predict": ([_VP, _VP, dbl, _VP, _VP, ctypes.POINTER(dbl)], i32),
        "spamm_tau_select": ([_VP, _VP, dbl, _VP, i32, dbl, _VP, PP, ctypes.POINTER(TauInfo)], i32),
        "spamm_generate_decay": ([i64, i64, i32, ctypes.POINTER(dbl), ctypes.c_uint64, dbl, dbl, i32,
                                  ctypes.POINTER(dbl), _VP, _VP], i32),
        "spamm_free": ([_VP], None),
        "spamm_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def declared_symbols() -> list[str]:
    """Function names declared in include/*.h (the ABI this binding wraps)."""
    import glob
    import re
    inc = os.path.join(os.path.dirname(_HERE), "include")
    names = []
    for h in sorted(glob.glob(os.path.join(inc, "*.h"))):
        text = open(h).read()
        names += re.findall(r"^\s*(?:spamm_status|void|const char\*)\s+(spamm_\w+)\s*\(", text, re.M)
    return names


def _check(code):
    if code != 0:
        msg = lib().spamm_last_error()
        raise SpammError(code, msg.decode() if msg else "")


def _check_result(code, h, out):
    """_check for calls that hand back a result handle: a syncing check that
    fails after the product was written (ECAPACITY, ENONFINITE) still returns
    a fresh handle, which is freed before raising."""
    if code != 0 and out is None and h.value:
        lib().spamm_free(h)
        h.value = None
    _check(code)


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def use_torch_allocator(enable: bool = True):
    """Back the library's device allocations with torch's caching allocator.

    The library passes the stream each block is used on: the block is taken
    from (and returned to) that stream's pool, so a block released right
    after the kernels that read it is reused only by later work on the same
    stream.  Every handle keeps the allocator it was created with (its
    storage is returned to it when the handle is freed), so the callbacks are
    made once and live as long as the process: a handle made while they were
    installed may be freed after the library's allocator was switched back or
    set again."""
    global _alloc_cb, _dealloc_cb
    import torch

    if not enable:
        _check(lib().spamm_set_allocator(_ALLOC_FN(), _DEALLOC_FN(), None))
        return
    if _alloc_cb is None:
        def _alloc(nbytes, stream, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
            except Exception:          # OOM: the library reports SPAMM_ENOMEM
                return None

        def _dealloc(ptr, stream, ctx):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:
                pass

        _alloc_cb = _ALLOC_FN(_alloc)
        _dealloc_cb = _DEALLOC_FN(_dealloc)
    _check(lib().spamm_set_allocator(_alloc_cb, _dealloc_cb, None))


class Matrix:
    """Owning wrapper of a spamm_matrix handle."""

    def __init__(self, handle: ctypes.c_void_p, source=None):
        self._h = handle
        self.source = source  # the tensor a view reads its tiles from (kept alive)
        n, b, dt, lv = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().spamm_info(handle, ctypes.byref(n), ctypes.byref(b), ctypes.byref(dt), ctypes.byref(lv)))
        self.n, self.leaf, self.levels = n.value, b.value, lv.value
        self.dtype = "f64" if dt.value == 0 else "f32"
        self.nb = -(-self.n // self.leaf)

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h:
            lib().spamm_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def to_dense(self, stream=None):
        import torch
        dt = torch.float64 if self.dtype == "f64" else torch.float32
        out = torch.empty((self.n, self.n), dtype=dt, device="cuda")
        _check(lib().spamm_to_dense(self._h, ctypes.c_void_p(out.data_ptr()), self.n, _stream(stream)))
        return out

    def norms(self, level: int = 0, stream=None) -> np.ndarray:
        m = self.nb
        for _ in range(level):
            m = -(-m // 2)
        out = np.empty((m, m), dtype=np.float64)
        _check(lib().spamm_norms(self._h, level, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 out.size, _stream(stream)))
        return out

    def task_list(self, stream=None) -> np.ndarray:
        cnt = ctypes.c_int64()
        _check(lib().spamm_task_list(self._h, None, 0, ctypes.byref(cnt), _stream(stream)))
        keys = np.empty(max(cnt.value, 1), dtype=np.uint64)
        _check(lib().spamm_task_list(self._h, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                     keys.size, ctypes.byref(cnt), _stream(stream)))
        return np.sort(keys[:cnt.value])


def build(a, leaf: int, out: Matrix | None = None, stream=None, prec: str | None = None,
          view: bool = False) -> Matrix:
    """Quadtree of a dense CUDA tensor (float32 or float64, row-major).

    With out given (same n, leaf, dtype) the handle is rebuilt in place.  With
    prec naming a 16-bit leaf precision the same pass also writes the split
    hi/lo tiles those products read (spamm_build_ex).  With view=True the
    handle reads its tiles from `a` itself (spamm_build_view: norms only, no
    copy; with prec, spamm_build_view_ex also writes the split tiles); it
    keeps a reference to `a`, which must not change while in use."""
    import torch
    if not (a.is_cuda and a.dim() == 2 and a.shape[0] == a.shape[1]):
        raise ValueError("build expects a square CUDA tensor")
    if a.dtype not in (torch.float32, torch.float64):
        raise ValueError("build expects float32 or float64")
    if a.stride(1) != 1:
        raise ValueError("build expects unit column stride")
    h = ctypes.c_void_p(out.handle.value if out is not None else None)
    dt = 0 if a.dtype == torch.float64 else 1
    if view:
        if prec is None:
            _check(lib().spamm_build_view(ctypes.c_void_p(a.data_ptr()), a.shape[0], a.stride(0), dt, leaf,
                                          _stream(stream), ctypes.byref(h)))
        else:
            _check(lib().spamm_build_view_ex(ctypes.c_void_p(a.data_ptr()), a.shape[0], a.stride(0), dt, leaf,
                                             LEAF[prec], _stream(stream), ctypes.byref(h)))
        if out is not None:
            out.source = a
            return out
        return Matrix(h, source=a)
    if prec is None:
        _check(lib().spamm_build(ctypes.c_void_p(a.data_ptr()), a.shape[0], a.stride(0), dt, leaf,
                                 _stream(stream), ctypes.byref(h)))
    else:
        _check(lib().spamm_build_ex(ctypes.c_void_p(a.data_ptr()), a.shape[0], a.stride(0), dt, leaf, LEAF[prec],
                                    _stream(stream), ctypes.byref(h)))
    return out if out is not None else Matrix(h)


def build_batched(tensors, leaf: int, outs=None, stream=None, view: bool = False) -> list:
    """Quadtrees of several dense CUDA tensors of one dtype in one pass
    (spamm_build_batched; view=True: spamm_build_view_batched, see build).
    outs: None or a list of handles/None to rebuild."""
    import torch
    count = len(tensors)
    dts = {a.dtype for a in tensors}
    if len(dts) > 1 or (dts and dts.pop() not in (torch.float32, torch.float64)):
        raise ValueError("build_batched expects float32 or float64 tensors of one dtype")
    for a in tensors:
        if not (a.is_cuda and a.dim() == 2 and a.shape[0] == a.shape[1] and a.stride(1) == 1):
            raise ValueError("build_batched expects square CUDA tensors with unit column stride")
    dt = 0 if count and tensors[0].dtype == torch.float64 else 1
    PA = (ctypes.c_void_p * count)(*[a.data_ptr() for a in tensors])
    N = (ctypes.c_int64 * count)(*[a.shape[0] for a in tensors])
    LD = (ctypes.c_int64 * count)(*[a.stride(0) for a in tensors])
    outs = outs or [None] * count
    PO = (ctypes.c_void_p * count)(*[(o.handle.value if o is not None else None) for o in outs])
    fn = lib().spamm_build_view_batched if view else lib().spamm_build_batched
    _check(fn(count, PA, N, LD, dt, leaf, _stream(stream), PO))
    res = [o if o is not None else Matrix(ctypes.c_void_p(PO[m])) for m, o in enumerate(outs)]
    if view:
        for m, o in enumerate(res):
            o.source = tensors[m]
    return res


TAU_FLAT, TAU_DEPTH_SCALED = 0, 1


def multiply(A: Matrix, B: Matrix, tau: float, prec: str = "f32", out: Matrix | None = None,
             stats: bool = False, stream=None, depth_scaled: bool = False):
    """C ~= A B by the SpAMM recursion (Eq. 4).  Returns C, or (C, stats dict).

    depth_scaled: tau / 8^k at depth k below the root (spamm_multiply_ex)."""
    h = ctypes.c_void_p(out.handle.value if out is not None else None)
    st = Stats() if stats else None
    if depth_scaled:
        code = lib().spamm_multiply_ex(A.handle, B.handle, float(tau), LEAF[prec], TAU_DEPTH_SCALED,
                                       _stream(stream), ctypes.byref(h), ctypes.byref(st) if st is not None else None)
    else:
        code = lib().spamm_multiply(A.handle, B.handle, float(tau), LEAF[prec], _stream(stream), ctypes.byref(h),
                                    ctypes.byref(st) if st is not None else None)
    _check_result(code, h, out)
    C = out if out is not None else Matrix(h)
    return (C, st.to_dict()) if stats else C


def multiply_timed(A: Matrix, B: Matrix, tau: float, prec: str = "f32", out: Matrix | None = None,
                   stream=None, descent: bool = False):
    """multiply with HIP-event phase timing; returns (C, timing dict in ms).

    descent: the cull descends tier by tier from the root (same result)."""
    h = ctypes.c_void_p(out.handle.value if out is not None else None)
    t = Timing()
    _check(lib().spamm_multiply_timed_ex(A.handle, B.handle, float(tau), LEAF[prec], 1 if descent else 0,
                                         _stream(stream), ctypes.byref(h), ctypes.byref(t)))
    C = out if out is not None else Matrix(h)
    return C, t.to_dict()


def multiply_batched(As, Bs, taus, prec: str = "f32", outs=None, stats: bool = False,
                     schedule: str | None = None, stream=None):
    """Independent products C_m ~= A_m B_m in one cull pass and one leaf launch.

    schedule: None/"lpt" (persistent, largest first), "static" or "list" (persistent over the
    tiles that need a write)."""
    count = len(As)
    PA = (ctypes.c_void_p * count)(*[a.handle.value for a in As])
    PB = (ctypes.c_void_p * count)(*[b.handle.value for b in Bs])
    PC = (ctypes.c_void_p * count)(*[(o.handle.value if o is not None else None) for o in (outs or [None] * count)])
    T = (ctypes.c_double * count)(*[float(t) for t in taus])
    st = (Stats * count)() if stats else None
    tune = None
    if schedule is not None:
        tune = Tune()
        tune.schedule = SCHEDULE[schedule]
    code = lib().spamm_multiply_batched(count, PA, PB, T, LEAF[prec], ctypes.byref(tune) if tune else None,
                                        _stream(stream), PC, st if st is not None else None)
    if code != 0:
        for m in range(count):
            if (outs is None or outs[m] is None) and PC[m]:
                lib().spamm_free(ctypes.c_void_p(PC[m]))
    _check(code)
    Cs = []
    for m in range(count):
        if outs is not None and outs[m] is not None:
            Cs.append(outs[m])
        else:
            Cs.append(Matrix(ctypes.c_void_p(PC[m])))
    return (Cs, [s.to_dict() for s in st]) if stats else Cs


def multiply_batched_noalloc(As, Bs, taus, outs, prec: str = "f32", schedule: str | None = None, stream=None):
    """multiply_batched into existing results, with no device allocation: the
    batch scratch is the library's static per-device array, so calls that
    overlap on one device race.  Every outs[m] must be a result handle that
    has already received a product; returns outs."""
    count = len(As)
    PA = (ctypes.c_void_p * count)(*[a.handle.value for a in As])
    PB = (ctypes.c_void_p * count)(*[b.handle.value for b in Bs])
    PC = (ctypes.c_void_p * count)(*[o.handle.value for o in outs])
    T = (ctypes.c_double * count)(*[float(t) for t in taus])
    tune = None
    if schedule is not None:
        tune = Tune()
        tune.schedule = SCHEDULE[schedule]
    _check(lib().spamm_multiply_batched_noalloc(count, PA, PB, T, LEAF[prec], ctypes.byref(tune) if tune else None,
                                                _stream(stream), PC))
    return list(outs)


def autotune_batched(dense, taus, prec: str = "f32", leaves=(32, 64, 128), max_rel_err: float = 1e-5,
                     reps: int = 3, cache_path: str | None = None, stream=None):
    """Pick leaf size, operand staging and schedule for the products A_m A_m of dense CUDA tensors.

    Returns (tune dict {"leaf", "schedule", "split"}, report dict); split: build the
    operands with split tiles (build(..., prec=prec))."""
    import torch
    count = len(dense)
    for a in dense:
        if not (a.is_cuda and a.is_contiguous() and a.dim() == 2 and a.shape[0] == a.shape[1]):
            raise ValueError("autotune_batched expects square contiguous CUDA tensors")
    dt = 0 if dense[0].dtype == torch.float64 else 1
    PA = (ctypes.c_void_p * count)(*[a.data_ptr() for a in dense])
    N = (ctypes.c_int64 * count)(*[a.shape[0] for a in dense])
    T = (ctypes.c_double * count)(*[float(t) for t in taus])
    Lv = (ctypes.c_int32 * len(leaves))(*leaves)
    best, rep = Tune(), TuneReport()
    _check(lib().spamm_autotune_batched(count, PA, N, dt, T, LEAF[prec], Lv, len(leaves), float(max_rel_err),
                                        int(reps), cache_path.encode() if cache_path else None, _stream(stream),
                                        ctypes.byref(best), ctypes.byref(rep)))
    sched = {v: k for k, v in SCHEDULE.items()}
    return {"leaf": best.leaf, "schedule": sched[best.schedule], "split": bool(best.split)}, rep.to_dict()


def sp2(H: Matrix, n_occ: int, tau: float, max_iter: int = 60, idem_tol: float = 1e-6,
        prec: str = "f32", stream=None, symmetric: bool = False, dropping: bool = False):
    """TC2 purification (section 3) with SpAMM squarings; returns (P, log dict).

    symmetric: symmetric squarings (tiles I <= J formed, the others mirrored).
    dropping: the block-dropping scheme instead (tau is the drop threshold;
    exact squarings over the tiles present, small tiles of each iterate dropped)."""
    h = ctypes.c_void_p()
    log = Sp2Log()
    flags = (1 if symmetric else 0) | (2 if dropping else 0)
    code = lib().spamm_sp2_ex(H.handle, int(n_occ), float(tau), int(max_iter), float(idem_tol), LEAF[prec],
                              flags, _stream(stream), ctypes.byref(h), ctypes.byref(log))
    if code not in (0, 6):
        _check(code)
    d = log.to_dict()
    d["status"] = STATUS[code]
    return Matrix(h), d


class TauModel:
    """Device-resident tau network (weights + Adam moments)."""

    def __init__(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != TAU_NPARAM:
            raise ValueError(f"expected {TAU_NPARAM} parameters, got {p.size}")
        h = ctypes.c_void_p()
        _check(lib().spamm_tau_model_create(p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def params(self) -> np.ndarray:
        out = np.empty(TAU_NPARAM, dtype=np.float32)
        _check(lib().spamm_tau_model_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def free(self):
        if self._h:
            lib().spamm_tau_model_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def forward(self, X, stream=None):
        import torch
        X = X.contiguous()
        y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        _check(lib().spamm_tau_forward(self._h, ctypes.c_void_p(X.data_ptr()), X.shape[0],
                                       ctypes.c_void_p(y.data_ptr()), _stream(stream)))
        return y

    def grad(self, X, y, stream=None):
        g = np.empty(TAU_NPARAM, dtype=np.float32)
        loss = ctypes.c_float()
        X, y = X.contiguous(), y.contiguous()
        _check(lib().spamm_tau_grad(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                    X.shape[0], g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                    ctypes.byref(loss), _stream(stream)))
        return g, loss.value

    def train(self, X, y, epochs: int, batch: int, lr: float, stream=None):
        X, y = X.contiguous(), y.contiguous()
        losses = np.zeros(epochs, dtype=np.float32)
        _check(lib().spamm_tau_train(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                     X.shape[0], int(epochs), int(batch), float(lr), _stream(stream),
                                     losses.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return losses


def tau_features(A: Matrix, B: Matrix, target: float, stream=None):
    import torch
    out = torch.empty(TAU_NFEAT, dtype=torch.float32, device="cuda")
    _check(lib().spamm_tau_features(A.handle, B.handle, float(target), ctypes.c_void_p(out.data_ptr()),
                                    _stream(stream)))
    return out


def tau_predict(A: Matrix, B: Matrix, target: float, model: TauModel, stream=None) -> float:
    t = ctypes.c_double()
    _check(lib().spamm_tau_predict(A.handle, B.handle, float(target), model.handle, _stream(stream),
                                   ctypes.byref(t)))
    return t.value


def tau_select(A: Matrix, B: Matrix, target: float, model: TauModel | None = None, prec: str = "f32",
               resolution_decades: float = 0.05, out: Matrix | None = None, stream=None):
    """(C at the selected tau, info dict); checked against the exact product."""
    h = ctypes.c_void_p(out.handle.value if out is not None else None)
    info = TauInfo()
    code = lib().spamm_tau_select(A.handle, B.handle, float(target), model.handle if model else None, LEAF[prec],
                                  float(resolution_decades), _stream(stream), ctypes.byref(h), ctypes.byref(info))
    _check_result(code, h, out)
    C = out if out is not None else Matrix(h)
    return C, info.to_dict()


def generate_decay(table, seed: int, lo: float, hi: float, symmetric: bool, dtype="f32", diag=None,
                   stream=None):
    """Seeded decay matrix drawn on the device: a_ij = f(|i-j|) (lo + (hi-lo) u_ij).

    table: FP64 numpy array f(0..n-1) (e.g. spamm_inputs.exp_table); diag:
    optional FP64 diagonal.  Returns an n x n CUDA tensor."""
    import torch
    table = np.ascontiguousarray(table, dtype=np.float64)
    n = table.shape[0]
    out = torch.empty((n, n), dtype=torch.float64 if dtype == "f64" else torch.float32, device="cuda")
    dg = None
    if diag is not None:
        diag = np.ascontiguousarray(diag, dtype=np.float64)
        dg = diag.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib().spamm_generate_decay(n, n, 0 if dtype == "f64" else 1,
                                      table.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(seed), float(lo),
                                      float(hi), int(bool(symmetric)), dg, ctypes.c_void_p(out.data_ptr()),
                                      _stream(stream)))
    return out


def diff_norms(X: Matrix, Y: Matrix, stream=None):
    """(||X - Y||_F^2, ||Y||_F^2) in FP64."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(lib().spamm_diff_norms(X.handle, Y.handle, ctypes.byref(a), ctypes.byref(b), _stream(stream)))
    return a.value, b.value


def rel_err(X: Matrix, Y: Matrix, stream=None) -> float:
    d2, r2 = diff_norms(X, Y, stream)
    return float(np.sqrt(d2 / r2)) if r2 > 0 else float(np.sqrt(d2))
