"""Python binding of libbf (MI355X randomized butterfly factorization).

Argument marshalling only: every step of the factorization runs in the HIP
kernels of ``libbf.so`` through its C ABI (``include/bf.h``).  PyTorch provides
device memory and the current HIP stream.  There is no CPU fallback: if the
library is not built, or no gfx950 device is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbf.so")

__all__ = ["BFError", "lib", "Operator", "Factors", "construct", "segkernel", "helmholtz3d", "fio",
           "dense",
           "from_factors", "compose", "import_factors", "gauss", "cpqr_batched", "lsq_batched",
           "num_levels", "LIB_PATH", "profile_start", "profile_stop", "Server", "TorchAllocator",
           "torch_allocator"]


class BFError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = f"{where}: {lib().bf_strerror(code).decode()} ({code})"
        detail = lib().bf_last_error()
        if detail:
            msg += f": {detail.decode()}"
        super().__init__(msg)


class bf_c64(C.Structure):
    _fields_ = [("re", C.c_float), ("im", C.c_float)]


OPFN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int64,
                   C.POINTER(C.c_int64), C.c_int32, C.c_void_p)


class bf_operator(C.Structure):
    _fields_ = [("matvec", C.c_void_p), ("rmatvec", C.c_void_p), ("user", C.c_void_p),
                ("m", C.c_int64), ("n", C.c_int64)]


PROGRESSFN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int32)
PHASES = ("leaf V", "leaf U", "W", "R")


class bf_opts(C.Structure):
    _fields_ = [("p", C.c_int32), ("r0", C.c_int32), ("max_rank", C.c_int32),
                ("flags", C.c_int32), ("seed", C.c_uint64), ("work_bytes", C.c_int64),
                ("progress", PROGRESSFN), ("progress_user", C.c_void_p),
                ("center_level", C.c_int32), ("reserved", C.c_int32)]


BF_OPT_CENTER_LEVEL = 1
BF_OPT_SEQUENTIAL_LEAF = 2
BF_OPT_SEQUENTIAL_SWEEP = 4
BF_OPT_ONE_STREAM = 8
CENTERS = {"hybrid": None, "column": 0, "row": -1}


class bf_kernel_stats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("flops", C.c_double),
                ("bytes", C.c_double)]


KERNEL_CLASSES = ("matfree", "apply", "cpqr", "chain", "lsq", "other")


ALLOCFN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREEFN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class bf_alloc(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("alloc", ALLOCFN), ("free", FREEFN)]


class bf_server_opts(C.Structure):
    _fields_ = [("slots", C.c_int32), ("batch_cols", C.c_int32), ("hbm_budget", C.c_int64),
                ("alloc", C.POINTER(bf_alloc)), ("solve_rounds", C.c_int32),
                ("max_constructs", C.c_int32)]


class bf_request_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("batch", C.c_int32), ("arrival_ns", C.c_int64),
                ("start_ns", C.c_int64), ("finish_ns", C.c_int64), ("footprint", C.c_int64)]


class bf_info(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("L", C.c_int32), ("lm", C.c_int32),
                ("max_rank", C.c_int32), ("v_iters", C.c_int32), ("u_iters", C.c_int32),
                ("apply_graphs", C.c_int32),
                ("matvec_cols", C.c_int64), ("rmatvec_cols", C.c_int64),
                ("factor_entries", C.c_int64), ("device_bytes", C.c_int64),
                ("fused_launches", C.c_int32), ("merged_levels", C.c_int32),
                ("merge_misses", C.c_int32), ("reserved", C.c_int32)]


_LIB = None
_P = C.c_void_p
_I64P = C.POINTER(C.c_int64)
_I32P = C.POINTER(C.c_int32)

# name -> (restype, argtypes); every symbol of include/bf.h
SIGNATURES = {
    "bf_construct": (C.c_int, [_P, _P, _P, C.c_int64, C.c_int64, C.c_double, C.c_int64,
                               C.POINTER(bf_opts), C.POINTER(bf_alloc), _P, C.POINTER(_P)]),
    "bf_apply": (C.c_int, [_P, C.c_int, _P, C.c_int64, C.c_int64, _P, C.c_int64,
                           C.POINTER(bf_alloc), _P]),
    "bf_apply_noalloc": (C.c_int, [_P, C.c_int, _P, C.c_int64, C.c_int64, _P, C.c_int64, _P]),
    "bf_apply_noalloc_scratch_bytes": (C.c_int64, []),
    "bf_stats": (C.c_int, [_P, C.POINTER(bf_info)]),
    "bf_ranks": (C.c_int, [_P, _I32P, _I32P]),
    "bf_export": (C.c_int, [_P, _P, _I64P]),
    "bf_import": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, _I32P, _I32P, _P, C.c_int64,
                            C.POINTER(bf_alloc), _P, C.POINTER(_P)]),
    "bf_free": (C.c_int, [_P, _P]),
    "bf_release_cached_memory": (C.c_int, []),
    "bf_set_autotune": (C.c_int, [C.c_int]),
    "bf_autotune_entries": (C.c_int, [C.POINTER(C.c_int64)]),
    "bf_autotune_save": (C.c_int, [C.c_char_p]),
    "bf_autotune_load": (C.c_int, [C.c_char_p]),
    "bf_autotune_clear": (C.c_int, []),
    "bf_strerror": (C.c_char_p, [C.c_int]),
    "bf_last_error": (C.c_char_p, []),
    "bf_server_create": (C.c_int, [C.POINTER(bf_server_opts), C.POINTER(_P)]),
    "bf_server_destroy": (C.c_int, [_P]),
    "bf_server_submit_construct": (C.c_int, [_P, C.POINTER(bf_operator), C.c_double, C.c_int64,
                                             C.POINTER(bf_opts), C.POINTER(C.c_int64)]),
    "bf_server_submit_apply": (C.c_int, [_P, C.c_int64, C.c_int, _P, C.c_int64, C.c_int64, _P,
                                         C.c_int64, C.POINTER(C.c_int64)]),
    "bf_server_wait": (C.c_int, [_P, C.c_int64, C.POINTER(bf_request_info)]),
    "bf_server_factors": (C.c_int, [_P, C.c_int64, C.POINTER(_P)]),
    "bf_server_release": (C.c_int, [_P, C.c_int64]),
    "bf_server_rounds": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "bf_profile_start": (C.c_int, []),
    "bf_profile_stop": (C.c_int, [C.POINTER(bf_kernel_stats)]),
    "bf_gauss": (C.c_int, [C.c_uint64, C.c_uint64, C.c_int64, C.c_int64, C.c_int64, _P, _P]),
    "bf_cpqr_batched": (C.c_int, [C.c_int32, _I32P, _I32P, _P, _I64P, C.c_double, _P, _I64P,
                                  _I32P, _P]),
    "bf_lsq_batched": (C.c_int, [C.c_int32, _I32P, _I32P, _I32P, _P, _I64P, _P, _I64P, _P,
                                 _I64P, _P]),
    "bf_op_segkernel": (C.c_int, [_P, C.c_int64, _P, C.c_int64, C.c_double,
                                  C.POINTER(bf_operator)]),
    "bf_op_helmholtz3d": (C.c_int, [_P, C.c_int64, _P, C.c_int64, C.c_double,
                                    C.POINTER(bf_operator)]),
    "bf_op_fio": (C.c_int, [C.c_int64, C.POINTER(bf_operator)]),
    "bf_op_dense": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int64, C.POINTER(bf_operator)]),
    "bf_op_factors": (C.c_int, [_P, C.POINTER(bf_operator)]),
    "bf_op_compose": (C.c_int, [C.POINTER(bf_operator), C.POINTER(bf_operator),
                                C.POINTER(bf_operator)]),
    "bf_operator_destroy": (C.c_int, [C.POINTER(bf_operator)]),
    "bf_op_set_precision": (C.c_int, [C.POINTER(bf_operator), C.c_int]),
    "bf_set_apply_precision": (C.c_int, [_P, C.c_int]),
    "bf_set_apply_graph_cols": (C.c_int, [_P, C.c_int64]),
    "bf_set_apply_fusion": (C.c_int, [_P, C.c_int]),
}


def lib():
    """Load libbf.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2002_03400_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _check(rc, where):
    if rc != 0:
        raise BFError(rc, where)


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev_c64(x):
    torch = _torch()
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex64):
        raise TypeError("expected a complex64 CUDA tensor")
    return x


def _colmajor(x):
    """(rows, cols) tensor -> column-major storage (returns tensor, ld)."""
    if x.dim() == 1:
        x = x[:, None]
    if x.stride(0) == 1 and x.stride(1) >= max(1, x.shape[0]):
        return x, x.stride(1)
    y = x.t().contiguous().t()
    return y, max(1, y.shape[0])


def _empty_colmajor(rows, cols, dtype, device):
    torch = _torch()
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


class TorchAllocator:
    """A bf_alloc backed by torch's CUDA caching allocator, so the library's
    device memory (workspace and factor storage) is torch's: it shows in
    torch.cuda.memory_allocated and is reused by torch afterwards.  A block is
    given back on the stream it was allocated on; when the library frees it on
    another stream, the allocating stream first waits for that stream's work."""

    def __init__(self):
        import threading
        self._live = {}
        self._lock = threading.Lock()
        self._alloc_cb = ALLOCFN(self._alloc)
        self._free_cb = FREEFN(self._free)
        self.struct = bf_alloc(None, self._alloc_cb, self._free_cb)

    @staticmethod
    def _stream_obj(ptr, dev):
        torch = _torch()
        return torch.cuda.default_stream(dev) if not ptr else torch.cuda.ExternalStream(ptr, device=dev)

    def _alloc(self, _ctx, size, stream):
        torch = _torch()
        try:
            dev = torch.cuda.current_device()
            p = torch.cuda.caching_allocator_alloc(int(size), dev, int(stream or 0))
        except Exception:
            return None
        with self._lock:
            self._live[p] = (int(stream or 0), dev)
        return p

    def _free(self, _ctx, ptr, stream):
        torch = _torch()
        with self._lock:
            s_alloc, dev = self._live.pop(ptr)
        s_free = int(stream or 0)
        if s_free != s_alloc:
            ev = torch.cuda.Event()
            ev.record(self._stream_obj(s_free, dev))
            self._stream_obj(s_alloc, dev).wait_event(ev)
        torch.cuda.caching_allocator_delete(ptr)

    def live_blocks(self):
        with self._lock:
            return len(self._live)


_TORCH_ALLOC = None


def torch_allocator() -> TorchAllocator:
    """The process-wide TorchAllocator (created on first use)."""
    global _TORCH_ALLOC
    if _TORCH_ALLOC is None:
        _TORCH_ALLOC = TorchAllocator()
    return _TORCH_ALLOC


def _allocator(which):
    """None (the library's own pool), "torch" or a TorchAllocator."""
    if which is None:
        return None
    if which == "torch":
        return torch_allocator()
    if isinstance(which, TorchAllocator):
        return which
    raise ValueError(f"unknown allocator {which!r}")


def _alloc_ptr(a):
    return C.byref(a.struct) if a is not None else None


def num_levels(m, n, leaf):
    L = 0
    while -(-max(m, n) // (1 << L)) > leaf:
        L += 1
    return L


class Operator:
    """A black box with products by A and A^H (a bf_operator)."""

    def __init__(self, op: bf_operator, keep=()):
        self._op = op
        self._keep = keep
        self.m, self.n = op.m, op.n

    def _call(self, fnptr, X, seg, stream):
        X = _dev_c64(X)
        X, ldx = _colmajor(X)
        rows_out = self.n if fnptr == self._op.rmatvec else self.m
        ncols = X.shape[1]
        if seg is None:
            ycols, segp, nseg = ncols, None, 0
        else:
            seg = np.ascontiguousarray(seg, dtype=np.int64)
            nseg = len(seg) - 1
            ycols = nseg * ncols
            segp = seg.ctypes.data_as(_I64P)
        Y = _empty_colmajor(rows_out, ycols, X.dtype, X.device)
        fn = OPFN(fnptr)
        rc = fn(self._op.user, X.data_ptr(), ldx, ncols, Y.data_ptr(), max(1, rows_out), segp,
                nseg, _stream(stream))
        _check(rc, "operator callback")
        return Y

    def matvec(self, X, seg=None, stream=None):
        return self._call(self._op.matvec, X, seg, stream)

    def rmatvec(self, X, seg=None, stream=None):
        return self._call(self._op.rmatvec, X, seg, stream)

    def set_precision(self, precision):
        """'bf16x3' (split-BF16 matrix cores, default) or 'fp64' (FP64 matrix cores)."""
        code = {"fp64": 0, "bf16x3": 1}[precision]
        _check(lib().bf_op_set_precision(C.byref(self._op), code), "bf_op_set_precision")
        return self

    def close(self):
        if self._op.user:
            lib().bf_operator_destroy(C.byref(self._op))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def segkernel(targets, sources, k) -> Operator:
    """exp(i k r)/r between 2D target and source points ((m, 2), (n, 2))."""
    t = np.ascontiguousarray(targets, dtype=np.float64)
    s = np.ascontiguousarray(sources, dtype=np.float64)
    if t.ndim != 2 or t.shape[1] != 2 or s.ndim != 2 or s.shape[1] != 2:
        raise ValueError("segkernel needs (m, 2) targets and (n, 2) sources")
    op = bf_operator()
    _check(lib().bf_op_segkernel(t.ctypes.data, len(t), s.ctypes.data, len(s), float(k),
                                 C.byref(op)), "bf_op_segkernel")
    return Operator(op)


def helmholtz3d(targets, sources, k) -> Operator:
    """exp(i k r)/r between 3D target and source points ((m, 3), (n, 3))."""
    t = np.ascontiguousarray(targets, dtype=np.float64)
    s = np.ascontiguousarray(sources, dtype=np.float64)
    if t.ndim != 2 or t.shape[1] != 3 or s.ndim != 2 or s.shape[1] != 3:
        raise ValueError("helmholtz3d needs (m, 3) targets and (n, 3) sources")
    op = bf_operator()
    _check(lib().bf_op_helmholtz3d(t.ctypes.data, len(t), s.ctypes.data, len(s), float(k),
                                   C.byref(op)), "bf_op_helmholtz3d")
    return Operator(op)


def fio(n) -> Operator:
    op = bf_operator()
    _check(lib().bf_op_fio(int(n), C.byref(op)), "bf_op_fio")
    return Operator(op)


def dense(A) -> Operator:
    A = _dev_c64(A)
    A, lda = _colmajor(A)
    op = bf_operator()
    _check(lib().bf_op_dense(A.data_ptr(), A.shape[0], A.shape[1], lda, C.byref(op)), "bf_op_dense")
    return Operator(op, keep=(A,))


def from_factors(F: "Factors") -> Operator:
    op = bf_operator()
    _check(lib().bf_op_factors(F._h, C.byref(op)), "bf_op_factors")
    return Operator(op, keep=(F,))


def compose(a1: Operator, a2: Operator) -> Operator:
    op = bf_operator()
    _check(lib().bf_op_compose(C.byref(a1._op), C.byref(a2._op), C.byref(op)), "bf_op_compose")
    return Operator(op, keep=(a1, a2))


@dataclass
class Info:
    m: int
    n: int
    L: int
    lm: int
    max_rank: int
    v_iters: int
    u_iters: int
    apply_graphs: int
    matvec_cols: int
    rmatvec_cols: int
    factor_entries: int
    device_bytes: int
    fused_launches: int
    merged_levels: int
    merge_misses: int
    reserved: int


class Factors:
    """Handle of a hybrid butterfly factorization (owned; freed on close)."""

    def __init__(self, handle, leaf, allocator=None):
        self._h = handle
        self.leaf = leaf
        self._alloc = allocator   # kept alive until the factors are freed
        inf = self.stats()
        self.m, self.n, self.L, self.lm = inf.m, inf.n, inf.L, inf.lm

    def stats(self) -> Info:
        i = bf_info()
        _check(lib().bf_stats(self._h, C.byref(i)), "bf_stats")
        return Info(*[getattr(i, f) for f, _ in bf_info._fields_])

    def ranks(self):
        nb = 1 << self.L
        kU = np.zeros((self.L - self.lm + 1) * nb, np.int32)
        kV = np.zeros((self.lm + 1) * nb, np.int32)
        _check(lib().bf_ranks(self._h, kU.ctypes.data_as(_I32P), kV.ctypes.data_as(_I32P)),
               "bf_ranks")
        return kU.reshape(self.L - self.lm + 1, nb), kV.reshape(self.lm + 1, nb)

    def export(self) -> np.ndarray:
        cnt = C.c_int64(0)
        _check(lib().bf_export(self._h, None, C.byref(cnt)), "bf_export")
        data = np.zeros(cnt.value, np.complex128)
        _check(lib().bf_export(self._h, data.ctypes.data, C.byref(cnt)), "bf_export")
        return data

    def set_precision(self, precision):
        """Arithmetic of apply and of the factors as a black box: 'bf16x3' (BF16
        matrix cores for >= 5 right-hand sides, operands split into three BF16
        terms; vector ALUs with FP32 sums below; default) or 'fp32' (vector
        ALUs, FP32)."""
        code = {"fp32": 2, "bf16x3": 1}[precision]
        _check(lib().bf_set_apply_precision(self._h, code), "bf_set_apply_precision")
        return self

    def set_fusion(self, enable):
        """Fused stages for applies of 1 to 4 columns (default True)."""
        _check(lib().bf_set_apply_fusion(self._h, int(bool(enable))), "bf_set_apply_fusion")
        return self

    def set_graph_cols(self, max_cols):
        """Run applies of at most max_cols columns as cached HIP graphs (0: off)."""
        _check(lib().bf_set_apply_graph_cols(self._h, int(max_cols)), "bf_set_apply_graph_cols")
        return self

    def apply(self, X, trans=False, out=None, stream=None, allocator="torch"):
        """Y = F X (or F^H X); the intermediates come from `allocator` ("torch":
        torch's caching allocator; None: the library's pool)."""
        X = _dev_c64(X)
        X, ldx = _colmajor(X)
        rows_out = self.n if trans else self.m
        if out is None:
            out = _empty_colmajor(rows_out, X.shape[1], X.dtype, X.device)
        Y, ldy = _colmajor(out)
        _check(lib().bf_apply(self._h, int(bool(trans)), X.data_ptr(), ldx, X.shape[1],
                              Y.data_ptr(), ldy, _alloc_ptr(_allocator(allocator)),
                              _stream(stream)), "bf_apply")
        return Y

    def close(self, stream=None):
        """Free the factors; their memory is reused only after the work already
        enqueued on `stream` (default: torch's current stream) has finished."""
        if self._h:
            lib().bf_free(self._h, _stream(stream))
            self._h = None
            self._alloc = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def construct(op: Operator, tol: float, leaf: int, p: int = 2, r0: int = 4, seed: int = 0,
              max_rank: int = 0, stream=None, work_bytes: int = 0, progress=None,
              center="hybrid", merge_leaf: bool = True, merge_sweeps: bool = True,
              two_sides: bool = True, allocator="torch") -> Factors:
    """Alg. 2 on the device; returns the factor handle.  work_bytes bounds the
    device memory of one sweep level's samples (0: 8 GiB).  progress(phase,
    level), if given, is called after each leaf-loop iteration and sweep level
    with phase one of PHASES.  center: the level of the centre factor B --
    "hybrid" (floor(L/2)), "column" (0: column-wise factorization), "row" (L:
    row-wise), or an integer level (negative counts from L + 1).  merge_leaf:
    consecutive passes of the adaptive leaf loops share a black-box call
    (same results, fewer calls); False makes one call per pass.  merge_sweeps:
    consecutive sweep levels may share a black-box call (built-in operators
    that evaluate their entries on the fly; bf.h BF_OPT_SEQUENTIAL_SWEEP);
    False makes one call per level.  two_sides: the row side of Alg. 2 may run
    on a second stream and host thread beside the column side (built-in
    operators without a progress callback; bf.h BF_OPT_ONE_STREAM; same
    factors); False keeps everything on `stream`.  allocator:
    where the device memory comes from -- "torch" (torch's caching allocator,
    default) or None (the library's own pool)."""
    o = bf_opts(p, r0, max_rank, 0, seed, work_bytes)
    lm = CENTERS[center] if isinstance(center, str) else int(center)
    if lm is not None:
        o.flags |= BF_OPT_CENTER_LEVEL
        o.center_level = lm
    if not merge_leaf:
        o.flags |= BF_OPT_SEQUENTIAL_LEAF
    if not merge_sweeps:
        o.flags |= BF_OPT_SEQUENTIAL_SWEEP
    if not two_sides:
        o.flags |= BF_OPT_ONE_STREAM
    cb = None    # held until bf_construct returns
    if progress is not None:
        cb = PROGRESSFN(lambda _u, ph, lv: progress(PHASES[ph], lv))
        o.progress = cb
    a = _allocator(allocator)
    h = C.c_void_p()
    _check(lib().bf_construct(op._op.matvec, op._op.rmatvec, op._op.user, op.m, op.n, float(tol),
                              int(leaf), C.byref(o), _alloc_ptr(a), _stream(stream), C.byref(h)),
           "bf_construct")
    return Factors(h, leaf, a)


def import_factors(m, n, leaf, kU, kV, data, stream=None, allocator="torch") -> Factors:
    kU = np.ascontiguousarray(kU, np.int32).ravel()
    kV = np.ascontiguousarray(kV, np.int32).ravel()
    data = np.ascontiguousarray(data, np.complex128)
    a = _allocator(allocator)
    h = C.c_void_p()
    _check(lib().bf_import(m, n, leaf, kU.ctypes.data_as(_I32P), kV.ctypes.data_as(_I32P),
                           data.ctypes.data, len(data), _alloc_ptr(a), _stream(stream),
                           C.byref(h)), "bf_import")
    return Factors(h, leaf, a)


class _Borrowed(Factors):
    """Factors owned by a Server (not freed by this handle)."""

    def close(self, stream=None):
        self._h = None


class Server:
    """Request engine: concurrent constructions and applies on `slots` streams
    with admission by estimated device footprint (see include/bf.h)."""

    def __init__(self, slots=4, hbm_budget=0, batch_cols=0, allocator="torch",
                 solve_rounds=False, max_constructs=0):
        """batch_cols > 0 merges queued applies against the same factors into
        one product of at most that many columns (continuous batching).
        allocator: device memory of every request -- "torch" (torch's caching
        allocator, default) or None (the library's own pool).  solve_rounds:
        the level solves of in-flight constructions share persistent launches
        (cross-request rounds, replayed from captured graphs).  max_constructs
        > 0: at most that many constructions run at once (applies still take
        the idle slots)."""
        self._alloc = _allocator(allocator)
        o = bf_server_opts(slots, int(batch_cols), int(hbm_budget))
        o.solve_rounds = int(bool(solve_rounds))
        o.max_constructs = int(max_constructs)
        if self._alloc is not None:
            o.alloc = C.pointer(self._alloc.struct)
        h = C.c_void_p()
        _check(lib().bf_server_create(C.byref(o), C.byref(h)), "bf_server_create")
        self._h = h
        self._keep = {}

    def submit_construct(self, op: Operator, tol, leaf, p=2, r0=4, seed=0, max_rank=0,
                         work_bytes=0):
        t = C.c_int64()
        o = bf_opts(p, r0, max_rank, 0, seed, work_bytes)
        _check(lib().bf_server_submit_construct(self._h, C.byref(op._op), float(tol), int(leaf),
                                                C.byref(o), C.byref(t)), "submit_construct")
        self._keep[t.value] = (op,)
        return t.value

    def submit_apply(self, ticket, X, trans=False, out=None):
        X = _dev_c64(X)
        X, ldx = _colmajor(X)
        F = self._keep[ticket][0]
        rows_out = F.n if trans else F.m
        if out is None:
            out = _empty_colmajor(rows_out, X.shape[1], X.dtype, X.device)
        Y, ldy = _colmajor(out)
        # the device buffers are read/written on a worker stream: order them
        # after the caller's pending work on its own stream
        _torch().cuda.current_stream().synchronize()
        t = C.c_int64()
        _check(lib().bf_server_submit_apply(self._h, ticket, int(bool(trans)), X.data_ptr(), ldx,
                                            X.shape[1], Y.data_ptr(), ldy, C.byref(t)),
               "submit_apply")
        self._keep[t.value] = (X, Y)
        return t.value

    def wait(self, ticket):
        """Block until done; returns (status, info dict).  Raises on failure."""
        i = bf_request_info()
        rc = lib().bf_server_wait(self._h, ticket, C.byref(i))
        info = {f: getattr(i, f) for f, _ in bf_request_info._fields_}
        if rc != 0:
            raise BFError(rc, f"request {ticket}")
        return info

    def result(self, ticket):
        """Output of a finished apply request (the Y tensor)."""
        return self._keep[ticket][1]

    def factors(self, ticket) -> Factors:
        h = C.c_void_p()
        _check(lib().bf_server_factors(self._h, ticket, C.byref(h)), "bf_server_factors")
        return _Borrowed(h, 0)

    def rounds(self):
        """(solve rounds launched, blocks they held)."""
        r, i = C.c_int64(), C.c_int64()
        _check(lib().bf_server_rounds(self._h, C.byref(r), C.byref(i)), "bf_server_rounds")
        return r.value, i.value

    def release(self, ticket):
        _check(lib().bf_server_release(self._h, ticket), "bf_server_release")
        self._keep.pop(ticket, None)

    def close(self):
        if self._h:
            lib().bf_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def release_cached_memory():
    """Give back the device and pinned host blocks the library keeps for
    reuse after factors and temporaries are freed (bf_release_cached_memory)."""
    _check(lib().bf_release_cached_memory(), "bf_release_cached_memory")


def set_autotune(enable=True):
    """Launch-shape autotuner (bf_set_autotune; on by default)."""
    _check(lib().bf_set_autotune(1 if enable else 0), "bf_set_autotune")


def autotune_entries() -> int:
    """Shape classes in the autotuner's table (loaded or timed)."""
    n = C.c_int64(0)
    _check(lib().bf_autotune_entries(C.byref(n)), "bf_autotune_entries")
    return n.value


def autotune_save(path=None):
    """Write the autotuner's table (default: tune_gfx950.tsv beside libbf.so)."""
    _check(lib().bf_autotune_save(path.encode() if path else None), "bf_autotune_save")


def autotune_load(path=None):
    """Merge a saved table into the autotuner's."""
    _check(lib().bf_autotune_load(path.encode() if path else None), "bf_autotune_load")


def autotune_clear():
    """Empty the autotuner's table (classes are timed again on first use)."""
    _check(lib().bf_autotune_clear(), "bf_autotune_clear")


def profile_start():
    _check(lib().bf_profile_start(), "bf_profile_start")


def profile_stop():
    """Per kernel class: {launches, ms, flops, bytes} of the launches since start."""
    arr = (bf_kernel_stats * len(KERNEL_CLASSES))()
    _check(lib().bf_profile_stop(arr), "bf_profile_stop")
    return {name: {f: getattr(arr[k], f) for f, _ in bf_kernel_stats._fields_}
            for k, name in enumerate(KERNEL_CLASSES)}


def gauss(seed, tag, row0, rows, cols, device="cuda"):
    torch = _torch()
    out = _empty_colmajor(rows, cols, torch.complex128, device)
    _check(lib().bf_gauss(seed, tag, row0, rows, cols, out.data_ptr(), _stream()), "bf_gauss")
    return out


def cpqr_batched(blocks, tol, device="cuda"):
    """Truncated pivoted QR of each block (list of 2D complex arrays) on the GPU."""
    torch = _torch()
    M = np.array([b.shape[0] for b in blocks], np.int32)
    N = np.array([b.shape[1] for b in blocks], np.int32)
    zoff = np.zeros(len(blocks), np.int64)
    qoff = np.zeros(len(blocks), np.int64)
    parts, zo, qo = [], 0, 0
    for t, b in enumerate(blocks):
        zoff[t], qoff[t] = zo, qo
        parts.append(np.asarray(b, np.complex128).ravel(order="F"))
        zo += b.size
        qo += b.shape[0] * min(b.shape)
    Z = torch.from_numpy(np.concatenate(parts) if parts else np.zeros(1, np.complex128)).to(device)
    Q = torch.zeros(max(qo, 1), dtype=torch.complex128, device=device)
    ranks = np.zeros(len(blocks), np.int32)
    _check(lib().bf_cpqr_batched(len(blocks), M.ctypes.data_as(_I32P), N.ctypes.data_as(_I32P),
                                 Z.data_ptr(), zoff.ctypes.data_as(_I64P), float(tol), Q.data_ptr(),
                                 qoff.ctypes.data_as(_I64P), ranks.ctypes.data_as(_I32P),
                                 _stream()), "bf_cpqr_batched")
    Qh = Q.cpu().numpy()
    out = []
    for t, b in enumerate(blocks):
        k = int(ranks[t])
        out.append(Qh[qoff[t]:qoff[t] + b.shape[0] * k].reshape((b.shape[0], k), order="F"))
    return out, ranks


def lsq_batched(Cs, Xs, device="cuda"):
    """B_b = argmin ||C_b - B X_b||_F for each pair, on the GPU."""
    torch = _torch()
    kU = np.array([c.shape[0] for c in Cs], np.int32)
    kV = np.array([x.shape[0] for x in Xs], np.int32)
    s = np.array([x.shape[1] for x in Xs], np.int32)
    coff, xoff, boff = (np.zeros(len(Cs), np.int64) for _ in range(3))
    cp, xp, co, xo, bo = [], [], 0, 0, 0
    for t in range(len(Cs)):
        coff[t], xoff[t], boff[t] = co, xo, bo
        cp.append(np.asarray(Cs[t], np.complex128).ravel(order="F"))
        xp.append(np.asarray(Xs[t], np.complex128).ravel(order="F"))
        co += Cs[t].size
        xo += Xs[t].size
        bo += kU[t] * kV[t]
    Cd = torch.from_numpy(np.concatenate(cp)).to(device)
    Xd = torch.from_numpy(np.concatenate(xp)).to(device)
    Bd = torch.zeros(max(bo, 1), dtype=torch.complex128, device=device)
    _check(lib().bf_lsq_batched(len(Cs), kU.ctypes.data_as(_I32P), kV.ctypes.data_as(_I32P),
                                s.ctypes.data_as(_I32P), Cd.data_ptr(), coff.ctypes.data_as(_I64P),
                                Xd.data_ptr(), xoff.ctypes.data_as(_I64P), Bd.data_ptr(),
                                boff.ctypes.data_as(_I64P), _stream()), "bf_lsq_batched")
    Bh = Bd.cpu().numpy()
    return [Bh[boff[t]:boff[t] + kU[t] * kV[t]].reshape((kU[t], kV[t]), order="F")
            for t in range(len(Cs))]
