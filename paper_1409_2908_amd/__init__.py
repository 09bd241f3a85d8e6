"""MI355X recursive fast matrix multiplication (Benson and Ballard, PPoPP 2015).

A thin ctypes binding over the C ABI in ``include/fmm.h``: every step of the
path (operand formation, grouped leaf GEMMs, W-combination) runs in the HIP
kernels of ``libfmm.so``.  This module only marshals arguments; it raises
``FmmError`` with the library's message on any non-zero status, and
``ImportError`` if the built library is missing (there is no fallback).
PyTorch supplies device memory and streams.
"""
import ctypes
import os

import numpy as np

__all__ = ["FmmError", "Plan", "Server", "gemm", "multiply_batched", "rank_candidates",
           "algorithm_coeffs", "algorithm_names",
           "check_algorithms", "library_path", "F64", "F32", "F32_BF16X3",
           "STAGE_FORM_S", "STAGE_FORM_T", "STAGE_LEAF", "STAGE_COMBINE", "LOC_A", "LOC_B",
           "LOC_C", "LOC_WORKSPACE"]

F64, F32, F32_BF16X3 = 0, 1, 2
STAGE_FORM_S, STAGE_FORM_T, STAGE_LEAF, STAGE_COMBINE = 0, 1, 2, 3
LOC_A, LOC_B, LOC_C, LOC_WORKSPACE = 0, 1, 2, 3
NOALLOC_MAX_BYTES = 64 << 20  # FMM_NOALLOC_MAX_BYTES of fmm.h
_DTYPE_NAMES = {"f64": F64, "float64": F64, "f32": F32, "float32": F32, "bf16x3": F32_BF16X3,
                "f32_bf16x3": F32_BF16X3}

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path():
    return os.path.join(_HERE, "libfmm.so")


class FmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fmm status {code}: {msg}")
        self.code = code


class _Info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("k", ctypes.c_int64), ("n", ctypes.c_int64),
                ("levels", ctypes.c_int), ("dtype", ctypes.c_int),
                ("M", ctypes.c_int), ("K", ctypes.c_int), ("N", ctypes.c_int), ("R", ctypes.c_int),
                ("m0", ctypes.c_int64), ("k0", ctypes.c_int64), ("n0", ctypes.c_int64),
                ("leaf_m", ctypes.c_int64), ("leaf_k", ctypes.c_int64), ("leaf_n", ctypes.c_int64),
                ("num_leaves", ctypes.c_int64), ("num_s_materialized", ctypes.c_int64),
                ("num_t_materialized", ctypes.c_int64), ("num_gemm_problems", ctypes.c_int64),
                ("gemm_tiles", ctypes.c_int64), ("workspace_bytes", ctypes.c_size_t),
                ("leaf_flops", ctypes.c_double), ("classical_flops", ctypes.c_double),
                ("add_bytes", ctypes.c_double), ("gemm_min_bytes", ctypes.c_double),
                ("fuse_levels", ctypes.c_int), ("alg", ctypes.c_char * 80), ("leaf_tile", ctypes.c_int),
                ("pair_form", ctypes.c_int), ("error_bound", ctypes.c_double), ("leaf_form", ctypes.c_int)]


class _Options(ctypes.Structure):
    _fields_ = [("fuse_levels", ctypes.c_int), ("host_only", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("defer_device_memory", ctypes.c_int),
                ("leaf_tile", ctypes.c_int), ("max_error", ctypes.c_double), ("leaf_form", ctypes.c_int)]


class _Candidate(ctypes.Structure):
    _fields_ = [("alg", ctypes.c_char * 80), ("levels", ctypes.c_int), ("fuse_levels", ctypes.c_int),
                ("leaf_tile", ctypes.c_int), ("model_ms", ctypes.c_double), ("leaf_ms", ctypes.c_double),
                ("add_ms", ctypes.c_double), ("workspace_bytes", ctypes.c_size_t), ("error_bound", ctypes.c_double)]


class _ServerOptions(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_size_t), ("max_batch", ctypes.c_int),
                ("max_inflight", ctypes.c_int), ("fuse_levels", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("max_error", ctypes.c_double * 3), ("num_streams", ctypes.c_int),
                ("large_flops", ctypes.c_double), ("small_model", ctypes.c_int)]


class _Request(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("k", ctypes.c_int64), ("n", ctypes.c_int64),
                ("dtype", ctypes.c_int), ("alg", ctypes.c_char_p), ("levels", ctypes.c_int),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64), ("B", ctypes.c_void_p),
                ("ldb", ctypes.c_int64), ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64),
                ("user", ctypes.c_void_p), ("wait_stream", ctypes.c_int), ("stream", ctypes.c_void_p)]


class _Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("user", ctypes.c_void_p), ("status", ctypes.c_int),
                ("submit_ms", ctypes.c_double), ("launch_ms", ctypes.c_double),
                ("done_ms", ctypes.c_double), ("batch_size", ctypes.c_int),
                ("alg", ctypes.c_char * 80), ("levels", ctypes.c_int), ("lane", ctypes.c_int)]


def _load():
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() "
                          "or python paper_1409_2908_amd/build.py")
    # torch first: its wheel carries its own HIP runtime (soname
    # libamdhip64.so.7).  Loaded before libfmm.so, that runtime satisfies the
    # library's dependency, so the process has one HIP runtime; loaded after,
    # a second runtime would be mapped from the ROCm install and would find
    # no usable device once torch's runtime holds it.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    i64, i32, vp, dp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_double
    P = ctypes.c_void_p
    sig = {
        "fmm_plan": ([ctypes.POINTER(P), ctypes.c_char_p, i64, i64, i64, i32, i32], i32),
        "fmm_plan_host": ([ctypes.POINTER(P), ctypes.c_char_p, i64, i64, i64, i32, i32], i32),
        "fmm_plan_ex": ([ctypes.POINTER(P), ctypes.c_char_p, i64, i64, i64, i32, i32,
                         ctypes.POINTER(_Options)], i32),
        "fmm_multiply": ([P, vp, i64, vp, i64, vp, i64, vp], i32),
        "fmm_multiply_noalloc": ([P, vp, i64, vp, i64, vp, i64, vp], i32),
        "fmm_multiply_batched": ([ctypes.POINTER(P), ctypes.POINTER(vp), ctypes.POINTER(i64),
                                  ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(vp),
                                  ctypes.POINTER(i64), i32, vp], i32),
        "fmm_plan_device_bytes": ([P], ctypes.c_size_t),
        "fmm_plan_bind": ([P, vp, ctypes.c_size_t, vp], i32),
        "fmm_rank_candidates": ([i64, i64, i64, i32, ctypes.c_char_p, ctypes.c_size_t, dp,
                                 ctypes.POINTER(_Candidate), i32, ctypes.POINTER(i32)], i32),
        "fmm_server_create": ([ctypes.POINTER(P), ctypes.POINTER(_ServerOptions), vp], i32),
        "fmm_server_submit": ([P, ctypes.POINTER(_Request), ctypes.POINTER(i64)], i32),
        "fmm_server_progress": ([P, i32, ctypes.POINTER(_Completion), i32, ctypes.POINTER(i32)], i32),
        "fmm_server_pending": ([P], i64),
        "fmm_server_arena_bytes": ([P], ctypes.c_size_t),
        "fmm_server_destroy": ([P], i32),
        "fmm_run_stage": ([P, i32, vp, i64, vp, i64, vp, i64, vp], i32),
        "fmm_plan_operand": ([P, i32, i64, ctypes.POINTER(i32), ctypes.POINTER(i64),
                              ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                              ctypes.POINTER(dp)], i32),
        "fmm_plan_workspace": ([P], vp),
        "fmm_plan_workspace_bytes": ([P], ctypes.c_size_t),
        "fmm_plan_info": ([P, ctypes.POINTER(_Info)], i32),
        "fmm_plan_enable_timing": ([P, i32], i32),
        "fmm_plan_stage_ms": ([P, ctypes.POINTER(dp)], i32),
        "fmm_plan_destroy": ([P], i32),
        "fmm_gemm": ([i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp], i32),
        "fmm_num_algorithms": ([], i32),
        "fmm_algorithm_name": ([i32], ctypes.c_char_p),
        "fmm_algorithm_coeffs": ([ctypes.c_char_p] + [ctypes.POINTER(i32)] * 4 + [vp] * 3, i32),
        "fmm_check_algorithms": ([], i32),
        "fmm_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def _check(status):
    if status != 0:
        raise FmmError(status, _lib.fmm_last_error().decode())


def _dtype_code(dtype):
    if isinstance(dtype, str):
        return _DTYPE_NAMES[dtype]
    return int(dtype)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _mat(t, name, elt):
    """(pointer, leading dimension) of a row-major (unit column stride) tensor."""
    import torch
    if t.dtype != elt:
        raise TypeError(f"{name} must be {elt}, got {t.dtype}")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if t.numel() and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride (row-major)")
    if t.numel() and not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.size(0) > 1 and t.numel() and t.stride(0) < t.size(1):
        # rows would overlap (an expanded or overlapping view): the library
        # would read or write past the tensor's storage
        raise ValueError(f"{name} must have row stride >= its number of columns, got stride "
                         f"{t.stride(0)} for {t.size(1)} columns")
    ld = t.stride(0) if t.size(0) > 1 else max(t.size(1), 1)
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0), ld


class Plan:
    """A planned product C = A @ B (``fmm_plan``).  ``host_only`` plans
    (``fmm_plan_host``) can be inspected but not run."""

    def __init__(self, alg, m, k, n, levels, dtype=F64, host_only=False, fuse_levels=0,
                 use_graph=False, defer_device_memory=False, leaf_tile=0, max_error=0.0, leaf_form=0):
        self._p = ctypes.c_void_p()
        self.dtype = _dtype_code(dtype)
        opts = _Options(int(fuse_levels), 1 if host_only else 0, 1 if use_graph else 0,
                        1 if defer_device_memory else 0, int(leaf_tile), float(max_error), int(leaf_form))
        _check(_lib.fmm_plan_ex(ctypes.byref(self._p), alg.encode(), m, k, n, levels, self.dtype,
                                ctypes.byref(opts)))
        self.m, self.k, self.n = m, k, n
        inf = self.info
        # "auto" / levels -1 resolve to the cost model's choice
        self.alg, self.levels = inf["alg"], inf["levels"]
        self.host_only = host_only

    def _elt(self):
        import torch
        return torch.float64 if self.dtype == F64 else torch.float32

    @property
    def info(self):
        inf = _Info()
        _check(_lib.fmm_plan_info(self._p, ctypes.byref(inf)))
        d = {f: getattr(inf, f) for f, _ in _Info._fields_}
        d["alg"] = d["alg"].decode()
        return d

    @property
    def device_bytes(self):
        """Bytes fmm_plan_bind needs (workspace + tables) for deferred plans."""
        return int(_lib.fmm_plan_device_bytes(self._p))

    def bind(self, ptr, nbytes, stream=None):
        """Bind device memory [ptr, ptr + nbytes) to a defer_device_memory plan."""
        _check(_lib.fmm_plan_bind(self._p, ctypes.c_void_p(int(ptr)), int(nbytes), _stream_ptr(stream)))

    @property
    def workspace_bytes(self):
        return int(_lib.fmm_plan_workspace_bytes(self._p))

    @property
    def workspace_ptr(self):
        return _lib.fmm_plan_workspace(self._p)

    def _args(self, A, B, C):
        import torch
        elt = self._elt()
        if C is None:
            C = torch.empty((self.m, self.n), dtype=elt, device=A.device)
        if tuple(A.shape) != (self.m, self.k) or tuple(B.shape) != (self.k, self.n) \
                or tuple(C.shape) != (self.m, self.n):
            raise ValueError(f"shapes {tuple(A.shape)} {tuple(B.shape)} {tuple(C.shape)} do not "
                             f"match the plan ({self.m}, {self.k}, {self.n})")
        a, lda = _mat(A, "A", elt)
        b, ldb = _mat(B, "B", elt)
        c, ldc = _mat(C, "C", elt)
        return a, lda, b, ldb, c, ldc, C

    def multiply(self, A, B, C=None, stream=None):
        a, lda, b, ldb, c, ldc, C = self._args(A, B, C)
        _check(_lib.fmm_multiply(self._p, a, lda, b, ldb, c, ldc, _stream_ptr(stream)))
        return C

    def multiply_noalloc(self, A, B, C, stream=None):
        """C = A @ B through fmm_multiply_noalloc: the workspace and tables go
        into the library's fixed device array (at most NOALLOC_MAX_BYTES), so
        nothing is allocated; C must be given."""
        if C is None:
            raise ValueError("multiply_noalloc needs the output tensor C")
        a, lda, b, ldb, c, ldc, C = self._args(A, B, C)
        _check(_lib.fmm_multiply_noalloc(self._p, a, lda, b, ldb, c, ldc, _stream_ptr(stream)))
        return C

    def run_stage(self, stage, A, B, C=None, stream=None):
        a, lda, b, ldb, c, ldc, C = self._args(A, B, C)
        _check(_lib.fmm_run_stage(self._p, stage, a, lda, b, ldb, c, ldc, _stream_ptr(stream)))
        return C

    def operand(self, side, leaf):
        """(loc, offset, row, col, ld, alpha) of a leaf operand (fmm_plan_operand)."""
        loc = ctypes.c_int()
        off, row, col, ld = (ctypes.c_int64() for _ in range(4))
        alpha = ctypes.c_double()
        _check(_lib.fmm_plan_operand(self._p, side, leaf, ctypes.byref(loc), ctypes.byref(off),
                                     ctypes.byref(row), ctypes.byref(col), ctypes.byref(ld),
                                     ctypes.byref(alpha)))
        return loc.value, off.value, row.value, col.value, ld.value, alpha.value

    def enable_timing(self, slots=64):
        """Record per-stage HIP events for the next multiplies (ring of `slots`)."""
        _check(_lib.fmm_plan_enable_timing(self._p, int(slots)))

    def stage_ms(self):
        out = (ctypes.c_double * 4)()
        _check(_lib.fmm_plan_stage_ms(self._p, out))
        return list(out)

    def close(self):
        if self._p:
            _check(_lib.fmm_plan_destroy(self._p))
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._p:
                _lib.fmm_plan_destroy(self._p)
                self._p = ctypes.c_void_p()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def gemm(A, B, C=None, dtype=None, stream=None):
    """Classical C = A @ B with the library's MFMA kernel (fmm_gemm)."""
    import torch
    if dtype is None:
        dtype = F64 if A.dtype == torch.float64 else F32
    dtype = _dtype_code(dtype)
    elt = torch.float64 if dtype == F64 else torch.float32
    m, k = A.shape
    n = B.shape[1]
    if C is None:
        C = torch.empty((m, n), dtype=elt, device=A.device)
    a, lda = _mat(A, "A", elt)
    b, ldb = _mat(B, "B", elt)
    c, ldc = _mat(C, "C", elt)
    _check(_lib.fmm_gemm(dtype, m, k, n, a, lda, b, ldb, c, ldc, _stream_ptr(stream)))
    return C


def multiply_batched(plans, As, Bs, Cs=None, stream=None):
    """C[i] = A[i] @ B[i] for every i as one batch (fmm_multiply_batched)."""
    n = len(plans)
    if Cs is None:
        Cs = [None] * n
    if not (len(As) == len(Bs) == len(Cs) == n):
        raise ValueError("plans, As, Bs and Cs must have the same length")
    P = (ctypes.c_void_p * n)()
    pa, pb, pc = (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)()
    la, lb, lc = (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)()
    outs = []
    for i, (p, A, B, C) in enumerate(zip(plans, As, Bs, Cs)):
        a, lda, b, ldb, c, ldc, C = p._args(A, B, C)
        P[i] = p._p.value
        pa[i], pb[i], pc[i] = a.value, b.value, c.value
        la[i], lb[i], lc[i] = lda, ldb, ldc
        outs.append(C)
    _check(_lib.fmm_multiply_batched(P, pa, la, pb, lb, pc, lc, n, _stream_ptr(stream)))
    return outs


def rank_candidates(m, k, n, dtype=F64, alg=None, budget_bytes=0, max_count=4096, max_error=0.0):
    """The cost model's candidates (fmm_rank_candidates), best predicted first;
    max_error 0 applies the dtype's default error budget, < 0 none."""
    out = (_Candidate * max_count)()
    cnt = ctypes.c_int()
    _check(_lib.fmm_rank_candidates(m, k, n, _dtype_code(dtype), alg.encode() if alg else None,
                                    int(budget_bytes), float(max_error), out, max_count, ctypes.byref(cnt)))
    res = []
    for c in out[:cnt.value]:
        d = {f: getattr(c, f) for f, _ in _Candidate._fields_}
        d["alg"] = d["alg"].decode()
        res.append(d)
    return res


class Server:
    """Continuous-batching request server (fmm_server_*).  Keeps the operand
    tensors of every request alive until its completion has been returned."""

    def __init__(self, arena_bytes, max_batch=8, max_inflight=2, fuse_levels=0, stream=None, use_graph=False,
                 max_error=(0.0, 0.0, 0.0), num_streams=1, large_flops=0.0, small_model=False):
        """arena_bytes 0: the device's free memory less a reserve.  num_streams
        2-4: large requests (2mkn >= large_flops, 0 = the library default) run
        one per batch on stream 0, the rest on the other streams.  Requests
        below large_flops without a named plan run the classical product
        unless small_model."""
        self._s = ctypes.c_void_p()
        opts = _ServerOptions(int(arena_bytes), int(max_batch), int(max_inflight), int(fuse_levels),
                              1 if use_graph else 0, (ctypes.c_double * 3)(*[float(x) for x in max_error]),
                              int(num_streams), float(large_flops), 1 if small_model else 0)
        sp = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(_lib.fmm_server_create(ctypes.byref(self._s), ctypes.byref(opts), sp))
        self._live = {}

    def submit(self, A, B, C=None, dtype=None, alg=None, levels=-1, stream=None):
        """Queue C = A @ B; returns (request id, C).  The request's batch runs
        after the work enqueued so far on `stream` (default: torch's current
        stream), which made A and B and last used C's memory."""
        import torch
        if dtype is None:
            dtype = F64 if A.dtype == torch.float64 else F32
        dtype = _dtype_code(dtype)
        elt = torch.float64 if dtype == F64 else torch.float32
        m, k = A.shape
        n = B.shape[1]
        if C is None:
            C = torch.empty((m, n), dtype=elt, device=A.device)
        a, lda = _mat(A, "A", elt)
        b, ldb = _mat(B, "B", elt)
        c, ldc = _mat(C, "C", elt)
        algb = alg.encode() if alg else None
        req = _Request(m, k, n, dtype, algb, int(levels), a, lda, b, ldb, c, ldc, None, 1, _stream_ptr(stream))
        rid = ctypes.c_int64()
        _check(_lib.fmm_server_submit(self._s, ctypes.byref(req), ctypes.byref(rid)))
        self._live[rid.value] = (A, B, C)
        return rid.value, C

    def progress(self, wait=False, max_done=1024):
        """Completions since the last call: dicts with id, status, times (ms)."""
        out = (_Completion * max_done)()
        cnt = ctypes.c_int()
        _check(_lib.fmm_server_progress(self._s, 1 if wait else 0, out, max_done, ctypes.byref(cnt)))
        res = []
        for c in out[:cnt.value]:
            d = {f: getattr(c, f) for f, _ in _Completion._fields_ if f != "user"}
            d["alg"] = d["alg"].decode()
            self._live.pop(d["id"], None)
            res.append(d)
        return res

    @property
    def pending(self):
        return int(_lib.fmm_server_pending(self._s))

    @property
    def arena_bytes(self):
        return int(_lib.fmm_server_arena_bytes(self._s))

    def close(self):
        if self._s:
            _check(_lib.fmm_server_destroy(self._s))
            self._s = ctypes.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def algorithm_names():
    return [_lib.fmm_algorithm_name(i).decode() for i in range(_lib.fmm_num_algorithms())]


def algorithm_coeffs(name):
    """(M, K, N, R, U, V, W) of a compiled-in base case, U/V/W as int numpy arrays."""
    dims = [ctypes.c_int() for _ in range(4)]
    _check(_lib.fmm_algorithm_coeffs(name.encode(), *[ctypes.byref(d) for d in dims], None, None, None))
    M, K, N, R = (d.value for d in dims)
    U = np.zeros((M * K, R), dtype=np.int8)
    V = np.zeros((K * N, R), dtype=np.int8)
    W = np.zeros((M * N, R), dtype=np.int8)
    _check(_lib.fmm_algorithm_coeffs(name.encode(), *[ctypes.byref(d) for d in dims],
                                     U.ctypes.data, V.ctypes.data, W.ctypes.data))
    return M, K, N, R, U.astype(int), V.astype(int), W.astype(int)


def check_algorithms():
    _check(_lib.fmm_check_algorithms())
