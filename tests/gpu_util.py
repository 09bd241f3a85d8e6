"""Helpers for the GPU tests (test infrastructure)."""
import ctypes
import os
import sys

import numpy as np

_hip = None


def hip():
    global _hip
    if _hip is None:
        import torch  # noqa: F401  (bind to the HIP runtime torch loaded)
        _hip = ctypes.CDLL("libamdhip64.so.7")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
        _hip.hipDeviceSynchronize.restype = ctypes.c_int
    return _hip


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def ws_read(plan, elem_offset, rows, cols, ld, dtype):
    """Copy a rows x cols region (leading dimension ld) of a plan's workspace."""
    es = np.dtype(dtype).itemsize
    flat = np.zeros(rows * ld, dtype=dtype)
    count = (rows - 1) * ld + cols if rows and cols else 0
    if count:
        assert hip().hipDeviceSynchronize() == 0
        src = plan.workspace_ptr + elem_offset * es
        assert hip().hipMemcpy(flat.ctypes.data, src, count * es, 2) == 0  # device to host
    return flat.reshape(rows, ld)[:, :cols].copy()


def ws_write(plan, elem_offset, X, ld):
    """Write matrix X into a plan's workspace at elem_offset with leading dim ld."""
    rows, cols = X.shape
    es = X.dtype.itemsize
    buf = np.zeros((rows, ld), dtype=X.dtype)
    buf[:, :cols] = X
    flat = buf.reshape(-1)[:(rows - 1) * ld + cols]
    dst = plan.workspace_ptr + elem_offset * es
    assert hip().hipMemcpy(dst, flat.ctypes.data, flat.nbytes, 1) == 0  # host to device
    assert hip().hipDeviceSynchronize() == 0


def relf(C, ref):
    C = np.asarray(C, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(C - ref) / den) if den else float(np.linalg.norm(C))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
