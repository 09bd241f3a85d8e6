"""Measured choice of base case, depth and addition-pass fusion per shape.

The paper selects the algorithm per shape by timing (Section 5: which base
case and how many levels win depends on m, k, n, and recursion pays only
while the leaf products stay efficient).  The library's cost model
(``rank_candidates``) is the prior; ``tune`` times the model's best few
candidates plus the classical product on the device, with each candidate's
one- and two-level fusion where both exist, records the winner in the
library (``fmm_tune_record``, which "auto" plans and the server then use for
that exact shape) and, if given a path, in a JSON cache that ``load_cache``
replays into the library in a later process.
"""
import ctypes
import json
import os

from . import F32_BF16X3, F64, FmmError, Plan, _check, _dtype_code, _lib, rank_candidates

__all__ = ["tune", "load_cache", "record", "clear"]

_lib.fmm_tune_record.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                 ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
_lib.fmm_tune_record.restype = ctypes.c_int
_lib.fmm_tune_clear.argtypes = []
_lib.fmm_tune_clear.restype = ctypes.c_int


def _key(m, k, n, dtype):
    return f"{m}x{k}x{n}:{dtype}"


def record(m, k, n, dtype, alg, levels, fuse_levels=0, leaf_tile=0):
    """Register a choice for the exact shape with the library."""
    _check(_lib.fmm_tune_record(m, k, n, _dtype_code(dtype), alg.encode(), int(levels), int(fuse_levels),
                                int(leaf_tile)))


def clear():
    _check(_lib.fmm_tune_clear())


def load_cache(path):
    """Register every entry of a JSON cache written by ``tune``; returns the count."""
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        data = json.load(f)
    for key, e in data.items():
        m, k, n = (int(x) for x in key.split(":")[0].split("x"))
        record(m, k, n, int(key.split(":")[1]), e["alg"], e["levels"], e.get("fuse_levels", 0),
               e.get("leaf_tile", 0))
    return len(data)


def _time_plan(p, A, B, C, reps, warmup):
    import torch
    s = torch.cuda.current_stream()
    for _ in range(warmup):
        p.multiply(A, B, C)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        p.multiply(A, B, C)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(m, k, n, dtype=F64, top=4, reps=3, warmup=1, cache=None, budget_bytes=0, seed=0, max_error=0.0):
    """Time the model's `top` candidates (and the classical product) for the
    shape on the current device, each with one and two levels per addition
    pass where both exist and, on the FP64 / FP32 paths, with 64 x 64 and
    128 x 128 leaf tiles; record and return the fastest as a dict
    {alg, levels, fuse_levels, leaf_tile, ms, tflops, candidates: [...]},
    where each candidate carries its model prediction and measured ms.
    Only candidates within the error budget `max_error` (0: the dtype's
    default, < 0: none) are timed, as for the automatic choice."""
    import torch
    dtype = _dtype_code(dtype)
    elt = torch.float64 if dtype == F64 else torch.float32
    cands = rank_candidates(m, k, n, dtype, budget_bytes=budget_bytes, max_error=max_error)
    trial = cands[:top]
    if not any(c["alg"] == "classical" for c in trial):
        trial += [c for c in cands if c["alg"] == "classical"]
    g = torch.Generator(device="cuda").manual_seed(seed)
    A = torch.rand((m, k), dtype=elt, device="cuda", generator=g) * 2 - 1
    B = torch.rand((k, n), dtype=elt, device="cuda", generator=g) * 2 - 1
    C = torch.empty((m, n), dtype=elt, device="cuda")
    results = []
    tiles = [0] if dtype == F32_BF16X3 else [64, 128]
    for c in trial:
        fuses = [0] if c["levels"] == 0 else ([1, 2] if c["levels"] >= 2 else [1])
        for fz in fuses:
            for tile in tiles:
                try:
                    with Plan(c["alg"], m, k, n, c["levels"], dtype, fuse_levels=fz, leaf_tile=tile) as p:
                        ms = _time_plan(p, A, B, C, reps, warmup)
                        fz_used = p.info["fuse_levels"]
                except FmmError as e:  # e.g. workspace beyond memory: not a candidate here
                    results.append(dict(c, fuse_levels=fz, leaf_tile=tile, ms=None, error=str(e)))
                    continue
                results.append(dict(c, fuse_levels=fz_used, leaf_tile=tile, ms=ms))
    ok = [r for r in results if r["ms"] is not None]
    if not ok:
        raise FmmError(2, "no candidate could run")
    best = min(ok, key=lambda r: r["ms"])
    record(m, k, n, dtype, best["alg"], best["levels"], best["fuse_levels"], best["leaf_tile"])
    out = {"alg": best["alg"], "levels": best["levels"], "fuse_levels": best["fuse_levels"],
           "leaf_tile": best["leaf_tile"],
           "ms": best["ms"], "tflops": 2.0 * m * k * n / (best["ms"] * 1e-3) / 1e12,
           "candidates": results}
    if cache:
        data = {}
        if os.path.exists(cache):
            with open(cache) as f:
                data = json.load(f)
        data[_key(m, k, n, dtype)] = {x: out[x] for x in ("alg", "levels", "fuse_levels", "leaf_tile", "ms")}
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    del A, B, C
    return out
