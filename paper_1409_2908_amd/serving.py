"""Serving driver: a Poisson stream of multiply requests through the
continuous-batching server (``fmm_server_*``), against one-at-a-time
classical GEMM on the same arrival sequence.

Operands stay on the device: every request's A and B are views, at seeded
random offsets, into two resident pools per dtype filled once with
uniform[-1, 1) values, so a stream of thousands of requests (over a TiB of
operands in total) needs only the pools plus the outputs in flight.  Each C
is allocated when its request arrives and released when it completes.

Latency is arrival -> completion event seen by the host; throughput is
requests (and effective 2mkn flops) per second of wall time from the first
arrival to the last completion.
"""
import math
import time

import numpy as np

from . import F32_BF16X3, F64, Plan, Server

# the library's default large-request threshold (FMM_SERVER_LARGE_FLOPS, 2mkn)
LARGE_FLOPS = 6.0e10

__all__ = ["make_requests", "Pools", "run_stream", "percentile", "check_alone"]


def make_requests(seed, count, lo=256, hi=8192, fp32_dtype=F32_BF16X3):
    """count requests (m, k, n, dtype): each dimension log-uniform on [lo, hi],
    dtype FP64 or FP32 with probability 1/2 each (FP32 computed as
    `fp32_dtype`)."""
    rng = np.random.default_rng(seed)
    dims = np.exp(rng.uniform(math.log(lo), math.log(hi), (count, 3)))
    dims = np.clip(np.rint(dims).astype(np.int64), lo, hi)
    fp64 = rng.random(count) < 0.5
    return [(int(m), int(k), int(n), F64 if f else fp32_dtype) for (m, k, n), f in zip(dims, fp64)]


def poisson_arrivals(seed, count, rate_per_s):
    """Arrival times in ms of a Poisson process of the given rate (first at 0)."""
    rng = np.random.default_rng(seed + 1)
    gaps = rng.exponential(1e3 / rate_per_s, count)
    gaps[0] = 0.0
    return np.cumsum(gaps)


class Pools:
    """Resident operand pools (side x side) per element type, and seeded
    offsets for each request's views."""

    def __init__(self, side, seed=0, dtypes=(F64, F32_BF16X3)):
        import torch
        self.side = side
        self.mats = {}
        g = torch.Generator(device="cuda").manual_seed(seed)
        for elt in {torch.float64 if d == F64 else torch.float32 for d in dtypes}:
            self.mats[elt] = [torch.rand((side, side), dtype=elt, device="cuda", generator=g) * 2 - 1
                              for _ in range(2)]
        self.rng = np.random.default_rng(seed + 2)

    def operands(self, m, k, n, dtype):
        import torch
        elt = torch.float64 if dtype == F64 else torch.float32
        PA, PB = self.mats[elt]
        r0, c0 = (int(x) for x in self.rng.integers(0, self.side - np.array([m, k]) + 1))
        r1, c1 = (int(x) for x in self.rng.integers(0, self.side - np.array([k, n]) + 1))
        return PA[r0:r0 + m, c0:c0 + k], PB[r1:r1 + k, c1:c1 + n]


def percentile(x, q):
    return float(np.percentile(np.asarray(x, dtype=np.float64), q)) if len(x) else float("nan")


def run_stream(requests, arrivals_ms, pools, arena_bytes, max_batch=8, max_inflight=2, alg=None,
               levels=-1, keep=None, max_outstanding=64, use_graph=False, num_streams=1, large_flops=0.0,
               small_model=False):
    """Replay the stream in real time through a server.  `alg`/`levels` apply
    to every request (None / -1: the library's per-shape choice).  At most
    `max_outstanding` requests are submitted and unfinished at once (their
    outputs are allocated); later arrivals wait on the host, and that wait
    counts in their latency.  `keep` is a set of request indices whose A, B,
    C, dtype and completion are returned for checking.  use_graph: every batch
    runs as one recorded HIP graph.  Returns a dict of metrics and the kept
    results."""
    import torch
    n = len(requests)
    lat, flops = np.zeros(n), 0.0
    kept = {}
    meta = {}
    batches = []
    algs = {}
    srv = Server(arena_bytes, max_batch=max_batch, max_inflight=max_inflight, use_graph=use_graph,
                 num_streams=num_streams, large_flops=large_flops, small_model=small_model)
    arena_gb = srv.arena_bytes / 1e9
    lanes = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i = done = 0

    def collect(comps):
        nonlocal done
        for c in comps:
            idx, arr_ms, sub_wall = meta.pop(c["id"])
            if c["status"] != 0:
                raise RuntimeError(f"request {idx} failed with status {c['status']}")
            # host delay from arrival to submit, plus the server's submit -> done
            lat[idx] = (sub_wall - arr_ms) + (c["done_ms"] - c["submit_ms"])
            batches.append(c["batch_size"])
            lanes[c["lane"]] = lanes.get(c["lane"], 0) + 1
            key = f"{c['alg']}/L{c['levels']}"
            algs[key] = algs.get(key, 0) + 1
            if idx in kept:
                kept[idx]["completion"] = c
            done += 1

    while done < n:
        now = (time.perf_counter() - t0) * 1e3
        while i < n and arrivals_ms[i] <= now and srv.pending < max_outstanding:
            m, k, nn, dt = requests[i]
            A, B = pools.operands(m, k, nn, dt)
            rid, C = srv.submit(A, B, dtype=dt, alg=alg, levels=levels)
            meta[rid] = (i, arrivals_ms[i], (time.perf_counter() - t0) * 1e3)
            if keep is not None and i in keep:
                kept[i] = {"A": A, "B": B, "C": C, "dtype": dt}
            flops += 2.0 * m * k * nn
            i += 1
            now = (time.perf_counter() - t0) * 1e3
        comps = srv.progress()
        if comps:
            collect(comps)
            continue
        if i < n and srv.pending < max_outstanding:
            wait_ms = arrivals_ms[i] - (time.perf_counter() - t0) * 1e3
            if wait_ms > 0.2 and srv.pending == 0:
                time.sleep(min(wait_ms, 5.0) * 1e-3)
            elif wait_ms > 0.05:
                time.sleep(2e-5)
        else:
            collect(srv.progress(wait=True))
    wall = time.perf_counter() - t0
    srv.close()
    # the server's large-request class (the library default threshold for 0)
    thr = large_flops or LARGE_FLOPS
    small = np.array([2.0 * m * k * nn < thr for m, k, nn, _ in requests])
    return {
        "requests": n,
        "wall_s": wall,
        "req_per_s": n / wall,
        "eff_tflops": flops / wall / 1e12,
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
        "p99_ms_below_large": percentile(lat[small], 99) if small.any() else 0.0,
        "p99_ms_large": percentile(lat[~small], 99) if (~small).any() else 0.0,
        "mean_batch": float(np.mean(batches)) if batches else 0.0,
        "arena_gb": round(arena_gb, 1),
        "requests_per_stream": {str(k): v for k, v in sorted(lanes.items())},
        "plans": dict(sorted(algs.items(), key=lambda kv: -kv[1])),
    }, kept


def check_alone(kept):
    """Recompute each kept request alone (same base case and depth, eager
    fmm_multiply) and compare with its result from the mix, bit for bit.
    Returns the number of requests checked; raises on a mismatch."""
    import torch
    for idx, r in kept.items():
        A, B, C, c = r["A"], r["B"], r["C"], r["completion"]
        with Plan(c["alg"], A.shape[0], A.shape[1], B.shape[1], c["levels"], dtype=r["dtype"]) as p:
            alone = p.multiply(A, B)
        torch.cuda.synchronize()
        if not torch.equal(alone, C):
            raise AssertionError(f"request {idx}: result in the mix differs from the same plan alone")
    return len(kept)
