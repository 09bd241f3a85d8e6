"""The serving stream end to end: a Poisson stream of mixed FP64 / BF16x3
requests through the continuous-batching server, each result recomputed alone
(bit for bit) and checked against the oracle:
  FP64:   relF <= 1e-12 on sampled rows against the binary64 product
  BF16x3: relF <= 2e-6 * 2^max(L,1) against the emulated fast algorithm
(the tolerances of the other GPU tests).
"""
import numpy as np
import pytest

from oracle import algorithms, bf16x3, classical
from gpu_util import relf, say

pytestmark = pytest.mark.gpu


def test_poisson_stream_alone_vs_mix_and_oracle():
    import torch
    import paper_1409_2908_amd as F
    from paper_1409_2908_amd import serving
    n_req = 240
    reqs = serving.make_requests(21, n_req, lo=64, hi=1024)
    pools = serving.Pools(2048, seed=5)
    arr = serving.poisson_arrivals(23, n_req, 4000.0)
    say(f"case serving stream {n_req} requests")
    stats, kept = serving.run_stream(reqs, arr, pools, arena_bytes=1 << 30, max_batch=8, max_inflight=2,
                                     keep=set(range(n_req)), max_outstanding=32)
    say(f"  {stats}")
    assert stats["requests"] == n_req and stats["mean_batch"] > 1
    assert serving.check_alone(kept) == n_req
    rng = np.random.default_rng(3)
    for idx, r in kept.items():
        A = r["A"].cpu().numpy()
        B = r["B"].cpu().numpy()
        C = r["C"].cpu().numpy()
        c = r["completion"]
        if r["dtype"] == F.F64:
            rows = np.unique(np.concatenate([[0, A.shape[0] - 1], rng.integers(0, A.shape[0], 6)]))
            ref = classical.gemm_rows(A, B, rows)
            assert relf(C[rows], ref) <= 1e-12, (idx, c)
        else:
            a = None if c["alg"] == "classical" else algorithms.get(c["alg"])
            emu = bf16x3.gemm(A, B) if a is None else bf16x3.fmm(a, c["levels"], A, B)
            assert relf(C, emu) <= 2e-6 * 2 ** max(c["levels"], 1), (idx, c)
    torch.cuda.synchronize()


def test_graph_served_batches_equal_eager():
    """With one recorded HIP graph per batch, every request's result is bit
    for bit the same plan run alone (the graph holds the same kernels with
    the same arguments)."""
    import torch
    from paper_1409_2908_amd import serving
    n_req = 120
    reqs = serving.make_requests(31, n_req, lo=64, hi=1024)
    pools = serving.Pools(2048, seed=7)
    arr = np.zeros(n_req)
    say(f"case graph-served stream {n_req} requests")
    stats, kept = serving.run_stream(reqs, arr, pools, arena_bytes=1 << 30, max_batch=8, max_inflight=2,
                                     keep=set(range(n_req)), max_outstanding=32, use_graph=True)
    say(f"  {stats}")
    assert stats["requests"] == n_req and stats["mean_batch"] > 1
    assert serving.check_alone(kept) == n_req
    torch.cuda.synchronize()
