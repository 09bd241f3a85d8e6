"""The serving stream end to end: a Poisson stream of mixed FP64 / BF16x3
requests through the continuous-batching server, each result recomputed alone
(bit for bit) and checked against the oracle:
  FP64:   relF <= 1e-12 on sampled rows against the binary64 product
  BF16x3: relF <= 2e-6 * 2^max(L,1) against the emulated fast algorithm
          (small requests), and relF <= oracle.bf16x3.gate(plan, k) against
          the binary64 product on sampled rows (every request)
(the tolerances of the other GPU tests).  The stream of the serving
workload's own sizes (m, k, n log-uniform on [256, 8192]) runs the model's
choice per request: fast base cases at one to three levels, 64 and 128 wide
leaf tiles.
"""
import numpy as np
import pytest

from oracle import algorithms, bf16x3, classical
from gpu_util import relf, say

import fmm_inputs


def _plan_algs(c):
    """Oracle base cases of a completion's plan (None for classical)."""
    if c["alg"] == "classical" or c["levels"] == 0:
        return None
    names = c["alg"].split("+")
    return [algorithms.get(x) for x in names] if len(names) > 1 else algorithms.get(names[0])


def _check_sampled_rows(F, kept, seed, rows_per_request=8):
    """Every kept request against the binary64 oracle on sampled rows; returns
    the largest error and the largest error / gate per dtype."""
    worst = {}
    for idx, r in sorted(kept.items()):
        c = r["completion"]
        m, k = r["A"].shape
        rows = fmm_inputs.sample_rows(seed + idx, m, rows_per_request, [0, m - 1])
        import torch
        ri = torch.from_numpy(rows).to(r["A"].device)
        Ar = r["A"][ri].double().cpu().numpy()
        Bh = r["B"].double().cpu().numpy()
        got = r["C"][ri].double().cpu().numpy()
        ref = classical.gemm_rows(Ar, Bh, np.arange(len(rows)))
        err = relf(got, ref)
        tol = 1e-12 if r["dtype"] == F.F64 else bf16x3.gate(_plan_algs(c), c["levels"], k)
        assert err <= tol, (idx, c["alg"], c["levels"], (m, k, r["B"].shape[1]), err, tol)
        w = worst.setdefault(r["dtype"], [0.0, 0.0])
        w[0] = max(w[0], err)
        w[1] = max(w[1], err / tol)
    return worst

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
    # small_model: the model's choice for these small requests too, so that
    # fast plans share batches
    stats, kept = serving.run_stream(reqs, arr, pools, arena_bytes=1 << 30, max_batch=8, max_inflight=2,
                                     keep=set(range(n_req)), max_outstanding=32, small_model=True)
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
    _check_sampled_rows(F, kept, 200)
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
                                     keep=set(range(n_req)), max_outstanding=32, use_graph=True,
                                     small_model=True)
    say(f"  {stats}")
    assert stats["requests"] == n_req and stats["mean_batch"] > 1
    assert serving.check_alone(kept) == n_req
    torch.cuda.synchronize()


def test_serving_workload_sizes_alone_vs_mix_and_oracle():
    """240 requests with m, k, n log-uniform on [256, 8192] (the serving
    workload's range), FP64 and BF16x3 1:1, each planned by the model: every
    result is bitwise the same plan alone, and within its gate against the
    binary64 oracle on sampled rows."""
    import torch
    import paper_1409_2908_amd as F
    from paper_1409_2908_amd import serving
    n_req = 240
    reqs = serving.make_requests(41, n_req)
    pools = serving.Pools(8192, seed=9)
    arr = serving.poisson_arrivals(43, n_req, 3000.0)
    say(f"case serving workload sizes {n_req} requests")
    stats, kept = serving.run_stream(reqs, arr, pools, arena_bytes=64 << 30, max_batch=8, max_inflight=2,
                                     keep=set(range(n_req)), max_outstanding=32)
    say(f"  {stats}")
    assert stats["requests"] == n_req
    fast = sum(v for key, v in stats["plans"].items() if not key.startswith("classical"))
    assert fast >= 10, stats["plans"]
    assert serving.check_alone(kept) == n_req
    worst = _check_sampled_rows(F, kept, 100)
    say(f"  oracle on sampled rows: worst relF / ratio to gate per dtype {worst}")
    torch.cuda.synchronize()


def test_three_streams_classes_alone_vs_mix_and_oracle():
    """Three server streams: every request of 2mkn >= the large threshold runs
    alone in its batch on stream 0 with the model's plan, every other request
    on streams 1-2 with the classical plan (the default for small requests);
    each result is bitwise the same plan run alone and within its gate
    against the binary64 oracle on sampled rows (the lanes share no device
    memory)."""
    import torch
    import paper_1409_2908_amd as F
    from paper_1409_2908_amd import serving
    n_req = 200
    reqs = serving.make_requests(51, n_req)
    pools = serving.Pools(8192, seed=11)
    arr = serving.poisson_arrivals(53, n_req, 3000.0)
    thr = 2.0 * 2048 ** 3
    say(f"case serving three streams {n_req} requests")
    stats, kept = serving.run_stream(reqs, arr, pools, arena_bytes=64 << 30, max_batch=8, max_inflight=2,
                                     keep=set(range(n_req)), max_outstanding=32, num_streams=3,
                                     large_flops=thr)
    say(f"  {stats}")
    assert stats["requests"] == n_req
    n_large = 0
    for idx, r in kept.items():
        c = r["completion"]
        m, k = r["A"].shape
        n = r["B"].shape[1]
        if 2.0 * m * k * n >= thr:
            n_large += 1
            assert c["lane"] == 0 and c["batch_size"] == 1, (idx, c)
        else:
            assert c["lane"] in (1, 2) and c["alg"] == "classical", (idx, c)
    assert 0 < n_large < n_req
    assert set(stats["requests_per_stream"]) == {"0", "1", "2"}
    assert serving.check_alone(kept) == n_req
    worst = _check_sampled_rows(F, kept, 300)
    say(f"  oracle on sampled rows: worst relF / ratio to gate per dtype {worst}")
    torch.cuda.synchronize()


def test_invalid_request_is_refused_alone():
    """A request whose ldc is below n is refused at submit with its own
    status; the valid requests around it run and complete normally."""
    import ctypes
    import torch
    import paper_1409_2908_amd as F
    say("case serving invalid request")
    dev = torch.device("cuda")
    A = torch.rand((300, 200), dtype=torch.float64, device=dev)
    B = torch.rand((200, 250), dtype=torch.float64, device=dev)
    with F.Server(1 << 28, max_batch=8) as srv:
        ids = [srv.submit(A, B, alg="strassen_222_7", levels=1)[0] for _ in range(3)]
        C = torch.empty((300, 250), dtype=torch.float64, device=dev)
        req = F._Request(300, 200, 250, F.F64, b"strassen_222_7", 1, A.data_ptr(), 200, B.data_ptr(), 250,
                         C.data_ptr(), 100, None, 0, None)
        rid = ctypes.c_int64()
        st = F._lib.fmm_server_submit(srv._s, ctypes.byref(req), ctypes.byref(rid))
        assert st == 1 and b"ldc" in F._lib.fmm_last_error()
        ids += [srv.submit(A, B, alg="strassen_222_7", levels=1)[0] for _ in range(3)]
        got = {}
        while len(got) < len(ids):
            for c in srv.progress(wait=True):
                got[c["id"]] = c
        assert sorted(got) == sorted(ids) and all(c["status"] == 0 for c in got.values())
        assert max(c["batch_size"] for c in got.values()) > 1


@pytest.mark.parametrize("num_streams", [1, 3])
def test_request_waits_for_its_stream(num_streams):
    """Operands written on another stream by work that has not finished when
    the request is submitted: the batch waits for that stream, so the result
    is that of the written operands (with one server stream and with three,
    where the request runs on a small-request stream)."""
    import torch
    import paper_1409_2908_amd as F
    say(f"case serving waits for the request's stream, {num_streams} server streams")
    dev = torch.device("cuda")
    m, k, n = 1024, 1024, 1024
    srcA = torch.rand((m, k), dtype=torch.float64, device=dev)
    srcB = torch.rand((k, n), dtype=torch.float64, device=dev)
    A = torch.zeros((m, k), dtype=torch.float64, device=dev)
    B = torch.zeros((k, n), dtype=torch.float64, device=dev)
    C = torch.empty((m, n), dtype=torch.float64, device=dev)
    X = torch.rand((4096, 4096), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    s1 = torch.cuda.Stream()
    with F.Server(1 << 28, max_batch=4, num_streams=num_streams) as srv:
        with torch.cuda.stream(s1):
            for _ in range(40):  # about 50 ms of work ahead of the writes
                Y = X @ X
            A.copy_(srcA)
            B.copy_(srcB)
            rid, _ = srv.submit(A, B, C, alg="strassen_222_7", levels=1, stream=s1)
        done = []
        while not done:
            done = srv.progress(wait=True)
        assert done[0]["id"] == rid and done[0]["status"] == 0
        assert done[0]["lane"] == (0 if num_streams == 1 else 1)
    torch.cuda.synchronize()
    del Y
    with F.Plan("strassen_222_7", m, k, n, 1) as p:
        ref = p.multiply(srcA, srcB)
    torch.cuda.synchronize()
    assert torch.equal(C, ref)
