"""GPU checks of the launch machinery around the kernels: HIP-graph replay,
batched multiplies (several plans' leaves in one grouped launch), plans bound
to caller memory, and the continuous-batching server.

Every result is compared bit for bit with the same plan run alone and eagerly
(the arithmetic and its order do not depend on how launches are grouped or
recorded), and against the oracle to the path's tolerance:
  FP64   relF <= 1e-12
  FP32   relF <= 2e-6 * 2^L
  BF16x3 relF <= 2e-6 * 2^L against the emulated fast algorithm, and
         relF <= oracle.bf16x3.gate(alg, L, k) against the binary64 product
"""
import numpy as np
import pytest

import fmm_inputs
from oracle import algorithms, bf16x3, classical
from gpu_util import relf, say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    import paper_1409_2908_amd as lib
    return lib


def _np_dtype(F, dtype):
    return np.float64 if dtype == F.F64 else np.float32


def _check_oracle(F, alg, L, A, B, C, dtype):
    ref = classical.gemm(A, B)
    if dtype == F.F64:
        assert relf(C, ref) <= 1e-12
    elif dtype == F.F32:
        assert relf(C, ref) <= 2e-6 * 2 ** L
    else:
        levels = [algorithms.get(x) for x in alg.split("+")] if "+" in alg else None
        algs = levels if levels else (None if alg == "classical" else algorithms.get(alg))
        emu = bf16x3.gemm(A, B) if algs is None else bf16x3.fmm(algs, L, A, B)
        assert relf(C, emu) <= 2e-6 * 2 ** max(L, 1)
        assert relf(C, ref) <= bf16x3.gate(algs, L if algs is not None else 0, A.shape[1])


def _alone(F, alg, L, A, B, dtype):
    with F.Plan(alg, A.shape[0], A.shape[1], B.shape[1], L, dtype) as p:
        return to_host(p.multiply(to_dev(A), to_dev(B)))


GRAPH_CASES = [("strassen_222_7", 2, (515, 262, 389), 0), ("fmm_424_26", 1, (260, 130, 250), 1),
               ("fmm_333_23", 1, (100, 91, 80), 2), ("classical", 0, (300, 200, 100), 0)]


@pytest.mark.parametrize("alg,L,shape,dtype", GRAPH_CASES)
def test_graph_replays_match_eager(F, alg, L, shape, dtype):
    import torch
    m, k, n = shape
    say(f"case graph {alg} L={L} {shape} dtype={dtype}")
    nd = _np_dtype(F, dtype)
    A1, B1 = fmm_inputs.operands(21, m, k, n, "uniform", nd)
    A2, B2 = fmm_inputs.operands(22, m, k, n, "uniform", nd)
    eager = F.Plan(alg, m, k, n, L, dtype)
    graph = F.Plan(alg, m, k, n, L, dtype, use_graph=True)
    ref1 = to_host(eager.multiply(to_dev(A1), to_dev(B1)))
    ref2 = to_host(eager.multiply(to_dev(A2), to_dev(B2)))
    _check_oracle(F, alg, L, A1, B1, ref1, dtype)
    dA, dB = to_dev(A1), to_dev(B1)
    dC = torch.empty((m, n), dtype=dA.dtype, device=dA.device)
    noise = torch.randn(1 << 16, device=dA.device)
    for rep in range(4):
        # same buffers every replay: one capture, then replays of it; the
        # operands change in place between replays, the graph reads them anew
        src = (A1, B1, ref1) if rep % 2 == 0 else (A2, B2, ref2)
        dA.copy_(to_dev(src[0]))
        dB.copy_(to_dev(src[1]))
        dC.fill_(float("nan"))
        graph.multiply(dA, dB, dC)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(dC), src[2]), f"replay {rep}"
        (noise * 2).sum().item()  # the program's own eager work between replays
        torch.cuda.synchronize()
    # new operand buffers: the plan records a new graph for them
    C2 = to_host(graph.multiply(to_dev(A2), to_dev(B2)))
    assert np.array_equal(C2, ref2)
    eager.close()
    graph.close()


BATCH = [("strassen_222_7", 1, (300, 260, 283), 0), ("fmm_424_26", 1, (130, 70, 140), 0),
         ("classical", 0, (64, 64, 64), 0), ("fmm_333_23", 1, (100, 90, 80), 0),
         ("fmm_423_20", 1, (97, 45, 70), 0), ("fmm_323_15", 2, (200, 41, 190), 0),
         ("strassen_222_7", 2, (129, 130, 131), 0), ("strassen_222_7", 1, (2, 2, 2), 0),
         ("fmm_424_26", 2, (70, 20, 70), 0), ("classical", 0, (1, 300, 5), 0),
         ("strassen_222_7", 1, (0, 5, 5), 0), ("strassen_222_7", 1, (6, 0, 6), 0),
         ("fmm_333_23", 1, (100, 90, 80), 1), ("strassen_222_7", 2, (200, 200, 200), 2),
         ("fmm_424_26", 1, (133, 66, 129), 2), ("classical", 0, (77, 55, 33), 1)]


def test_batched_matches_alone_bitwise(F):
    """16 requests, 12 of them FP64: the FP64 leaves need two grouped
    launches of up to 8 plans; FP32 and BF16x3 get their own."""
    import torch
    plans, As, Bs, host = [], [], [], []
    for i, (alg, L, (m, k, n), dt) in enumerate(BATCH):
        A, B = fmm_inputs.operands(30 + i, m, k, n, "uniform", _np_dtype(F, dt))
        plans.append(F.Plan(alg, m, k, n, L, dt))
        As.append(to_dev(A))
        Bs.append(to_dev(B))
        host.append((A, B))
    say("case batched 16 requests")
    Cs = F.multiply_batched(plans, As, Bs)
    torch.cuda.synchronize()
    for (alg, L, shape, dt), (A, B), C in zip(BATCH, host, Cs):
        got = to_host(C)
        alone = _alone(F, alg, L, A, B, dt)
        assert np.array_equal(got, alone), (alg, L, shape, dt)
        if shape[1] == 0:
            assert not got.any()
        elif got.size:
            _check_oracle(F, alg, L, A, B, got, dt)
    with pytest.raises(F.FmmError) as e:
        F.multiply_batched([plans[0], plans[0]], [As[0], As[0]], [Bs[0], Bs[0]])
    assert e.value.code == 1
    for p in plans:
        p.close()


def test_deferred_plan_bound_to_caller_memory(F):
    import torch
    m, k, n = 301, 257, 263
    A, B = fmm_inputs.operands(40, m, k, n, "uniform", np.float64)
    p = F.Plan("fmm_424_26", m, k, n, 1, F.F64, defer_device_memory=True)
    assert p.workspace_ptr is None
    dA, dB = to_dev(A), to_dev(B)
    with pytest.raises(F.FmmError) as e:
        p.multiply(dA, dB)
    assert e.value.code == 1
    nbytes = p.device_bytes
    mem = torch.empty(nbytes + 256, dtype=torch.uint8, device=dA.device)
    base = (mem.data_ptr() + 255) // 256 * 256
    with pytest.raises(F.FmmError):
        p.bind(base + 8, nbytes)  # misaligned
    with pytest.raises(F.FmmError):
        p.bind(base, nbytes - 1)  # too small
    p.bind(base, nbytes)
    C = to_host(p.multiply(dA, dB))
    assert np.array_equal(C, _alone(F, "fmm_424_26", 1, A, B, F.F64))
    # rebinding to another region works the same
    mem2 = torch.empty(nbytes + 256, dtype=torch.uint8, device=dA.device)
    p.bind((mem2.data_ptr() + 255) // 256 * 256, nbytes)
    assert np.array_equal(to_host(p.multiply(dA, dB)), C)
    torch.cuda.synchronize()
    p.close()


def test_server_continuous_batching(F):
    """Mixed shapes and dtypes through a small arena: requests wait for room,
    batches overlap, one request can never fit and fails alone.  Every result
    equals the same plan run alone, bit for bit."""
    import torch
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(30):
        m, k, n = (int(x) for x in np.exp(rng.uniform(np.log(16), np.log(700), 3)))
        dt = [F.F64, F.F32, F.F32_BF16X3][i % 3]
        alg, L = [(None, -1), ("strassen_222_7", 1), ("fmm_424_26", -1), ("classical", 0)][i % 4]
        reqs.append((m, k, n, dt, alg, L))
    reqs.insert(7, (3000, 3000, 3000, F.F64, "strassen_222_7", 1))  # workspace > arena
    arena = 48 << 20
    done = {}
    data = {}
    with F.Server(arena, max_batch=4, max_inflight=2) as srv:
        for i, (m, k, n, dt, alg, L) in enumerate(reqs):
            A, B = fmm_inputs.operands(50 + i, m, k, n, "uniform", _np_dtype(F, dt))
            rid, C = srv.submit(to_dev(A), to_dev(B), dtype=dt, alg=alg, levels=L)
            data[rid] = (A, B, C, dt)
            if i >= 20:  # the last ones arrive while earlier batches run
                for c in srv.progress():
                    done[c["id"]] = c
        say(f"case server {len(reqs)} requests, arena {arena >> 20} MiB")
        while srv.pending:
            for c in srv.progress(wait=True):
                done[c["id"]] = c
    assert len(done) == len(reqs)
    sizes = set()
    for rid, c in done.items():
        A, B, C, dt = data[rid]
        if A.shape == (3000, 3000):
            assert c["status"] == 2  # FMM_ENOMEM: cannot fit the arena even alone
            continue
        assert c["status"] == 0, c
        assert c["submit_ms"] <= c["launch_ms"] <= c["done_ms"]
        sizes.add(c["batch_size"])
        got = to_host(C)
        assert np.array_equal(got, _alone(F, c["alg"], c["levels"], A, B, dt)), c
        _check_oracle(F, c["alg"], c["levels"], A, B, got, dt)
    assert max(sizes) > 1  # requests were batched
    torch.cuda.synchronize()


MIXED_BATCH = [("fmm_424_26+strassen_222_7", 2, (300, 130, 270), 0), ("strassen_222_7+fmm_323_15", 2, (250, 90, 260), 0),
               ("fmm_424_26+strassen_222_7", 2, (300, 130, 270), 2), ("strassen_222_7", 2, (200, 200, 200), 0),
               ("fmm_333_23+strassen_222_7", 2, (190, 140, 200), 1)]


def test_batched_mixed_levels_and_graph(F):
    """Plans with one base case per level in a batch with other plans, and
    replayed from a recorded graph: bitwise those of each plan alone."""
    import torch
    plans, As, Bs, host = [], [], [], []
    for i, (alg, L, (m, k, n), dt) in enumerate(MIXED_BATCH):
        A, B = fmm_inputs.operands(60 + i, m, k, n, "uniform", _np_dtype(F, dt))
        plans.append(F.Plan(alg, m, k, n, L, dt))
        As.append(to_dev(A))
        Bs.append(to_dev(B))
        host.append((A, B))
    say("case batched mixed-level plans")
    Cs = F.multiply_batched(plans, As, Bs)
    torch.cuda.synchronize()
    for (alg, L, shape, dt), (A, B), C in zip(MIXED_BATCH, host, Cs):
        got = to_host(C)
        assert np.array_equal(got, _alone(F, alg, L, A, B, dt)), (alg, shape, dt)
        _check_oracle(F, alg, L, A, B, got, dt)
    for p in plans:
        p.close()
    alg, L, (m, k, n), dt = MIXED_BATCH[0]
    A, B = host[0]
    with F.Plan(alg, m, k, n, L, dt, use_graph=True) as p:
        dA, dB = to_dev(A), to_dev(B)
        outs = [to_host(p.multiply(dA, dB)) for _ in range(3)]
    for o in outs:
        assert np.array_equal(o, _alone(F, alg, L, A, B, dt))


def test_autotune_records_and_auto_plans_it(F, tmp_path):
    """The measured tuner times the model's best candidates on the device,
    records the fastest; an "auto" plan of that shape then is the recorded
    choice (base case, depth, fusion, tile), and it matches the oracle.  The
    JSON cache replays the same choice into a cleared table."""
    import torch
    from paper_1409_2908_amd import autotune
    m, k, n = 3000, 2048, 2500
    say(f"case autotune {m}x{k}x{n}")
    cache = str(tmp_path / "tune.json")
    try:
        autotune.clear()
        t = autotune.tune(m, k, n, F.F64, top=3, reps=2, cache=cache)
        say(f"  tuned {t['alg']} L={t['levels']} fuse={t['fuse_levels']} tile={t['leaf_tile']} "
            f"{t['ms']:.3f} ms; {len(t['candidates'])} timed")
        ok = [c for c in t["candidates"] if c["ms"] is not None]
        assert len(ok) >= 3 and t["ms"] == min(c["ms"] for c in ok)
        A, B = fmm_inputs.operands(61, m, k, n, "uniform")
        with F.Plan("auto", m, k, n, -1, F.F64) as p:
            inf = p.info
            assert (inf["alg"], inf["levels"], inf["leaf_tile"]) == (t["alg"], t["levels"], t["leaf_tile"])
            if t["levels"] > 0:
                assert inf["fuse_levels"] == t["fuse_levels"]
            C = to_host(p.multiply(to_dev(A), to_dev(B)))
        assert relf(C, classical.gemm(A, B)) <= 1e-12
        autotune.clear()
        assert autotune.load_cache(cache) == 1
        with F.Plan("auto", m, k, n, -1, F.F64, host_only=True) as p:
            assert (p.info["alg"], p.info["levels"]) == (t["alg"], t["levels"])
    finally:
        autotune.clear()
    torch.cuda.synchronize()
