"""GPU check of fmm_multiply_noalloc, the entry point for callers that cannot
allocate device memory: plans made with defer_device_memory run with their
workspace and tables in the library's fixed device array.

Each call is compared bit for bit with fmm_multiply of an ordinary plan of the
same product (the same kernels in the same order), and with the oracle to the
path's tolerance (FP64 relF <= 1e-12; integer inputs exact; BF16x3 against the
emulated fast algorithm at 2e-6 * 2^L).  Two calls in a row share the array,
the second on a smaller product, so stale contents of the first must not leak
into the second.
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


# (alg, levels, (m, k, n), dtype, kind): each pair runs the larger product
# first and the smaller second
SEQUENCES = [
    [("strassen_222_7", 2, (515, 262, 389), 0, "uniform"), ("fmm_424_26", 1, (260, 130, 250), 0, "uniform")],
    [("fmm_424_26", 2, (700, 300, 650), 0, "integer"), ("strassen_222_7", 1, (128, 96, 72), 0, "integer")],
    [("strassen_222_7", 2, (600, 520, 610), 2, "uniform"), ("fmm_333_23", 1, (100, 91, 80), 2, "uniform")],
    [("fmm_323_15", 1, (450, 300, 420), 1, "uniform"), ("classical", 0, (97, 45, 33), 1, "uniform")],
]


def _oracle_ok(F, alg, L, A, B, C, dtype, kind):
    ref = classical.gemm(A, B)
    if kind == "integer":
        return np.array_equal(C.astype(np.float64), ref)
    if dtype == F.F64:
        return relf(C, ref) <= 1e-12
    if dtype == F.F32:
        return relf(C, ref) <= 2e-6 * 2 ** L
    emu = bf16x3.gemm(A, B) if alg == "classical" else bf16x3.fmm(algorithms.get(alg), L, A, B)
    return relf(C, emu) <= 2e-6 * 2 ** max(L, 1)


@pytest.mark.parametrize("seq", range(len(SEQUENCES)))
def test_noalloc_matches_multiply_on_consecutive_calls(F, seq):
    import torch
    for call, (alg, L, (m, k, n), dtype, kind) in enumerate(SEQUENCES[seq]):
        say(f"case noalloc seq={seq} call={call} {alg} L={L} {(m, k, n)} dtype={dtype} {kind}")
        nd = np.float64 if dtype == F.F64 else np.float32
        A, B = fmm_inputs.operands(40 + seq * 2 + call, m, k, n, kind, nd)
        dA, dB = to_dev(A), to_dev(B)
        with F.Plan(alg, m, k, n, L, dtype) as ref_plan:
            ref = to_host(ref_plan.multiply(dA, dB))
        p = F.Plan(alg, m, k, n, L, dtype, defer_device_memory=True)
        assert p.device_bytes <= F.NOALLOC_MAX_BYTES
        dC = torch.full((m, n), float("nan"), dtype=dA.dtype, device=dA.device)
        p.multiply_noalloc(dA, dB, dC)
        got = to_host(dC)
        p.close()
        assert np.array_equal(got, ref), f"max |diff| {np.nanmax(np.abs(got - ref))}"
        assert _oracle_ok(F, alg, L, A, B, got, dtype, kind)


def test_noalloc_leaves_an_owning_plan_untouched(F):
    """A plan with its own workspace runs through the array too, and its own
    memory (here: the leaf operands of the previous fmm_multiply) is not
    written by the no-allocation call."""
    import torch
    from gpu_util import ws_read
    m, k, n = 300, 260, 283
    say("case noalloc owning plan strassen_222_7 L=1")
    A, B = fmm_inputs.operands(50, m, k, n, "uniform")
    A2, B2 = fmm_inputs.operands(51, m, k, n, "uniform")
    with F.Plan("strassen_222_7", m, k, n, 1, F.F64) as p:
        C1 = to_host(p.multiply(to_dev(A), to_dev(B)))
        loc, off, _, _, ld, _ = p.operand(0, 0)
        assert loc == F.LOC_WORKSPACE
        inf = p.info
        before = ws_read(p, off, inf["leaf_m"], inf["leaf_k"], ld, np.float64)
        dC = torch.empty((m, n), dtype=torch.float64, device="cuda")
        p.multiply_noalloc(to_dev(A2), to_dev(B2), dC)
        C2 = to_host(dC)
        after = ws_read(p, off, inf["leaf_m"], inf["leaf_k"], ld, np.float64)
        C3 = to_host(p.multiply(to_dev(A2), to_dev(B2)))
    assert np.array_equal(before, after)
    assert np.array_equal(C2, C3)
    assert relf(C1, classical.gemm(A, B)) <= 1e-12


def test_noalloc_rejects_plans_beyond_the_array(F):
    """A plan whose workspace exceeds the array is refused before anything is
    enqueued; the C argument is never written."""
    import torch
    m = k = n = 4096  # Strassen L=1 FP64: 21 blocks of 2048^2 doubles, ~700 MB
    say("case noalloc too large")
    p = F.Plan("strassen_222_7", m, k, n, 1, F.F64, defer_device_memory=True)
    assert p.device_bytes > F.NOALLOC_MAX_BYTES
    dA = torch.zeros((m, k), dtype=torch.float64, device="cuda")
    dB = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    dC = torch.full((m, n), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FmmError) as ei:
        p.multiply_noalloc(dA, dB, dC)
    assert ei.value.code == 2 and "fmm_multiply_noalloc has" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((dC == 7.0).all())
    p.close()
