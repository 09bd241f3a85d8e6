"""Leaf operands formed inside the leaf GEMM (plans with leaf_form = 2): the
GEMM loads the blocks of A (B) named by each column of U (V) and sums them
while it stages the tile, in the formation pass's order and precision.  The
products must therefore equal those of the same plan with separate formation
passes (leaf_form = 1) bit for bit, for every eligible base case, both
element types and ragged sizes (peel strips in every dimension), alone, in a
batch mixed with other plans, replayed from a HIP graph and through the
allocation-free entry point; and match the binary64 oracle (relF <= 1e-12
FP64, 2e-6 * 2 FP32; integer inputs bit for bit).
"""
import numpy as np
import pytest

import fmm_inputs
from oracle import classical
from gpu_util import relf, say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    import paper_1409_2908_amd as lib
    return lib


def _eligible(F):
    """Compiled base cases whose U and V columns have at most 2 non-zeros,
    each +-1 (the rule leaf_form = 2 accepts)."""
    out = []
    for name in F.algorithm_names():
        M, K, N, R, U, V, W = F.algorithm_coeffs(name)
        ok = all(set(np.unique(X)) <= {-1, 0, 1} and (X != 0).sum(axis=0).max() <= 2 for X in (U, V))
        if ok:
            out.append(name)
    return out


def _run(F, alg, A, B, dtype, leaf_form):
    m, k = A.shape
    n = B.shape[1]
    with F.Plan(alg, m, k, n, 1, dtype, leaf_form=leaf_form) as p:
        assert p.info["leaf_form"] == (2 if leaf_form == 2 else 0)
        return to_host(p.multiply(to_dev(A), to_dev(B)))


def test_eligible_cases_cover_the_tables(F):
    names = _eligible(F)
    say(f"leaf-form eligible base cases: {len(names)} of {len(F.algorithm_names())}")
    assert {"strassen_222_7", "fmm_223_11", "fmm_232_11", "fmm_322_11", "fmm_225_18"} <= set(names)


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_leaf_form_bitwise_equal_to_passes(F, dtype_name):
    dtype = F.F64 if dtype_name == "f64" else F.F32
    np_dt = np.float64 if dtype_name == "f64" else np.float32
    for i, alg in enumerate(_eligible(F)):
        M, K, N, R, _, _, _ = F.algorithm_coeffs(alg)
        # leaf blocks over several 64 x 64 tiles with ragged edges, plus peels
        m, k, n = M * 70 + M - 1, K * 45 + 1, N * 66 + N - 1
        say(f"case leaf form {alg} {dtype_name} m={m} k={k} n={n}")
        A, B = fmm_inputs.operands(60 + i, m, k, n, "uniform", np_dt)
        got = _run(F, alg, A, B, dtype, 2)
        ref = _run(F, alg, A, B, dtype, 1)
        assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), alg
        err = relf(got, classical.gemm(A.astype(np.float64), B.astype(np.float64)))
        assert err <= (1e-12 if dtype == F.F64 else 4e-6), (alg, err)


@pytest.mark.parametrize("alg", ["strassen_222_7", "fmm_225_18", "fmm_232_11"])
def test_leaf_form_integer_inputs_exact(F, alg):
    M, K, N, R, _, _, _ = F.algorithm_coeffs(alg)
    m, k, n = M * 33 + 1, K * 40 + 1, N * 29 + 1
    say(f"case leaf form integer {alg} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(7, m, k, n, "integer")
    ref = classical.gemm(A, B)
    assert np.array_equal(_run(F, alg, A, B, F.F64, 2), ref)
    C32 = _run(F, alg, A.astype(np.float32), B.astype(np.float32), F.F32, 2)
    assert np.array_equal(C32.astype(np.float64), ref)


def test_leaf_form_in_a_mixed_batch_graph_and_noalloc(F):
    """A batch holding leaf-forming and pass-forming plans of both element
    types gives each product bit for bit as its plan alone; so do a HIP graph
    replay and the allocation-free entry point."""
    import torch
    shapes = [("strassen_222_7", 512, 512, 512, F.F64), ("fmm_323_15", 300, 250, 333, F.F64),
              ("strassen_222_7", 4096, 2048, 4096, F.F64), ("fmm_232_11", 200, 301, 402, F.F32),
              ("strassen_222_7", 512, 384, 640, F.F32)]
    plans, ops, alone = [], [], []
    for i, (alg, m, k, n, dt) in enumerate(shapes):
        np_dt = np.float64 if dt == F.F64 else np.float32
        A, B = fmm_inputs.operands(80 + i, m, k, n, "uniform", np_dt)
        dA, dB = to_dev(A), to_dev(B)
        p = F.Plan(alg, m, k, n, 1, dt, leaf_form=2 if i in (0, 4) else 1)
        plans.append(p)
        ops.append((dA, dB))
        alone.append(to_host(p.multiply(dA, dB)))
    say("case leaf form mixed batch: leaf_form " + str([p.info["leaf_form"] for p in plans]))
    assert any(p.info["leaf_form"] for p in plans) and not all(p.info["leaf_form"] for p in plans)
    Cs = F.multiply_batched(plans, [a for a, _ in ops], [b for _, b in ops])
    for C, ref in zip(Cs, alone):
        assert np.array_equal(to_host(C).view(np.uint8), ref.view(np.uint8))
    for p, (dA, dB), ref in zip(plans, ops, alone):
        if not p.info["leaf_form"]:
            continue
        C = torch.empty((p.m, p.n), dtype=dA.dtype, device="cuda")
        p.multiply_noalloc(dA, dB, C)
        assert np.array_equal(to_host(C).view(np.uint8), ref.view(np.uint8))
    for p in plans:
        p.close()
    alg, m, k, n, dt = shapes[0]
    dA, dB = ops[0]
    with F.Plan(alg, m, k, n, 1, dt, use_graph=True, leaf_form=2) as p:
        assert p.info["leaf_form"] == 2
        for _ in range(3):
            C = p.multiply(dA, dB)
            torch.cuda.synchronize()
            assert np.array_equal(to_host(C).view(np.uint8), alone[0].view(np.uint8))
