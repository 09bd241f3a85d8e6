"""GPU parity of the base cases derived from the base tables: their
permutations by Propositions 2.1 and 2.2 (Section 2.3) and the direct sums
<2,2,3;11>, <2,2,5;18> with their permutations (Table 2's ranks in every
order of the dimensions).

For each: FP64 products on ragged sizes (M^L t + r, peel strips in every
direction, leaf blocks spanning several tiles) at one and two levels against
the binary64 oracle (relF <= 1e-12); integer inputs bit-exact on the FP64,
FP32 and BF16x3 paths; every leaf operand of the formation stage and the
combination stage bit for bit against the oracle's chains; BF16x3 within
oracle.bf16x3.gate against the binary64 product.
"""
import numpy as np
import pytest

import fmm_inputs
from oracle import algorithms, bf16x3, classical, recursive
from gpu_util import relf, say, to_dev, to_host, ws_read, ws_write

pytestmark = pytest.mark.gpu

BASE = {"classical_222_8", "strassen_222_7", "fmm_333_23", "fmm_323_15", "fmm_423_20", "fmm_424_26"}
NEW = [n for n in algorithms.names() if n not in BASE]


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    import paper_1409_2908_amd as lib
    return lib


def _run(F, alg, L, A, B, dtype):
    m, k = A.shape
    n = B.shape[1]
    with F.Plan(alg, m, k, n, L, dtype) as p:
        return to_host(p.multiply(to_dev(A), to_dev(B)))


@pytest.mark.parametrize("alg", NEW)
@pytest.mark.parametrize("L", [1, 2])
def test_fp64_parity_ragged(F, alg, L):
    a = algorithms.get(alg)
    lm, lk, ln = (130, 70, 140) if L == 1 else (36, 20, 34)
    fm, fk, fn = a.M ** L, a.K ** L, a.N ** L
    m, k, n = fm * lm + fm - 1, fk * lk + 1, fn * ln + fn - 1
    say(f"case fp64 {alg} L={L} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(31, m, k, n, "uniform")
    err = relf(_run(F, alg, L, A, B, F.F64), classical.gemm(A, B))
    say(f"  relF={err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("alg", NEW)
def test_integer_bit_exact_every_path(F, alg):
    a = algorithms.get(alg)
    m, k, n = a.M * 9 + 1, a.K * 7 + 2, a.N * 8 + 1
    say(f"case int {alg} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(32, m, k, n, "integer")
    ref = classical.gemm(A, B)
    assert np.array_equal(_run(F, alg, 1, A, B, F.F64), ref)
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    assert np.array_equal(_run(F, alg, 1, A32, B32, F.F32).astype(np.float64), ref)
    assert np.array_equal(_run(F, alg, 1, A32, B32, F.F32_BF16X3).astype(np.float64), ref)


@pytest.mark.parametrize("alg", NEW)
def test_bf16x3_gate(F, alg):
    a = algorithms.get(alg)
    m, k, n = a.M * 60 + 3, a.K * 40 + 1, a.N * 50 + 2
    say(f"case bf16x3 {alg} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(33, m, k, n, "normal_rowscaled", np.float32)
    C = _run(F, alg, 1, A, B, F.F32_BF16X3)
    err, gate = relf(C, classical.gemm(A, B)), bf16x3.gate(a, 1, k)
    e_emu = relf(C, bf16x3.fmm(a, 1, A, B))
    say(f"  relF={err:.2e} gate={gate:.2e} vs emulation {e_emu:.2e}")
    assert err <= gate and e_emu <= 4e-6


@pytest.mark.parametrize("alg", NEW)
@pytest.mark.parametrize("L", [1, 2])
def test_stages_bit_exact(F, alg, L):
    """Leaf operands (views times alpha, materialised ones read back) and the
    W-combination of seeded leaf products equal the oracle's chains bit for
    bit; at two levels the library fuses both levels in one pass where the
    base case allows it."""
    a = algorithms.get(alg)
    m, k, n = a.M ** L * 5, a.K ** L * 4, a.N ** L * 6
    say(f"case stages {alg} L={L} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(34, m, k, n, "uniform")
    S = recursive.form_operands(a, L, A, "A")
    T = recursive.form_operands(a, L, B, "B")
    with F.Plan(alg, m, k, n, L, F.F64) as p:
        info = p.info
        dA, dB = to_dev(A), to_dev(B)
        C = p.run_stage(F.STAGE_FORM_S, dA, dB)
        p.run_stage(F.STAGE_FORM_T, dA, dB, C)
        lm, lk, ln = info["leaf_m"], info["leaf_k"], info["leaf_n"]
        for side, X, ref, (h, w) in ((0, A, S, (lm, lk)), (1, B, T, (lk, ln))):
            for leaf in range(a.R ** L):
                loc, off, row, col, ld, alpha = p.operand(side, leaf)
                got = ws_read(p, off, h, w, ld, np.float64) * alpha if loc == F.LOC_WORKSPACE else \
                    X[row:row + h, col:col + w] * alpha
                assert np.array_equal(got.view(np.int64), ref[leaf].view(np.int64)), (side, leaf)
        Ms = []
        for leaf in range(a.R ** L):
            Mv = fmm_inputs.matrix(200 + leaf, 7, lm, ln, "uniform")
            Ms.append(Mv)
            loc, off, row, col, ld, alpha = p.operand(2, leaf)
            ws_write(p, off, Mv, ld)
        got = to_host(p.run_stage(F.STAGE_COMBINE, dA, dB))
    ref = recursive.combine_products(a, L, Ms)
    assert np.array_equal(got.view(np.int64), ref.view(np.int64))
