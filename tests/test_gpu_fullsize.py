"""GPU parity at the full workload sizes, on sampled rows the oracle computes
one by one.

Shapes: the FP64 rectangular workloads (16384 x 1600 x 16384,
16384 x 16384 x 2400, 9000^3, the last with and without peeling), the FP64
square 16384^3 (also at three levels) and the FP32 BF16x3 workloads (16384^3
at two levels, 8192^3 at three), each with the base case the benchmark runs
there.  Every sampled set holds the first and
last row, every leaf-block boundary row and every row of the m-peel strip;
each sampled row holds all n columns, so the n-peel strip is checked in
every row.

Gates (relative Frobenius error over the sampled rows):
  FP64 uniform inputs: 1e-12, the FP64 gate for depth <= 3.
  Integer inputs in {-8..8}: bit-exact.  FP64: every intermediate is a
      dyadic rational of well under 53 significant bits.  BF16x3 Strassen
      at two levels: operand sums hold at most 4 inputs (|s| <= 32, exact in
      bf16, lo part zero), leaf products are at most 1024 and a leaf sums
      4096 of them (< 2^24, exact in FP32), and the combination is FP64.
  BF16x3 on the row-scaled normal inputs: 2e-5 * 2^L against the binary64
      product (split error 2^-16 per operand, grown by the base case's
      coefficients; a mistake in indexing gives errors of order one).
"""
import numpy as np
import pytest

import fmm_inputs
from oracle import algorithms, classical
from gpu_util import relf, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    import paper_1409_2908_amd as lib
    return lib


def _rows(alg, L, m, count, seed):
    """Sampled rows: ends, every leaf-block boundary, the whole m-peel strip."""
    a = algorithms.get(alg)
    blocks = a.M ** L
    h = m // blocks
    m0 = h * blocks
    must = [0, m - 1] + [b * h for b in range(blocks)] + [b * h - 1 for b in range(1, blocks + 1)]
    must += list(range(m0, m))
    return fmm_inputs.sample_rows(seed, m, count + len(set(must)), must)


def _sampled(F, alg, L, A, B, dtype, rows):
    import torch
    m, k = A.shape
    n = B.shape[1]
    with F.Plan(alg, m, k, n, L, dtype) as p:
        C = p.multiply(to_dev(A), to_dev(B))
        torch.cuda.synchronize()
        return C[torch.from_numpy(rows).cuda()].double().cpu().numpy()


@pytest.mark.parametrize("m,k,n,alg,L", [(16384, 1600, 16384, "fmm_424_26", 2),
                                         (16384, 16384, 2400, "strassen_222_7", 2),
                                         (9000, 9000, 9000, "fmm_323_15", 2),
                                         (9000, 9000, 9000, "fmm_424_26", 2),
                                         (16384, 16384, 16384, "strassen_222_7", 3)])
def test_fp64_full_size(F, m, k, n, alg, L):
    say(f"case fullsize fp64 {alg} L={L} {m}x{k}x{n}")
    A, B = fmm_inputs.operands(21, m, k, n, "uniform")
    rows = _rows(alg, L, m, 16, 21)
    got = _sampled(F, alg, L, A, B, F.F64, rows)
    err = relf(got, classical.gemm_rows(A, B, rows))
    say(f"  sampled {len(rows)} rows relF={err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("dtype_name,alg,L", [("F64", "fmm_424_26", 2), ("F32_BF16X3", "strassen_222_7", 2)])
def test_integer_full_size_bit_exact(F, dtype_name, alg, L):
    n = 16384
    say(f"case fullsize integer {dtype_name} {alg} L={L} n={n}")
    dt = np.float64 if dtype_name == "F64" else np.float32
    A, B = fmm_inputs.operands(22, n, n, n, "integer", dt)
    rows = _rows(alg, L, n, 8, 22)
    got = _sampled(F, alg, L, A, B, getattr(F, dtype_name), rows)
    ref = classical.gemm_rows(A, B, rows)
    say(f"  sampled {len(rows)} rows, max |diff| {np.abs(got - ref).max():.3e}")
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("n,L", [(16384, 2), (8192, 3)])
def test_bf16x3_rowscaled_full_size(F, n, L):
    alg = "strassen_222_7"
    say(f"case fullsize bf16x3 rowscaled {alg} L={L} n={n}")
    A, B = fmm_inputs.operands(23, n, n, n, "normal_rowscaled", np.float32)
    rows = _rows(alg, L, n, 16, 23)
    got = _sampled(F, alg, L, A, B, F.F32_BF16X3, rows)
    err = relf(got, classical.gemm_rows(A, B, rows))
    say(f"  sampled {len(rows)} rows relF={err:.3e}")
    assert err <= 2e-5 * 2 ** L
