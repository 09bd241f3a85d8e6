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
  BF16x3 on the row-scaled normal inputs: oracle.bf16x3.gate against the
      binary64 product: e0 * g^L with e0 = 3 * 2^-16 + (2 + sqrt(k)) 2^-24 the
      per-term error bound of the split product and g the base case's
      root-mean-square error growth per level (a mistake in indexing gives
      errors of order one, a lost product term about 2^-9 g^L).  The largest
      per-row error and the error of the rows that were not scaled are
      reported.
"""
import functools

import numpy as np
import pytest

import fmm_inputs
from oracle import algorithms, bf16x3, classical
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


@functools.lru_cache(maxsize=1)
def _rowscaled(n, seed):
    return fmm_inputs.operands(seed, n, n, n, "normal_rowscaled", np.float32)


@pytest.mark.parametrize("n,alg,L", [(16384, "strassen_222_7", 2), (8192, "strassen_222_7", 3),
                                     (8192, "fmm_333_23", 2), (8192, "fmm_323_15", 2),
                                     (8192, "fmm_423_20", 2), (8192, "fmm_424_26", 2)])
def test_bf16x3_rowscaled_full_size(F, n, alg, L):
    say(f"case fullsize bf16x3 rowscaled {alg} L={L} n={n}")
    A, B = _rowscaled(n, 23)
    rows = _rows(alg, L, n, 16, 23)
    got = _sampled(F, alg, L, A, B, F.F32_BF16X3, rows)
    ref = classical.gemm_rows(A, B, rows)
    err = relf(got, ref)
    gate = bf16x3.gate(algorithms.get(alg), L, n)
    scaled = np.isin(rows, fmm_inputs.scaled_rows(23, n, "A"))
    row_err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    say(f"  sampled {len(rows)} rows relF={err:.3e} gate={gate:.2e} max row {row_err.max():.2e} "
        f"unscaled rows relF={relf(got[~scaled], ref[~scaled]):.2e}")
    assert err <= gate
