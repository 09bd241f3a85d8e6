"""Emulated BF16x3 leaf product (test infrastructure; see oracle/__init__.py).

The split-precision leaf represents each FP32 operand x by two bfloat16
values, hi = bf16(x) and lo = bf16(x - hi), both rounded to nearest-even, and
forms A_hi B_hi + A_hi B_lo + A_lo B_hi.  Here the three products are summed in
binary64 (every bf16 x bf16 product is exact in binary64), so the result is the
exact value of the three-term product up to one final rounding per sum term:
a reference for the split itself.  The GPU accumulates in FP32 in an order the
matrix cores do not specify, so comparisons against this emulation use a
tolerance, never bit equality.  Parity unpinned beyond the pins in
tests/test_oracle_pins.py (rounding ties, exact reconstruction, integers).
"""
import numpy as np


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32.  Rounding on the 32-bit pattern: add 0x7FFF plus the lowest
    kept bit, then clear the 16 dropped bits.  Finite inputs only."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    keep_lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + keep_lsb) >> np.uint64(16)) << np.uint64(16)
    return (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)


def split(x):
    """(hi, lo) with hi = bf16(x), lo = bf16(x - hi); x - hi is exact in FP32."""
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_round(x)
    lo = bf16_round((x - hi).astype(np.float32))
    return hi, lo


def gemm(A, B):
    """A_hi B_hi + A_hi B_lo + A_lo B_hi with binary64 products and sums."""
    ah, al = split(A)
    bh, bl = split(B)
    ah, al, bh, bl = (v.astype(np.float64) for v in (ah, al, bh, bl))
    return ah @ bh + ah @ bl + al @ bh


def fmm(alg, levels, A, B):
    """C = A @ B by `levels` steps of `alg` (one base case, or one per level)
    with static peeling (peel once to multiples of the levels' block counts,
    M^L, K^L, N^L for one base case; Section 3.5's fix-ups for the strips) and every
    leaf product -- core leaves and peel strips alike -- taken as the emulated
    BF16x3 product of FP32 operands.  Leaf operands are formed in binary64
    (Section 3.1's addition chains) and rounded once to FP32; products are
    combined in binary64.  A kernel that forms the sums in FP32 differs from
    this only by FP32 rounding of the sums and of its accumulation, which is
    the tolerance a comparison should allow."""
    from . import recursive
    A = np.asarray(A, dtype=np.float32)
    B = np.asarray(B, dtype=np.float32)
    m, k = A.shape
    n = B.shape[1]
    algs = recursive._levels(alg, levels)  # one base case, or one per level
    fm = int(np.prod([a.M for a in algs])) if algs else 1
    fk = int(np.prod([a.K for a in algs])) if algs else 1
    fn = int(np.prod([a.N for a in algs])) if algs else 1
    m0, k0, n0 = fm * (m // fm), fk * (k // fk), fn * (n // fn)
    C = np.zeros((m, n), dtype=np.float64)
    if m0 and k0 and n0:
        S = recursive.form_operands(alg, levels, A[:m0, :k0].astype(np.float64), "A")
        T = recursive.form_operands(alg, levels, B[:k0, :n0].astype(np.float64), "B")
        Ms = [gemm(s.astype(np.float32), t.astype(np.float32)) for s, t in zip(S, T)]
        C[:m0, :n0] = recursive.combine_products(alg, levels, Ms)
    if k0 < k and m0 and n0:
        C[:m0, :n0] += gemm(A[:m0, k0:], B[k0:, :n0])
    if n0 < n and m0:
        C[:m0, n0:] = gemm(A[:m0, :], B[:, n0:])
    if m0 < m:
        C[m0:, :] = gemm(A[m0:, :], B)
    return C
