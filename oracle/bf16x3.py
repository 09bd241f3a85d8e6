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


def growth(alg):
    """Root-mean-square error growth of one step of `alg` for operands with
    i.i.d. zero-mean entries: g = sqrt(sum_r |u_r|^2 |v_r|^2 |w_r|^2 / (MKN)),
    with u_r, v_r the columns of U, V and w_r the column of W (the C blocks
    product r feeds).  Derivation: a block of S_r has entry variance
    |u_r|^2 var(A) (independent blocks add variances), T_r likewise, and an
    error in product r reaches |w_r|^2 blocks' worth of C; the classical
    product of the same blocks has MKN such terms of unit weight, so g = 1
    for a classical step (classical_222_8) and the ratio compounds over the
    levels.  Strassen (Section 2.1's formulas): sum = 32, g = 2."""
    U = np.asarray(alg.U, dtype=np.float64)
    V = np.asarray(alg.V, dtype=np.float64)
    W = np.asarray(alg.W, dtype=np.float64)
    s = float(np.sum((U ** 2).sum(0) * (V ** 2).sum(0) * (W ** 2).sum(0)))
    return float(np.sqrt(s / (alg.M * alg.K * alg.N)))


def gate(alg, levels, k):
    """Tolerance on the relative Frobenius error of the BF16x3 fast product
    against the exact (binary64) product, for inner dimension k:

        e0 * prod over the levels of growth(level's base case),
        e0 = 3 * 2^-16 + (2 + sqrt(k)) * 2^-24.

    e0 bounds the relative error each product term s*t carries: the two split
    residuals |x - hi - lo| <= 2^-16 |x| (each bf16 rounding has unit
    roundoff 2^-8), the dropped lo*lo term <= 2^-16 |s t|, the rounding of
    the binary64 operand sums to FP32 (2^-24 each), and FP32 accumulation
    over k terms taken as uncorrelated roundings (sqrt(k) 2^-24).  Errors of
    distinct terms are uncorrelated, so they add in quadrature, and the
    algorithm amplifies their root-mean-square by growth() per level.  Using
    the worst-case per-term bound as the root-mean-square makes the gate
    about an order of magnitude above what random inputs give."""
    from . import recursive
    algs = recursive._levels(alg, levels) if levels else []
    e0 = 3.0 * 2.0 ** -16 + (2.0 + np.sqrt(max(k, 1))) * 2.0 ** -24
    g = 1.0
    for a in algs:
        g *= growth(a)
    return e0 * g
