"""O2: the recursive bilinear fast algorithm on the CPU.

Test infrastructure (see oracle/__init__.py).  Written from the steps of
Section 3.1 (form S_r and T_r from the columns of U and V, multiply
recursively, combine the products with the rows of W) and the peeling of
Section 3.5.  Works on float64 numpy arrays (binary64 arithmetic) and on
object arrays of ints / Fractions (exact arithmetic).

Readings where the paper is silent:
* Summation order in every addition chain is ascending block index; the
  first non-zero term initialises the sum (a copy, a negation or a scaling).
* Dynamic peeling (the paper's choice, Section 3.5): at each level the core
  m0 = M*floor(m/M), k0 = K*floor(k/K), n0 = N*floor(n/N) is split into
  blocks and the remainders are fixed up classically:
  C[:m0,:n0] += A[:m0,k0:] B[k0:,:n0];  C[:m0,n0:] = A[:m0,:] B[:,n0:];
  C[m0:,:] = A[m0:,:] B.
* Static peeling (the GPU library's choice) peels once, at the top, to
  multiples of M^L, K^L, N^L and recurses on the core without further peels.
  Both are exact in exact arithmetic.
"""
import numpy as np

from . import classical


class FlopCounter:
    """Counts flops the way Section 2.1 does: a classical m x k x n leaf costs
    m*n*(2k-1) (so F_C(1) = 1), each extra term of an addition chain costs one
    flop per element, and a scaling by a coefficient other than +-1 costs one
    flop per element."""

    def __init__(self):
        self.flops = 0


def _leaf(A, B, counter):
    m, k = A.shape
    n = B.shape[1]
    if counter is not None and m and n and k:
        counter.flops += m * n * (2 * k - 1)
    if A.dtype == object or B.dtype == object:
        out = np.empty((m, n), dtype=object)
        res = classical.gemm_exact(A.tolist(), B.tolist())
        for i in range(m):
            for j in range(n):
                out[i, j] = res[i][j]
        return out
    return classical.gemm(A, B)


def chain(coeffs, blocks, counter=None):
    """sum_i coeffs[i] * blocks[i] in ascending i, first non-zero term
    initialising (Section 3.1's addition chains)."""
    acc = None
    for c, X in zip(coeffs, blocks):
        if c == 0:
            continue
        if acc is None:
            if c == 1:
                acc = X.copy()
            elif c == -1:
                acc = -X
            else:
                acc = c * X
                if counter is not None:
                    counter.flops += X.size
        else:
            if c == 1:
                acc = acc + X
                if counter is not None:
                    counter.flops += X.size
            elif c == -1:
                acc = acc - X
                if counter is not None:
                    counter.flops += X.size
            else:
                acc = acc + c * X
                if counter is not None:
                    counter.flops += 2 * X.size
    if acc is None:
        acc = np.zeros_like(blocks[0])
    return acc


def _levels(alg, levels):
    """The base case of every level, top first: `alg` is one algorithm (used at
    every level) or a sequence with one per level (Section 5.2 composes
    different base cases across levels)."""
    if isinstance(alg, (list, tuple)):
        assert len(alg) == levels, (len(alg), levels)
        return list(alg)
    return [alg] * levels


def _split(X, rows, cols):
    """Blocks of X (already trimmed to multiples) in row-wise order."""
    h = X.shape[0] // rows
    w = X.shape[1] // cols
    return [X[a * h:(a + 1) * h, b * w:(b + 1) * w] for a in range(rows) for b in range(cols)]


def _one_level(alg, A, B, recurse, counter):
    """One recursive step on divisible dimensions: S_r, T_r, M_r = S_r T_r,
    C_k = sum_r W[k][r] M_r."""
    M, K, N, R = alg.M, alg.K, alg.N, alg.R
    Ab = _split(A, M, K)
    Bb = _split(B, K, N)
    Ms = []
    for r in range(R):
        S = chain([alg.U[i][r] for i in range(M * K)], Ab, counter)
        T = chain([alg.V[j][r] for j in range(K * N)], Bb, counter)
        Ms.append(recurse(S, T))
    m, n = A.shape[0], B.shape[1]
    h, w = m // M, n // N
    C = np.empty((m, n), dtype=np.result_type(A.dtype, B.dtype))
    for a in range(M):
        for c in range(N):
            C[a * h:(a + 1) * h, c * w:(c + 1) * w] = chain(list(alg.W[a * N + c]), Ms, counter)
    return C


def _fixups(A, B, C, m0, k0, n0, counter):
    m, k = A.shape
    n = B.shape[1]
    if k0 < k and m0 and n0:
        P = _leaf(A[:m0, k0:], B[k0:, :n0], counter)
        C[:m0, :n0] = C[:m0, :n0] + P
        if counter is not None:
            counter.flops += P.size
    if n0 < n and m0:
        C[:m0, n0:] = _leaf(A[:m0, :], B[:, n0:], counter)
    if m0 < m:
        C[m0:, :] = _leaf(A[m0:, :], B, counter)
    return C


def fmm(alg, levels, A, B, peel="dynamic", counter=None):
    """C = A @ B by `levels` recursive steps of `alg` (one base case, or one
    per level, top first), classical leaves."""
    A = np.asarray(A)
    B = np.asarray(B)
    m, k = A.shape
    assert B.shape[0] == k
    n = B.shape[1]
    algs = _levels(alg, levels)
    dt = np.result_type(A.dtype, B.dtype)
    if peel == "dynamic":
        if levels == 0 or m < algs[0].M or k < algs[0].K or n < algs[0].N:
            return _leaf(A, B, counter)
        M, K, N = algs[0].M, algs[0].K, algs[0].N
        m0, k0, n0 = M * (m // M), K * (k // K), N * (n // N)
        C = np.zeros((m, n), dtype=dt) if dt != object else np.full((m, n), 0, dtype=object)
        C[:m0, :n0] = _one_level(algs[0], A[:m0, :k0], B[:k0, :n0],
                                 lambda S, T: fmm(algs[1:], levels - 1, S, T, "dynamic", counter),
                                 counter)
        return _fixups(A, B, C, m0, k0, n0, counter)
    if peel == "static":
        fm = int(np.prod([a.M for a in algs])) if algs else 1
        fk = int(np.prod([a.K for a in algs])) if algs else 1
        fn = int(np.prod([a.N for a in algs])) if algs else 1
        m0, k0, n0 = fm * (m // fm), fk * (k // fk), fn * (n // fn)
        C = np.zeros((m, n), dtype=dt) if dt != object else np.full((m, n), 0, dtype=object)
        if m0 and k0 and n0:
            C[:m0, :n0] = _core(algs, levels, A[:m0, :k0], B[:k0, :n0], counter)
        elif m0 and n0:
            C[:m0, :n0] = 0
        return _fixups(A, B, C, m0, k0, n0, counter)
    raise ValueError(peel)


def _core(algs, levels, A, B, counter):
    if levels == 0:
        return _leaf(A, B, counter)
    return _one_level(algs[0], A, B, lambda S, T: _core(algs[1:], levels - 1, S, T, counter), counter)


def form_operands(alg, levels, X, which):
    """The leaf operands of a static-peeled plan on the divisible core X,
    in leaf order rho = (rho_1, ..., rho_L) (rho_1 most significant): the
    S_rho (which='A', coefficients from U) or T_rho (which='B', from V),
    each formed level by level with `chain`.  Used to check operand-formation
    kernels bit for bit.  `alg` is one base case or one per level."""
    cur = [X]
    for a in _levels(alg, levels):
        rows, cols = (a.M, a.K) if which == "A" else (a.K, a.N)
        coef = a.U if which == "A" else a.V
        nxt = []
        for Y in cur:
            blocks = _split(Y, rows, cols)
            for r in range(a.R):
                nxt.append(chain([coef[i][r] for i in range(rows * cols)], blocks))
        cur = nxt
    return cur


def combine_products(alg, levels, Ms):
    """C from the R^L leaf products (leaf order as in form_operands), deepest
    level first, each level with `chain` over the rows of W: the order the
    recursion of Section 3.1 produces.  `alg` is one base case or one per
    level (top first)."""
    cur = list(Ms)
    for al in reversed(_levels(alg, levels)):
        nxt = []
        for g in range(len(cur) // al.R):
            group = cur[g * al.R:(g + 1) * al.R]
            h, w = group[0].shape
            C = np.empty((al.M * h, al.N * w), dtype=group[0].dtype)
            for a in range(al.M):
                for c in range(al.N):
                    C[a * h:(a + 1) * h, c * w:(c + 1) * w] = chain(list(al.W[a * al.N + c]), group)
            nxt.append(C)
        cur = nxt
    return cur[0]
