"""The oracle's own base-case decompositions [[U,V,W]].

Test infrastructure (see oracle/__init__.py).  These are the oracle's copies;
the product library carries its own.  Each table is accepted only if it
passes the exact Brent check (oracle.tensor.brent_residual).

Conventions (Section 2.2, Table 1): A is M x K with block index i = a*K + b,
B is K x N with j = b*N + c, C is M x N with k = a*N + c (row-wise
vectorisation, 0-indexed here).  U is MK x R, V is KN x R, W is MN x R, so
S_r = sum_i U[i][r] A_i, T_r = sum_j V[j][r] B_j, C_k = sum_r W[k][r] M_r.
"""
import os
import re
from dataclasses import dataclass
from typing import List

from . import tensor

_HERE = os.path.dirname(os.path.abspath(__file__))


@dataclass(frozen=True)
class Algorithm:
    name: str
    M: int
    K: int
    N: int
    R: int
    U: tuple  # MK rows of R ints
    V: tuple  # KN rows
    W: tuple  # MN rows

    @property
    def dims(self):
        return (self.M, self.K, self.N)


def _terms(expr, letter, rows, cols):
    """Parse a sum like 'A11 - A21 + A22' into a coefficient vector over the
    row-wise block index (rows x cols blocks, 1-indexed names)."""
    v = [0] * (rows * cols)
    for sign, a, b in re.findall(r"([+-]?)\s*" + letter + r"(\d)(\d)", expr):
        v[(int(a) - 1) * cols + int(b) - 1] += -1 if sign == "-" else 1
    return v


def _from_formulas(name, M, K, N, S, T, C):
    """Build [[U,V,W]] from S_r / T_r formulas over A_ab / B_bc blocks and
    C_ac = sum of +-M_r formulas (the form in which Section 2.1 writes them)."""
    R = len(S)
    Ucols = [_terms(s, "A", M, K) for s in S]
    Vcols = [_terms(t, "B", K, N) for t in T]
    U = tuple(tuple(Ucols[r][i] for r in range(R)) for i in range(M * K))
    V = tuple(tuple(Vcols[r][j] for r in range(R)) for j in range(K * N))
    W = []
    for a in range(M):
        for c in range(N):
            row = [0] * R
            expr = C[f"C{a + 1}{c + 1}"]
            for sign, r in re.findall(r"([+-]?)\s*M(\d+)", expr):
                row[int(r) - 1] += -1 if sign == "-" else 1
            W.append(tuple(row))
    return Algorithm(name, M, K, N, R, U, V, tuple(W))


def classical_222():
    """The classical <2,2,2;8> block recursion of Section 2.1 (eight products
    M1..M8 and four block sums)."""
    S = ["A11", "A12", "A11", "A12", "A21", "A22", "A21", "A22"]
    T = ["B11", "B21", "B12", "B22", "B11", "B21", "B12", "B22"]
    C = {"C11": "M1 + M2", "C12": "M3 + M4", "C21": "M5 + M6", "C22": "M7 + M8"}
    return _from_formulas("classical_222_8", 2, 2, 2, S, T, C)


def strassen():
    """Strassen's <2,2,2;7> from the S_r, T_r and C_ij formulas of Section 2.1.

    Reading: the W matrix printed with the U and V matrices in Section 2.2
    does not agree with these formulas (its C12/C21 rows are swapped and its
    C22 row has M4 where M6 belongs) and fails the Brent equations; the
    formulas pass, so they are the definition used here."""
    S = ["A11 + A22", "A21 + A22", "A11", "A22", "A11 + A12", "A21 - A11", "A12 - A22"]
    T = ["B11 + B22", "B11", "B12 - B22", "B21 - B11", "B22", "B11 + B12", "B21 + B22"]
    C = {"C11": "M1 + M4 - M5 + M7", "C12": "M3 + M5",
         "C21": "M2 + M4", "C22": "M1 - M2 + M3 + M6"}
    return _from_formulas("strassen_222_7", 2, 2, 2, S, T, C)


def winograd_222():
    """The Strassen-Winograd variant of <2,2,2;7> (S. Winograd's 1971 form,
    the one Section 3.3's common-subexpression discussion concerns): its
    seven products written out as full sums of blocks.  Scheduled with shared
    intermediates (S1 = A21 + A22, S2 = S1 - A11, S4 = A12 - S2; T1 = B12 - B11,
    T2 = B22 - T1, T4 = T2 - B21; U2 = M1 + M6, U3 = U2 + M7, U4 = U2 + M5) it
    needs 15 block additions against Strassen's 18; as a bilinear table its
    columns are denser (24 additions without sharing)."""
    S = ["A11", "A12", "A11 + A12 - A21 - A22", "A22", "A21 + A22", "A21 + A22 - A11", "A11 - A21"]
    T = ["B11", "B21", "B22", "B11 - B12 - B21 + B22", "B12 - B11", "B11 - B12 + B22", "B22 - B12"]
    C = {"C11": "M1 + M2", "C12": "M1 + M3 + M5 + M6",
         "C21": "M1 - M4 + M6 + M7", "C22": "M1 + M5 + M6 + M7"}
    return _from_formulas("winograd_222_7", 2, 2, 2, S, T, C)


def laderman_333():
    """A rank-23 <3,3,3> decomposition (Table 2 lists rank 23 for <3,3,3>; the
    paper does not print coefficients).  This is Laderman's 1976 scheme
    (J. D. Laderman, Bull. AMS 82(1):126-128), restated as products of A-sums
    and B-sums and accepted by the exact Brent check."""
    P = [
        ("A11+A12+A13-A21-A22-A32-A33", "B22"),
        ("A11-A21", "-B12+B22"),
        ("A22", "-B11+B12+B21-B22-B23-B31+B33"),
        ("-A11+A21+A22", "B11-B12+B22"),
        ("A21+A22", "-B11+B12"),
        ("A11", "B11"),
        ("-A11+A31+A32", "B11-B13+B23"),
        ("-A11+A31", "B13-B23"),
        ("A31+A32", "-B11+B13"),
        ("A11+A12+A13-A22-A23-A31-A32", "B23"),
        ("A32", "-B11+B13+B21-B22-B23-B31+B32"),
        ("-A13+A32+A33", "B22+B31-B32"),
        ("A13-A33", "B22-B32"),
        ("A13", "B31"),
        ("A32+A33", "-B31+B32"),
        ("-A13+A22+A23", "B23+B31-B33"),
        ("A13-A23", "B23-B33"),
        ("A22+A23", "-B31+B33"),
        ("A12", "B21"),
        ("A23", "B32"),
        ("A21", "B13"),
        ("A31", "B12"),
        ("A33", "B33"),
    ]
    C = {
        "C11": "M6 + M14 + M19",
        "C12": "M1 + M4 + M5 + M6 + M12 + M14 + M15",
        "C13": "M6 + M7 + M9 + M10 + M14 + M16 + M18",
        "C21": "M2 + M3 + M4 + M6 + M14 + M16 + M17",
        "C22": "M2 + M4 + M5 + M6 + M20",
        "C23": "M14 + M16 + M17 + M18 + M21",
        "C31": "M6 + M7 + M8 + M11 + M12 + M13 + M14",
        "C32": "M12 + M13 + M14 + M15 + M22",
        "C33": "M6 + M7 + M8 + M9 + M23",
    }
    return _from_formulas("fmm_333_23", 3, 3, 3, [p[0] for p in P], [p[1] for p in P], C)


def load_table(path, name=None):
    """Read a text table: a header line 'M K N R', then the MK rows of U, the
    KN rows of V and the MN rows of W (R integers each); '#' lines are
    comments."""
    rows = []
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([int(t) for t in line.split()])
    M, K, N, R = rows[0]
    body = rows[1:]
    assert len(body) == M * K + K * N + M * N, path
    U = tuple(tuple(r) for r in body[:M * K])
    V = tuple(tuple(r) for r in body[M * K:M * K + K * N])
    W = tuple(tuple(r) for r in body[M * K + K * N:])
    assert all(len(r) == R for r in U + V + W), path
    nm = name or os.path.splitext(os.path.basename(path))[0]
    return Algorithm(nm, M, K, N, R, U, V, W)


def classical(M, K, N):
    """The classical <M,K,N;MKN> scheme written as a bilinear algorithm:
    product (a, b, c) multiplies A_ab by B_bc and goes to C_ac."""
    R = M * K * N
    U = [[0] * R for _ in range(M * K)]
    V = [[0] * R for _ in range(K * N)]
    W = [[0] * R for _ in range(M * N)]
    r = 0
    for a in range(M):
        for b in range(K):
            for c in range(N):
                U[a * K + b][r] = 1
                V[b * N + c][r] = 1
                W[a * N + c][r] = 1
                r += 1
    return Algorithm(f"classical_{M}{K}{N}_{R}", M, K, N, R, tuple(map(tuple, U)),
                     tuple(map(tuple, V)), tuple(map(tuple, W)))


def permuted(alg, dims, name=None):
    """An algorithm for `dims` obtained from `alg` by Propositions 2.1 and 2.2
    (Section 2.3): the first sequence of them, by length and with 2.1 before
    2.2 at each position, whose result has the wanted dimensions."""
    from itertools import product
    for length in range(4):
        for seq in product((1, 2), repeat=length):
            U, V, W, d = alg.U, alg.V, alg.W, alg.dims
            for prop in seq:
                fn = tensor.prop21 if prop == 1 else tensor.prop22
                U, V, W, d = fn(U, V, W, *d)
            if tuple(d) == tuple(dims):
                return Algorithm(name or alg.name, d[0], d[1], d[2], alg.R, tuple(map(tuple, U)),
                                 tuple(map(tuple, V)), tuple(map(tuple, W)))
    raise ValueError(dims)


def direct_sum_n(algs, name):
    """The direct sum along N of algorithms for <M,K,N_1>, <M,K,N_2>, ...:
    B and C are split into column blocks of N_1, N_2, ... block columns and
    each part is multiplied by its own algorithm; the products of the first
    algorithm come first."""
    M, K = algs[0].M, algs[0].K
    N = sum(a.N for a in algs)
    R = sum(a.R for a in algs)
    U = [[] for _ in range(M * K)]
    V = [[0] * R for _ in range(K * N)]
    W = [[0] * R for _ in range(M * N)]
    r0 = c0 = 0
    for a in algs:
        assert (a.M, a.K) == (M, K)
        for i in range(M * K):
            U[i] += list(a.U[i])
        for r in range(a.R):
            for b in range(K):
                for c in range(a.N):
                    V[b * N + c0 + c][r0 + r] = a.V[b * a.N + c][r]
            for x in range(M):
                for c in range(a.N):
                    W[x * N + c0 + c][r0 + r] = a.W[x * a.N + c][r]
        r0 += a.R
        c0 += a.N
    return Algorithm(name, M, K, N, R, tuple(map(tuple, U)), tuple(map(tuple, V)), tuple(map(tuple, W)))


def _dims(name):
    d = name.split("_")[1]
    return int(d[0]), int(d[1]), int(d[2])


# Permutations (Propositions 2.1 / 2.2) and direct sums of the base tables
# that give the other shapes of Table 2's ranks.
_PERMUTED = {"fmm_332_15": "fmm_323_15", "fmm_233_15": "fmm_323_15",
             "fmm_324_20": "fmm_423_20", "fmm_342_20": "fmm_423_20", "fmm_243_20": "fmm_423_20",
             "fmm_234_20": "fmm_423_20", "fmm_432_20": "fmm_423_20",
             "fmm_442_26": "fmm_424_26", "fmm_244_26": "fmm_424_26",
             "fmm_232_11": "fmm_223_11", "fmm_322_11": "fmm_223_11",
             "fmm_252_18": "fmm_225_18", "fmm_522_18": "fmm_225_18",
             "fmm_343_29": "fmm_334_29", "fmm_433_29": "fmm_334_29",
             "fmm_344_38": "fmm_434_38", "fmm_443_38": "fmm_434_38"}


def get(name) -> Algorithm:
    if name == "strassen_222_7":
        return strassen()
    if name == "classical_222_8":
        return classical_222()
    if name == "fmm_333_23":
        return laderman_333()
    if name == "winograd_222_7":
        return winograd_222()
    if name == "fmm_223_11":
        # Strassen on two block columns of B and C, classical on the third
        return direct_sum_n([strassen(), classical(2, 2, 1)], name)
    if name == "fmm_225_18":
        return direct_sum_n([strassen(), strassen(), classical(2, 2, 1)], name)
    if name in _PERMUTED:
        return permuted(get(_PERMUTED[name]), _dims(name), name)
    path = os.path.join(_HERE, "tables", name + ".txt")
    if os.path.exists(path):
        return load_table(path, name)
    raise KeyError(name)


def names() -> List[str]:
    out = ["classical_222_8", "strassen_222_7", "fmm_333_23", "fmm_223_11", "fmm_225_18", "winograd_222_7"]
    out += sorted(_PERMUTED)
    for fn in sorted(os.listdir(os.path.join(_HERE, "tables"))):
        if fn.endswith(".txt"):
            out.append(fn[:-4])
    return out


def additions(alg: Algorithm) -> int:
    """Block additions of one recursive step: sum over the columns of U and V
    and the rows of W of (nnz - 1), the count Section 2.1 gives as 18 for
    Strassen."""
    cnt = 0
    for r in range(alg.R):
        cnt += max(0, sum(1 for i in range(alg.M * alg.K) if alg.U[i][r]) - 1)
        cnt += max(0, sum(1 for j in range(alg.K * alg.N) if alg.V[j][r]) - 1)
    for k in range(alg.M * alg.N):
        cnt += max(0, sum(1 for r in range(alg.R) if alg.W[k][r]) - 1)
    return cnt


def compose(a, b):
    """The bilinear algorithm of two recursion levels, `a` on top and `b`
    below (Section 5.2 composes base cases across levels): the
    <a.M b.M, a.K b.K, a.N b.N; a.R b.R> algorithm whose product r = r1 b.R + r2
    multiplies S_{r1 r2} = sum U_a[i1][r1] U_b[i2][r2] A_{i1 i2} by the
    corresponding T, where block (x1, x2) of a level-one block x1 is block
    x1 * (inner count) + x2 in each row and column direction of the composed
    partition.  Its factor matrices are Kronecker products of a's and b's with
    the block indices interleaved, so it passes the Brent equations exactly
    when a and b do."""
    M, K, N, R = a.M * b.M, a.K * b.K, a.N * b.N, a.R * b.R

    def side(Xa, Xb, rows_a, cols_a, rows_b, cols_b):
        out = [[0] * R for _ in range(rows_a * rows_b * cols_a * cols_b)]
        for r1 in range(a.R):
            for r2 in range(b.R):
                r = r1 * b.R + r2
                for i1 in range(rows_a * cols_a):
                    c1 = Xa[i1][r1]
                    if c1 == 0:
                        continue
                    x1, y1 = divmod(i1, cols_a)
                    for i2 in range(rows_b * cols_b):
                        c2 = Xb[i2][r2]
                        if c2 == 0:
                            continue
                        x2, y2 = divmod(i2, cols_b)
                        row, col = x1 * rows_b + x2, y1 * cols_b + y2
                        out[row * (cols_a * cols_b) + col][r] = c1 * c2
        return tuple(tuple(v) for v in out)

    U = side(a.U, b.U, a.M, a.K, b.M, b.K)
    V = side(a.V, b.V, a.K, a.N, b.K, b.N)
    W = side(a.W, b.W, a.M, a.N, b.M, b.N)
    return Algorithm(f"{a.name}+{b.name}", M, K, N, R, U, V, W)
