"""Matrix-multiplication tensor, exact Brent check and permutation transforms.

Test infrastructure (see oracle/__init__.py).  Everything here is exact
integer/rational arithmetic.
"""
from fractions import Fraction


def matmul_tensor(M, K, N):
    """The <M,K,N> tensor of Section 2.2 as a dict {(i,j,k): 1} of its MKN
    non-zeros, 0-indexed, built from the 1-indexed membership rule stated
    there: T_ijk = 1 iff (i-1) mod K == floor((j-1)/N), (j-1) mod N ==
    (k-1) mod N and floor((i-1)/K) == floor((k-1)/N).  Indices follow the
    row-wise vectorisation of Table 1 (A is MxK, B is KxN, C is MxN)."""
    nz = {}
    for i1 in range(1, M * K + 1):
        for j1 in range(1, K * N + 1):
            for k1 in range(1, M * N + 1):
                if ((i1 - 1) % K == (j1 - 1) // N
                        and (j1 - 1) % N == (k1 - 1) % N
                        and (i1 - 1) // K == (k1 - 1) // N):
                    nz[(i1 - 1, j1 - 1, k1 - 1)] = 1
    return nz


def apply_tensor(nz, x, y, size_k):
    """z = T x_1 x x_2 y, i.e. z_k = sum_ij T_ijk x_i y_j (Equation (1))."""
    z = [0] * size_k
    for (i, j, k), t in nz.items():
        z[k] += t * x[i] * y[j]
    return z


def brent_residual(U, V, W, M, K, N):
    """All (i,j,k) where sum_r U_ir V_jr W_kr differs from T_ijk
    (Equation (2)); U is MK x R, V is KN x R, W is MN x R, entries int or
    Fraction.  An empty list means [[U,V,W]] is an exact algorithm."""
    R = len(U[0])
    assert len(U) == M * K and len(V) == K * N and len(W) == M * N
    assert all(len(row) == R for row in list(U) + list(V) + list(W))
    T = matmul_tensor(M, K, N)
    bad = []
    for i in range(M * K):
        ui = [Fraction(u) for u in U[i]]
        for j in range(K * N):
            vj = [Fraction(v) for v in V[j]]
            uv = [ui[r] * vj[r] for r in range(R)]
            for k in range(M * N):
                s = sum((uv[r] * W[k][r] for r in range(R) if uv[r] != 0), Fraction(0))
                if s != T.get((i, j, k), 0):
                    bad.append((i, j, k))
    return bad


def vec_transpose_perm(I, J):
    """P_{IxJ} of Section 2.3: the permutation matrix with P vec(A) = vec(A^T)
    for an I x J matrix A under row-wise vectorisation, as a list of rows."""
    P = [[0] * (I * J) for _ in range(I * J)]
    for i in range(I):
        for j in range(J):
            P[j * I + i][i * J + j] = 1
    return P


def _matmul(P, X):
    return [[sum(P[a][b] * X[b][c] for b in range(len(X))) for c in range(len(X[0]))]
            for a in range(len(P))]


def prop21(U, V, W, M, K, N):
    """Proposition 2.1: [[P_{KxN} V, P_{MxK} U, P_{MxN} W]] solves <N,K,M>."""
    return (_matmul(vec_transpose_perm(K, N), V),
            _matmul(vec_transpose_perm(M, K), U),
            _matmul(vec_transpose_perm(M, N), W), (N, K, M))


def prop22(U, V, W, M, K, N):
    """Proposition 2.2: [[P_{MxN} W, U, P_{KxN} V]] solves <N,M,K>."""
    return (_matmul(vec_transpose_perm(M, N), W),
            [list(r) for r in U],
            _matmul(vec_transpose_perm(K, N), V), (N, M, K))
