"""Generate the base-case tables compiled into the library.

Each table is a bilinear decomposition [[U,V,W]] of the <M,K,N> matrix
multiplication tensor (Section 2.2 of Benson and Ballard, PPoPP 2015): U is
MK x R over the row-wise blocks of A, V is KN x R over the blocks of B, W is
MN x R over the blocks of C.  The library checks every table against the
Brent equations when it loads (fmm_check_algorithms), so a corrupted table
fails loudly rather than computing a wrong product.

Three kinds of table:
* text tables in this folder (the classical and Strassen schemes, Laderman's
  <3,3,3;23>, and decompositions found by the search in search.c);
* permutations of those by Propositions 2.1 and 2.2 of Section 2.3: from an
  algorithm for <M,K,N>, [[P_KxN V, P_MxK U, P_MxN W]] solves <N,K,M> and
  [[P_MxN W, U, P_KxN V]] solves <N,M,K> (P_IxJ maps the row-wise vector of
  an I x J matrix to that of its transpose); the sequence applied is the
  first, in the order '', '1', '2', '11', '12', '21', '22', ..., whose
  dimensions are the wanted ones;
* direct sums along N: an algorithm for <M,K,N1> and one for <M,K,N2> give
  <M,K,N1+N2> with R1 + R2 products (B and C split into column blocks), e.g.
  <2,2,3;11> from Strassen's <2,2,2;7> and the classical <2,2,1;4>.

Writes csrc/fmm_tables.h (all tables as compile-time constants) and one
source file per table under csrc/gen/ that instantiates the addition kernels
for that table, so the library builds them in parallel.

Run as a build step: ``python paper_1409_2908_amd/algorithms/gen_tables.py``.
"""
import itertools
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "csrc")
OUT = os.path.join(CSRC, "fmm_tables.h")
GEN = os.path.join(CSRC, "gen")

# name -> recipe.  ("text",): the text table of that name.  ("perm", base):
# a permutation of `base` by Propositions 2.1 / 2.2 to the name's dimensions.
# ("sum", a, b, ...): the direct sum along N of the named algorithms.
# The order fixes the algorithm ids of the kernels' template dispatch.
RECIPES = [
    ("classical_222_8", ("text",)),
    ("strassen_222_7", ("text",)),
    ("fmm_333_23", ("text",)),
    ("fmm_323_15", ("text",)),
    ("fmm_423_20", ("text",)),
    ("fmm_424_26", ("text",)),
    ("winograd_222_7", ("text",)),
    ("fmm_334_29", ("text",)),
    ("fmm_343_29", ("perm", "fmm_334_29")),
    ("fmm_433_29", ("perm", "fmm_334_29")),
    ("fmm_332_15", ("perm", "fmm_323_15")),
    ("fmm_233_15", ("perm", "fmm_323_15")),
    ("fmm_324_20", ("perm", "fmm_423_20")),
    ("fmm_342_20", ("perm", "fmm_423_20")),
    ("fmm_243_20", ("perm", "fmm_423_20")),
    ("fmm_234_20", ("perm", "fmm_423_20")),
    ("fmm_432_20", ("perm", "fmm_423_20")),
    ("fmm_442_26", ("perm", "fmm_424_26")),
    ("fmm_244_26", ("perm", "fmm_424_26")),
    ("fmm_223_11", ("sum", "strassen_222_7", "classical_221_4")),
    ("fmm_232_11", ("perm", "fmm_223_11")),
    ("fmm_322_11", ("perm", "fmm_223_11")),
    ("fmm_225_18", ("sum", "strassen_222_7", "strassen_222_7", "classical_221_4")),
    ("fmm_252_18", ("perm", "fmm_225_18")),
    ("fmm_522_18", ("perm", "fmm_225_18")),
    ("fmm_434_38", ("text",)),
    ("fmm_344_38", ("perm", "fmm_434_38")),
    ("fmm_443_38", ("perm", "fmm_434_38")),
]


def read(name):
    rows = []
    with open(os.path.join(HERE, name + ".txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([int(t) for t in line.split()])
    M, K, N, R = rows[0]
    body = rows[1:]
    assert len(body) == M * K + K * N + M * N
    U = body[:M * K]
    V = body[M * K:M * K + K * N]
    W = body[M * K + K * N:]
    return M, K, N, R, U, V, W


def classical(M, K, N):
    """The classical <M,K,N;MKN> scheme: product (a, b, c) = A_ab B_bc into C_ac."""
    R = M * K * N
    U = [[0] * R for _ in range(M * K)]
    V = [[0] * R for _ in range(K * N)]
    W = [[0] * R for _ in range(M * N)]
    for r, (a, b, c) in enumerate(itertools.product(range(M), range(K), range(N))):
        U[a * K + b][r] = 1
        V[b * N + c][r] = 1
        W[a * N + c][r] = 1
    return M, K, N, R, U, V, W


def transpose_perm(I, J, X):
    """Rows of X permuted by P_IxJ: row i*J + j of X becomes row j*I + i."""
    out = [None] * (I * J)
    for i in range(I):
        for j in range(J):
            out[j * I + i] = list(X[i * J + j])
    return out


def prop21(alg):
    M, K, N, R, U, V, W = alg
    return N, K, M, R, transpose_perm(K, N, V), transpose_perm(M, K, U), transpose_perm(M, N, W)


def prop22(alg):
    M, K, N, R, U, V, W = alg
    return N, M, K, R, transpose_perm(M, N, W), [list(r) for r in U], transpose_perm(K, N, V)


def permute_to(alg, dims):
    """The first proposition sequence (by length, then '1' before '2')
    taking alg to the wanted dimensions."""
    for length in range(0, 4):
        for seq in itertools.product("12", repeat=length):
            x = alg
            for p in seq:
                x = prop21(x) if p == "1" else prop22(x)
            if x[:3] == dims:
                return x
    raise ValueError(f"no permutation gives {dims}")


def direct_sum(algs):
    """Direct sum along N: products of the first algorithm first."""
    M, K = algs[0][0], algs[0][1]
    assert all(a[0] == M and a[1] == K for a in algs)
    N = sum(a[2] for a in algs)
    R = sum(a[3] for a in algs)
    U = [[] for _ in range(M * K)]
    V = [[0] * R for _ in range(K * N)]
    W = [[0] * R for _ in range(M * N)]
    r0 = c0 = 0
    for (_, _, n, rr, u, v, w) in algs:
        for i in range(M * K):
            U[i] += list(u[i])
        for b in range(K):
            for c in range(n):
                for r in range(rr):
                    V[b * N + c0 + c][r0 + r] = v[b * n + c][r]
        for a in range(M):
            for c in range(n):
                for r in range(rr):
                    W[a * N + c0 + c][r0 + r] = w[a * n + c][r]
        r0 += rr
        c0 += n
    return M, K, N, R, U, V, W


def dims_of(name):
    d = name.split("_")[1]
    return int(d[0]), int(d[1]), int(d[2])


def build_all():
    made = {}

    def get(name):
        if name in made:
            return made[name]
        if name.startswith("classical_") and name != "classical_222_8":
            made[name] = classical(*dims_of(name))
            return made[name]
        recipe = dict(RECIPES)[name]
        if recipe[0] == "text":
            alg = read(name)
        elif recipe[0] == "perm":
            alg = permute_to(get(recipe[1]), dims_of(name))
        else:
            alg = direct_sum([get(x) for x in recipe[1:]])
        M, K, N, R, U, V, W = alg
        assert (M, K, N) == dims_of(name) and R == int(name.split("_")[2]), name
        for X in (U, V, W):
            for r in X:
                assert len(r) == R
                for v in r:
                    # 0 or +-2^e, so that a fused multiply-add rounds like the
                    # scaled add; +-3 only in base cases that are never fused
                    # (the fused combination kernels use multiply-adds and
                    # check their coefficients at compile time)
                    assert v == 0 or (abs(v) & (abs(v) - 1)) == 0 or (abs(v) == 3 and R > 32), (name, v)
        made[name] = alg
        return alg

    return [(name, get(name)) for name, _ in RECIPES]


def arr(X):
    return "{" + ", ".join("{" + ", ".join(str(v) for v in r) + "}" for r in X) + "}"


def write_if_changed(path, text):
    old = open(path).read() if os.path.exists(path) else None
    if old != text:
        with open(path, "w") as f:
            f.write(text)


INST = """// Generated by algorithms/gen_tables.py. Do not edit.
// Addition kernels (operand formation and W-combination) of base case {id} ({name}).
#include "../fmm_add_kernels.h"

namespace fmm {{
template hipError_t launch_form_id<{id}>(const FormArgs&, int, int, int, hipStream_t);
template hipError_t launch_form_pair_id<{id}>(const FormArgs&, int, const FormArgs&, int, hipStream_t);
template hipError_t launch_combine_id<{id}>(const CombineArgs&, int, int, hipStream_t);
}}  // namespace fmm
"""


def generate():
    tables = build_all()
    out = ["// Generated by algorithms/gen_tables.py from the text tables beside it. Do not edit.",
           "// Bilinear base cases [[U,V,W]] for <M,K,N;R> (row-wise block vectorisation:",
           "// A block i = a*K+b, B block j = b*N+c, C block k = a*N+c).",
           "#pragma once", "", "namespace fmm {", "",
           f"constexpr int kNumAlgorithms = {len(tables)};", "",
           "template <int ID> struct Alg;", ""]
    for i, (name, (M, K, N, R, U, V, W)) in enumerate(tables):
        out += [f"// {name}",
                f"template <> struct Alg<{i}> {{",
                f"  static constexpr int M = {M}, K = {K}, N = {N}, R = {R};",
                f"  static constexpr signed char U[{M * K}][{R}] = {arr(U)};",
                f"  static constexpr signed char V[{K * N}][{R}] = {arr(V)};",
                f"  static constexpr signed char W[{M * N}][{R}] = {arr(W)};",
                "};", ""]
    out += ["struct AlgInfo { const char* name; int M, K, N, R; const signed char* U; const signed char* V; const signed char* W; };",
            "", "inline const AlgInfo& alg_info(int id) {", "  static const AlgInfo table[kNumAlgorithms] = {"]
    for i, (name, _) in enumerate(tables):
        out.append(f'    {{"{name}", Alg<{i}>::M, Alg<{i}>::K, Alg<{i}>::N, Alg<{i}>::R, '
                   f"&Alg<{i}>::U[0][0], &Alg<{i}>::V[0][0], &Alg<{i}>::W[0][0]}},")
    out += ["  };", "  return table[id];", "}", "", "}  // namespace fmm", ""]
    write_if_changed(OUT, "\n".join(out))
    os.makedirs(GEN, exist_ok=True)
    sources = []
    for i, (name, _) in enumerate(tables):
        path = os.path.join(GEN, f"fmm_add_{i:02d}.hip")
        write_if_changed(path, INST.format(id=i, name=name))
        sources.append(os.path.relpath(path, CSRC))
    return OUT, sources


if __name__ == "__main__":
    print(generate())
