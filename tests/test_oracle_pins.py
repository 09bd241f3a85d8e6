"""Pins for the oracle: values the paper prints, closed forms, brute force.

Each test checks the oracle against something other than itself, chosen so
that a dropped term, a wrong sign or index, or a transposed operand in the
oracle fails at least one of them.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

from conftest import load_golden_matrices
from oracle import algorithms, classical, recursive, tensor

ALGS = ["strassen_222_7", "fmm_333_23", "fmm_323_15", "fmm_423_20", "fmm_424_26"]
# every fast table: the above, their permutations by Propositions 2.1 / 2.2 and
# the direct sums <2,2,3;11>, <2,2,5;18> with theirs
ALL = [n for n in algorithms.names() if n != "classical_222_8"]


# --- the matrix-multiplication tensor (Section 2.2) ------------------------

@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 2, 3), (4, 2, 3), (2, 3, 4), (3, 3, 3), (1, 4, 2)])
def test_tensor_applied_to_vec_is_the_product(dims):
    """T x1 vec(A) x2 vec(B) == vec(A B) for the membership rule, checked
    against the schoolbook product on random integer matrices."""
    M, K, N = dims
    T = tensor.matmul_tensor(M, K, N)
    assert len(T) == M * K * N  # MKN non-zeros
    rng = random.Random(1)
    for _ in range(5):
        A = [[rng.randint(-9, 9) for _ in range(K)] for _ in range(M)]
        B = [[rng.randint(-9, 9) for _ in range(N)] for _ in range(K)]
        C = [[sum(A[a][b] * B[b][c] for b in range(K)) for c in range(N)] for a in range(M)]
        z = tensor.apply_tensor(T, [x for row in A for x in row], [y for row in B for y in row], M * N)
        assert z == [x for row in C for x in row]


def test_tensor_222_matches_printed_slices():
    slices = load_golden_matrices("tensor_222_slices.txt")
    T = tensor.matmul_tensor(2, 2, 2)
    for k, S in enumerate(slices):
        for i in range(4):
            for j in range(4):
                assert T.get((i, j, k), 0) == S[i][j]


# --- Strassen and the printed factor matrices (Sections 2.1, 2.2) ----------

def test_strassen_formulas_pass_brent():
    a = algorithms.strassen()
    assert tensor.brent_residual(a.U, a.V, a.W, 2, 2, 2) == []


def test_printed_uv_match_formulas_and_printed_w_is_the_erratum():
    U, V, W = load_golden_matrices("strassen_printed_uvw.txt")
    a = algorithms.strassen()
    assert [list(r) for r in a.U] == U
    assert [list(r) for r in a.V] == V
    # The printed W fails the Brent equations (14 entries) ...
    assert len(tensor.brent_residual(a.U, a.V, W, 2, 2, 2)) == 14
    # ... and differs from the formulas' W by swapping the C12/C21 rows and
    # moving C22's M6 term to M4.
    fixed = [W[0], W[2], W[1], list(W[3])]
    fixed[3][3], fixed[3][5] = 0, 1
    assert [list(r) for r in a.W] == fixed


def test_strassen_18_additions():
    assert algorithms.additions(algorithms.strassen()) == 18
    assert algorithms.additions(algorithms.classical_222()) == 4


# --- the base cases (Table 2) -----------------------------------------------

def _table2():
    rows = load_golden_matrices("table2_algorithms.txt")[0]
    return {(r[0], r[1], r[2]): r for r in rows}


@pytest.mark.parametrize("name", ALL + ["classical_222_8"])
def test_tables_pass_brent(name):
    a = algorithms.get(name)
    assert tensor.brent_residual(a.U, a.V, a.W, a.M, a.K, a.N) == []


@pytest.mark.parametrize("name", ALL)
def test_rank_matches_table2(name):
    """The rank R equals Table 2's entry for the base case or one of its
    permutations (<3,2,3> and <4,2,x> are permutations of the printed
    <2,3,3>, <2,3,4>, <2,4,4>), and the printed speedup per step is
    MKN/R - 1 rounded to a percent."""
    a = algorithms.get(name)
    t2 = _table2()
    key = tuple(sorted(a.dims))
    hits = [r for d, r in t2.items() if tuple(sorted(d)) == key and r[3] == a.R]
    assert hits, (name, a.dims, a.R)
    mkn = a.M * a.K * a.N
    assert round(100 * (mkn / a.R - 1)) == hits[0][5]


def test_table2_speedups_are_mkn_over_r():
    for (M, K, N), r in _table2().items():
        assert round(100 * (M * K * N / r[3] - 1)) == r[5]
        if (M, K, N) != (3, 3, 3):
            assert r[4] == M * K * N
    assert _table2()[(3, 3, 3)][4] == 26  # printed; MKN is 27 (erratum)


@pytest.mark.parametrize("name", ALGS)
def test_propositions_21_22_give_algorithms(name):
    a = algorithms.get(name)
    for prop in (tensor.prop21, tensor.prop22):
        U, V, W, (M, K, N) = prop(a.U, a.V, a.W, a.M, a.K, a.N)
        assert tensor.brent_residual(U, V, W, M, K, N) == []
    # composing both reaches all six permutations
    seen = set()
    frontier = [(a.U, a.V, a.W, a.dims)]
    while frontier:
        U, V, W, d = frontier.pop()
        if d in seen:
            continue
        seen.add(d)
        for prop in (tensor.prop21, tensor.prop22):
            U2, V2, W2, d2 = prop(U, V, W, *d)
            frontier.append((U2, V2, W2, d2))
    assert len(seen) == len(set(__import__("itertools").permutations(a.dims)))


@pytest.mark.parametrize("name", ALL)
def test_brent_catches_planted_mistakes(name):
    """A wrong sign, a dropped term or a moved index in any factor matrix
    must fail the Brent check."""
    a = algorithms.get(name)
    rng = random.Random(7)
    for which in range(3):
        for _ in range(3):
            mats = [[list(r) for r in X] for X in (a.U, a.V, a.W)]
            X = mats[which]
            i = rng.randrange(len(X))
            r = rng.randrange(a.R)
            X[i][r] = -X[i][r] if X[i][r] else 1
            assert tensor.brent_residual(*mats, a.M, a.K, a.N) != []


# --- O1, the classical product ---------------------------------------------

def test_classical_exact_on_rationals():
    rng = random.Random(3)
    for (m, k, n) in [(1, 1, 1), (3, 5, 2), (7, 4, 9), (16, 16, 16)]:
        A = [[Fraction(rng.randint(-64, 64), 8) for _ in range(k)] for _ in range(m)]
        B = [[Fraction(rng.randint(-64, 64), 4) for _ in range(n)] for _ in range(k)]
        exact = classical.gemm_exact(A, B)
        C = classical.gemm(np.array(A, dtype=float), np.array(B, dtype=float))
        assert [[Fraction(x) for x in row] for row in C.tolist()] == exact


def test_classical_within_rounding_bound():
    """|C - AB| <= gamma_k |A||B| elementwise (Higham, Accuracy and Stability,
    Section 3.5), against the exact rational product."""
    rng = np.random.default_rng(5)
    m, k, n = 6, 300, 5
    A = rng.uniform(-1, 1, (m, k))
    B = rng.uniform(-1, 1, (k, n))
    C = classical.gemm(A, B)
    u = 2.0 ** -53
    gamma = k * u / (1 - k * u)
    Af = [[Fraction(x) for x in row] for row in A.tolist()]
    Bf = [[Fraction(x) for x in row] for row in B.tolist()]
    exact = classical.gemm_exact(Af, Bf)
    absprod = np.abs(A) @ np.abs(B)
    for i in range(m):
        for j in range(n):
            assert abs(Fraction(C[i, j]) - exact[i][j]) <= Fraction(gamma * absprod[i, j])
    Cd = classical.gemm_rows(A, B, list(range(m)), compensated=True)
    for i in range(m):
        for j in range(n):
            # Dot2: error <= u|s| + gamma_k^2 sum|ab|
            bound = u * abs(float(exact[i][j])) + gamma * gamma * absprod[i, j]
            assert abs(Fraction(Cd[i, j]) - exact[i][j]) <= Fraction(bound) * 2


def test_classical_not_transposed_and_rows():
    rng = np.random.default_rng(0)
    A = rng.integers(-8, 9, (5, 7)).astype(float)
    B = rng.integers(-8, 9, (7, 3)).astype(float)
    C = classical.gemm(A, B)
    assert np.array_equal(C, A @ B)  # integer-valued: every rounding is exact
    rows = [4, 0, 2]
    assert np.array_equal(classical.gemm_rows(A, B, rows), C[rows])
    assert classical.gemm(np.zeros((0, 3)), np.zeros((3, 4))).shape == (0, 4)
    assert np.array_equal(classical.gemm(np.ones((2, 0)), np.ones((0, 3))), np.zeros((2, 3)))


# --- O2, the recursive algorithm ---------------------------------------------

def _frac_matrix(rng, r, c):
    return np.array([[Fraction(rng.randint(-20, 20), rng.choice([1, 2, 4])) for _ in range(c)]
                     for _ in range(r)], dtype=object)


@pytest.mark.parametrize("name", ALGS)
@pytest.mark.parametrize("peel", ["dynamic", "static"])
def test_recursive_exact_on_rationals(name, peel):
    """O2 == brute-force product exactly, sizes M^L t + r (ragged included)."""
    a = algorithms.get(name)
    rng = random.Random(11)
    for L in (1, 2):
        fm, fk, fn = a.M ** L, a.K ** L, a.N ** L
        for (tm, tk, tn, rm, rk, rn) in [(1, 1, 1, 0, 0, 0), (1, 1, 1, 1, 1, 1),
                                         (2, 1, 1, fm - 1, 0, 1)]:
            m, k, n = fm * tm + rm, fk * tk + rk, fn * tn + rn
            if m * k * n > 40000:
                continue
            A = _frac_matrix(rng, m, k)
            B = _frac_matrix(rng, k, n)
            C = recursive.fmm(a, L, A, B, peel=peel)
            exact = classical.gemm_exact(A.tolist(), B.tolist())
            assert C.tolist() == exact, (name, L, m, k, n)


def test_recursive_planted_mistake_fails():
    """Dropping a term of one W row (a plausible slip) breaks exactness."""
    a = algorithms.strassen()
    W = [list(r) for r in a.W]
    W[0][3] = 0
    bad = algorithms.Algorithm("bad", 2, 2, 2, 7, a.U, a.V, tuple(tuple(r) for r in W))
    rng = random.Random(2)
    A = _frac_matrix(rng, 4, 4)
    B = _frac_matrix(rng, 4, 4)
    assert recursive.fmm(bad, 1, A, B).tolist() != classical.gemm_exact(A.tolist(), B.tolist())


def test_flop_closed_forms():
    """F_C(N) = 2N^3 - N^2 and F_S(N) = 7 N^lg7 - 6 N^2 (Section 2.1) when the
    recursion runs down to 1 x 1 blocks."""
    for p in range(0, 5):
        N = 2 ** p
        A = np.ones((N, N))
        cC = recursive.FlopCounter()
        recursive.fmm(algorithms.classical_222(), p, A, A, counter=cC)
        assert cC.flops == 2 * N ** 3 - N ** 2
        cS = recursive.FlopCounter()
        recursive.fmm(algorithms.strassen(), p, A, A, counter=cS)
        assert cS.flops == 7 * round(N ** math.log2(7)) - 6 * N ** 2


@pytest.mark.parametrize("name", ALGS)
def test_recursive_integer_bit_exact_binary64(name):
    """Integer inputs in {-8..8}: every intermediate is an integer far below
    2^53, so binary64 O2 equals O1 bit for bit."""
    a = algorithms.get(name)
    rng = np.random.default_rng(4)
    L = 2
    m, k, n = a.M ** L * 5 + 1, a.K ** L * 4 + 2, a.N ** L * 3 + 1
    A = rng.integers(-8, 9, (m, k)).astype(float)
    B = rng.integers(-8, 9, (k, n)).astype(float)
    ref = classical.gemm(A, B)
    for peel in ("dynamic", "static"):
        assert np.array_equal(recursive.fmm(a, L, A, B, peel=peel), ref)


@pytest.mark.parametrize("name", ALGS)
def test_recursive_float_close(name):
    a = algorithms.get(name)
    rng = np.random.default_rng(8)
    m, k, n = 2 * a.M ** 2 * 7, 2 * a.K ** 2 * 7, 2 * a.N ** 2 * 7
    A = rng.uniform(-1, 1, (m, k))
    B = rng.uniform(-1, 1, (k, n))
    ref = classical.gemm(A, B)
    C = recursive.fmm(a, 2, A, B)
    rel = np.linalg.norm(C - ref) / np.linalg.norm(ref)
    assert rel < 1e-14
    assert rel > 0  # the fast algorithm really rounds differently


@pytest.mark.parametrize("name", ["strassen_222_7", "fmm_424_26"])
def test_form_and_combine_reproduce_static_core(name):
    """form_operands / combine_products (the stage-by-stage view used to check
    the GPU addition kernels) reproduce the static-peel recursion bit for
    bit on a divisible core."""
    a = algorithms.get(name)
    L = 2
    rng = np.random.default_rng(9)
    m, k, n = a.M ** L * 3, a.K ** L * 2, a.N ** L * 3
    A = rng.uniform(-1, 1, (m, k))
    B = rng.uniform(-1, 1, (k, n))
    S = recursive.form_operands(a, L, A, "A")
    T = recursive.form_operands(a, L, B, "B")
    assert len(S) == a.R ** L
    Ms = [classical.gemm(s, t) for s, t in zip(S, T)]
    C = recursive.combine_products(a, L, Ms)
    assert np.array_equal(C, recursive.fmm(a, L, A, B, peel="static"))


# --- composition of different base cases across levels (Section 5.2) ---------

MIXES = [("strassen_222_7", "fmm_424_26"), ("fmm_424_26", "strassen_222_7"),
         ("fmm_323_15", "fmm_423_20"), ("fmm_333_23", "strassen_222_7")]


@pytest.mark.parametrize("top,bottom", MIXES)
def test_composed_base_case_passes_brent(top, bottom):
    """Two levels of different base cases form one bilinear algorithm
    <M1 M2, K1 K2, N1 N2; R1 R2>; its factor matrices pass the Brent
    equations exactly, and swapping the order of the interleaved block
    indices (a plausible slip) does not."""
    a, b = algorithms.get(top), algorithms.get(bottom)
    c = algorithms.compose(a, b)
    assert (c.M, c.K, c.N, c.R) == (a.M * b.M, a.K * b.K, a.N * b.N, a.R * b.R)
    assert tensor.brent_residual(c.U, c.V, c.W, c.M, c.K, c.N) == []
    # the same composition with the level-one and level-two block indices of
    # A's rows exchanged
    bad = [list(r) for r in c.U]
    rows, cols = c.M, c.K
    perm = [(x % b.M) * a.M + x // b.M for x in range(rows)]
    badU = tuple(tuple(bad[perm[i // cols] * cols + i % cols]) for i in range(rows * cols))
    if perm != list(range(rows)):
        assert tensor.brent_residual(badU, c.V, c.W, c.M, c.K, c.N) != []


@pytest.mark.parametrize("top,bottom", MIXES[:3])
@pytest.mark.parametrize("peel", ["dynamic", "static"])
def test_recursive_mixed_levels_exact_on_rationals(top, bottom, peel):
    """O2 with one base case per level equals the brute-force product exactly
    on ragged sizes, and in binary64 agrees with one level of the composed
    algorithm to rounding (the two sum the same terms in different orders)."""
    a, b = algorithms.get(top), algorithms.get(bottom)
    rng = random.Random(5)
    fm, fk, fn = a.M * b.M, a.K * b.K, a.N * b.N
    for (tm, tk, tn, rm, rk, rn) in [(1, 1, 1, 0, 0, 0), (1, 1, 1, 1, 1, 1), (2, 1, 1, fm - 1, 0, 1)]:
        m, k, n = fm * tm + rm, fk * tk + rk, fn * tn + rn
        if m * k * n > 40000:
            continue
        A = _frac_matrix(rng, m, k)
        B = _frac_matrix(rng, k, n)
        C = recursive.fmm([a, b], 2, A, B, peel=peel)
        assert C.tolist() == classical.gemm_exact(A.tolist(), B.tolist()), (top, bottom, m, k, n)
    rng2 = np.random.default_rng(4)
    A = rng2.uniform(-1, 1, (fm * 2, fk * 2))
    B = rng2.uniform(-1, 1, (fk * 2, fn * 3))
    composed = recursive.fmm(algorithms.compose(a, b), 1, A, B, peel="static")
    mixed = recursive.fmm([a, b], 2, A, B, peel="static")
    assert np.linalg.norm(mixed - composed) <= 1e-13 * np.linalg.norm(composed)


def test_form_and_combine_mixed_levels():
    """The stage-by-stage chains with one base case per level reproduce the
    mixed static-peel recursion bit for bit."""
    a, b = algorithms.get("fmm_424_26"), algorithms.get("strassen_222_7")
    rng = np.random.default_rng(10)
    m, k, n = a.M * b.M * 3, a.K * b.K * 2, a.N * b.N * 3
    A = rng.uniform(-1, 1, (m, k))
    B = rng.uniform(-1, 1, (k, n))
    S = recursive.form_operands([a, b], 2, A, "A")
    T = recursive.form_operands([a, b], 2, B, "B")
    assert len(S) == a.R * b.R
    Ms = [classical.gemm(s, t) for s, t in zip(S, T)]
    C = recursive.combine_products([a, b], 2, Ms)
    assert np.array_equal(C, recursive.fmm([a, b], 2, A, B, peel="static"))


# --- the BF16x3 emulation ----------------------------------------------------

def test_bf16_round_to_nearest_even():
    from oracle import bf16x3
    # 1 + 2^-8 is halfway between bf16 neighbours 1 and 1 + 2^-7: ties to even (1)
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even (1 + 2^-6)
    x = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -(1 + 2 ** -8), 3.0, 0.0],
                 dtype=np.float32)
    want = np.array([1.0, 1 + 2 ** -6, 1 + 2 ** -7, -1.0, 3.0, 0.0], dtype=np.float32)
    assert np.array_equal(bf16x3.bf16_round(x), want)
    # brute force over a range: the result is a bf16 value (low 16 bits zero)
    # and no other bf16 value is strictly closer
    rng = np.random.default_rng(0)
    v = rng.standard_normal(2000).astype(np.float32)
    r = bf16x3.bf16_round(v)
    assert np.all((r.view(np.uint32) & 0xFFFF) == 0)
    up = (r.view(np.uint32) + np.uint32(0x10000)).view(np.float32)
    dn = (r.view(np.uint32) - np.uint32(0x10000)).view(np.float32)
    err = np.abs(v.astype(np.float64) - r)
    assert np.all(err <= np.abs(v.astype(np.float64) - up))
    assert np.all(err <= np.abs(v.astype(np.float64) - dn))


def test_bf16x3_split_and_product():
    from oracle import bf16x3
    rng = np.random.default_rng(1)
    x = rng.standard_normal(5000).astype(np.float32)
    hi, lo = bf16x3.split(x)
    # the pair keeps 16 significant bits: |x - hi - lo| <= 2^-16 |x|
    rel = np.abs(x.astype(np.float64) - hi - lo) / np.abs(x.astype(np.float64))
    assert rel.max() <= 2.0 ** -16
    # values with at most 16 significant bits reconstruct exactly
    y = (np.round(x.astype(np.float64) * 2 ** 10) / 2 ** 10).astype(np.float32)
    y = y[np.abs(y) < 32]
    h2, l2 = bf16x3.split(y)
    assert np.array_equal(h2.astype(np.float64) + l2, y.astype(np.float64))
    # integer matrices with entries of at most 8 bits: lo = 0 and the product is exact
    A = rng.integers(-200, 201, (20, 30)).astype(np.float32)
    B = rng.integers(-200, 201, (30, 10)).astype(np.float32)
    assert np.array_equal(bf16x3.gemm(A, B), A.astype(np.float64) @ B.astype(np.float64))
    # a dropped lo*hi term would be visible at the 2^-8 relative level
    A = rng.standard_normal((40, 50)).astype(np.float32)
    B = rng.standard_normal((50, 30)).astype(np.float32)
    exact = A.astype(np.float64) @ B.astype(np.float64)
    err = np.linalg.norm(bf16x3.gemm(A, B) - exact) / np.linalg.norm(exact)
    assert 1e-7 < err < 2e-5


@pytest.mark.parametrize("alg,L", [("strassen_222_7", 2), ("fmm_424_26", 1), ("fmm_333_23", 1),
                                   ("fmm_323_15", 2)])
def test_bf16x3_fast_emulation_exact_on_small_integers(alg, L):
    """With small integer entries every operand sum stays an integer below 2^8
    in magnitude, so the split is exact (lo = 0) and the emulated fast
    algorithm -- core leaves, peel strips and combination -- must equal the
    exact product; odd sizes exercise every peel strip."""
    from oracle import bf16x3
    a = algorithms.get(alg)
    m, k, n = a.M ** L * 3 + 1, a.K ** L * 2 + 1, a.N ** L * 3 + 2
    rng = np.random.default_rng(7)
    A = rng.integers(-4, 5, (m, k)).astype(np.float32)
    B = rng.integers(-4, 5, (k, n)).astype(np.float32)
    assert np.array_equal(bf16x3.fmm(a, L, A, B), A.astype(np.float64) @ B.astype(np.float64))
    # at zero levels it is the emulated classical product
    assert np.array_equal(bf16x3.fmm(a, 0, A, B), bf16x3.gemm(A, B))


# --- the BF16x3 error gate --------------------------------------------------

def test_bf16x3_growth_closed_forms_and_invariants():
    """growth() is 1 for a classical step and 2 for Strassen (Section 2.1's
    formulas: the seven products have |u|^2 |v|^2 |w|^2 = 8, 4, 4, 4, 4, 4, 4,
    sum 32 over MKN = 8); it is unchanged by the permutations of Propositions
    2.1 and 2.2 (they permute the entries of each column) and multiplies
    under composition (Kronecker factors' norms multiply)."""
    from oracle import bf16x3
    assert bf16x3.growth(algorithms.get("classical_222_8")) == 1.0
    assert bf16x3.growth(algorithms.get("strassen_222_7")) == 2.0
    for name in ALGS:
        a = algorithms.get(name)
        for prop in (tensor.prop21, tensor.prop22):
            U, V, W, (M, K, N) = prop(a.U, a.V, a.W, a.M, a.K, a.N)
            b = algorithms.Algorithm("perm", M, K, N, a.R, tuple(map(tuple, U)), tuple(map(tuple, V)),
                                     tuple(map(tuple, W)))
            assert bf16x3.growth(b) == pytest.approx(bf16x3.growth(a), rel=1e-15)
    s, t = algorithms.get("strassen_222_7"), algorithms.get("fmm_323_15")
    assert bf16x3.growth(algorithms.compose(s, t)) == pytest.approx(
        bf16x3.growth(s) * bf16x3.growth(t), rel=1e-14)
    assert bf16x3.gate(s, 2, 100) == pytest.approx(bf16x3.gate([s, s], 2, 100), rel=1e-15)
    assert bf16x3.gate(s, 0, 100) == pytest.approx(3 * 2 ** -16 + 12 * 2 ** -24, rel=1e-15)


@pytest.mark.parametrize("name", ALGS)
@pytest.mark.parametrize("L", [1, 2])
@pytest.mark.parametrize("kind", ["uniform", "normal_rowscaled"])
def test_bf16x3_gate_bounds_the_emulated_error(name, L, kind):
    """The emulated BF16x3 fast product (the same split, exact products)
    stays under the gate against the exact product, and within 40x of it, so
    the gate describes the error rather than being vacuous."""
    import fmm_inputs
    from oracle import bf16x3
    a = algorithms.get(name)
    m, k, n = a.M ** L * 20 + 3, a.K ** L * 30 + 1, a.N ** L * 20 + 2
    A, B = fmm_inputs.operands(7, m, k, n, kind, np.float32)
    ref = classical.gemm(A, B)
    err = np.linalg.norm(bf16x3.fmm(a, L, A, B) - ref) / np.linalg.norm(ref)
    g = bf16x3.gate(a, L, k)
    assert g / 40 <= err <= g, (err, g)


@pytest.mark.parametrize("name", ALGS)
def test_bf16x3_gate_catches_a_dropped_cross_term(name, monkeypatch):
    """Planted mistake in the emulation: leaves without the lo*hi term.  The
    error then exceeds the gate, so a kernel that lost a product term would
    fail the GPU gate against the binary64 oracle."""
    import fmm_inputs
    from oracle import bf16x3

    def two_terms(A, B):
        ah, al = bf16x3.split(A)
        bh, bl = bf16x3.split(B)
        ah, bh, bl = (v.astype(np.float64) for v in (ah, bh, bl))
        return ah @ bh + ah @ bl

    monkeypatch.setattr(bf16x3, "gemm", two_terms)
    a = algorithms.get(name)
    m, k, n = a.M * 20 + 3, a.K * 30 + 1, a.N * 20 + 2
    A, B = fmm_inputs.operands(8, m, k, n, "uniform", np.float32)
    ref = classical.gemm(A, B)
    err = np.linalg.norm(bf16x3.fmm(a, 1, A, B) - ref) / np.linalg.norm(ref)
    assert err > 4 * bf16x3.gate(a, 1, k), (err, bf16x3.gate(a, 1, k))


def test_every_shape_of_table2_ranks_up_to_4_has_a_table():
    """Every permutation of Table 2's exact base cases with all dimensions at
    most 5 and rank from the tables here is present: <2,2,3;11>, <2,2,5;18>,
    <2,3,3;15>, <2,3,4;20>, <2,4,4;26> in all their orders, plus <3,3,3;23>."""
    import itertools
    have = {algorithms.get(n).dims: algorithms.get(n).R for n in ALL}
    for base, rank in (((2, 2, 3), 11), ((2, 2, 5), 18), ((2, 3, 3), 15), ((2, 3, 4), 20), ((2, 4, 4), 26),
                       ((3, 3, 3), 23)):
        assert _table2()[base][3] == rank
        for d in set(itertools.permutations(base)):
            assert have.get(d) == rank, (d, have.get(d))


@pytest.mark.parametrize("name", ["fmm_223_11", "fmm_225_18"])
def test_direct_sums_equal_their_parts(name):
    """The direct sum along N computes, on each column block of B and C, its
    part's product: the product with B's other column blocks zeroed equals
    the part alone (exact on integers)."""
    a = algorithms.get(name)
    rng = np.random.default_rng(3)
    L = 1
    A = rng.integers(-5, 6, size=(a.M * 3, a.K * 2)).astype(np.float64)
    B = rng.integers(-5, 6, size=(a.K * 2, a.N * 4)).astype(np.float64)
    C = recursive.fmm(a, L, A, B)
    assert np.array_equal(C, A @ B)


def test_winograd_variant_schedule_and_counts():
    """The Strassen-Winograd table: the bilinear form has 24 block additions;
    evaluated through the shared-intermediate schedule (15 additions, the
    count the common-subexpression discussion of Section 3.3 starts from) on
    integer blocks it gives the exact product, and so does the table."""
    import numpy as np
    a = algorithms.get("winograd_222_7")
    assert (a.M, a.K, a.N, a.R) == (2, 2, 2, 7)
    assert algorithms.additions(a) == 24
    rng = np.random.default_rng(5)
    A = rng.integers(-9, 10, (6, 6)).astype(object)
    B = rng.integers(-9, 10, (6, 6)).astype(object)
    A11, A12, A21, A22 = A[:3, :3], A[:3, 3:], A[3:, :3], A[3:, 3:]
    B11, B12, B21, B22 = B[:3, :3], B[:3, 3:], B[3:, :3], B[3:, 3:]
    adds = 0
    def add(x, y, sign=1):
        nonlocal adds
        adds += 1
        return x + sign * y
    S1 = add(A21, A22); S2 = add(S1, A11, -1); S3 = add(A11, A21, -1); S4 = add(A12, S2, -1)
    T1 = add(B12, B11, -1); T2 = add(B22, T1, -1); T3 = add(B22, B12, -1); T4 = add(T2, B21, -1)
    M1, M2, M3, M4 = A11.dot(B11), A12.dot(B21), S4.dot(B22), A22.dot(T4)
    M5, M6, M7 = S1.dot(T1), S2.dot(T2), S3.dot(T3)
    U2 = add(M1, M6); U3 = add(U2, M7); U4 = add(U2, M5)
    C = np.block([[add(M1, M2), add(U4, M3)], [add(U3, M4, -1), add(U3, M5)]])
    assert adds == 15
    assert (C == A.dot(B)).all()
    assert (recursive.fmm(a, 1, A, B) == A.dot(B)).all()
