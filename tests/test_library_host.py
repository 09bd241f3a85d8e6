"""Host-side checks of the C-ABI library: exports, compiled-in tables, planner.

No GPU needed: these call only entry points that do not touch a device
(fmm_plan_host, fmm_plan_info, fmm_plan_operand, the table queries).
"""
import ctypes
import math
import re

import numpy as np
import pytest

import paper_1409_2908_amd as F
from oracle import algorithms, tensor
from conftest import ROOT

ALGS = algorithms.names()


def test_library_exports_every_declared_symbol():
    with open(f"{ROOT}/include/fmm.h") as f:
        text = f.read()
    names = set(re.findall(r"\b(fmm_[a-z0-9_]+)\s*\(", text))
    assert len(names) >= 15
    lib = ctypes.CDLL(F.library_path())
    for nm in sorted(names):
        assert hasattr(lib, nm), nm


@pytest.mark.parametrize("name", ALGS)
def test_compiled_tables_pass_brent_and_match_oracle_copy(name):
    M, K, N, R, U, V, W = F.algorithm_coeffs(name)
    assert tensor.brent_residual(U.tolist(), V.tolist(), W.tolist(), M, K, N) == []
    a = algorithms.get(name)
    assert (M, K, N, R) == (a.M, a.K, a.N, a.R)
    assert U.tolist() == [list(r) for r in a.U]
    assert V.tolist() == [list(r) for r in a.V]
    assert W.tolist() == [list(r) for r in a.W]


def test_library_and_oracle_list_the_same_tables():
    assert sorted(F.algorithm_names()) == sorted(algorithms.names())


def test_two_level_fusion_rule():
    """Two levels per addition pass for narrow base cases (R <= 8) and for
    wide ones with at most 11 blocks per side and R <= 32; one otherwise."""
    for name in algorithms.names():
        a = algorithms.get(name)
        ok = a.R <= 8 or (a.M * a.K <= 11 and a.K * a.N <= 11 and a.R <= 32)
        p = F.Plan(name, a.M ** 2 * 3, a.K ** 2 * 3, a.N ** 2 * 3, 2, host_only=True, fuse_levels=2)
        assert p.info["fuse_levels"] == (2 if ok else 1), name


def test_library_brent_self_check():
    F.check_algorithms()


def test_unknown_algorithm_and_bad_args():
    with pytest.raises(F.FmmError) as e:
        F.Plan("no_such_alg", 8, 8, 8, 1, host_only=True)
    assert e.value.code == 5
    with pytest.raises(F.FmmError) as e:
        F.Plan("strassen_222_7", -1, 8, 8, 1, host_only=True)
    assert e.value.code == 1
    # depth leaves a leaf dimension < 1
    with pytest.raises(F.FmmError) as e:
        F.Plan("strassen_222_7", 7, 64, 64, 3, host_only=True)
    assert e.value.code == 1
    with pytest.raises(F.FmmError):
        F.Plan("strassen_222_7", 8, 8, 8, 1, dtype=7, host_only=True)
    # leaf tile edge: 0 (per launch), 64 or 128 only
    for tile in (0, 64, 128):
        F.Plan("strassen_222_7", 8, 8, 8, 1, host_only=True, leaf_tile=tile).close()
    for tile in (-1, 32, 96, 256):
        with pytest.raises(F.FmmError) as e:
            F.Plan("strassen_222_7", 8, 8, 8, 1, host_only=True, leaf_tile=tile)
        assert e.value.code == 1


def _ipow(b, e):
    return b ** e


@pytest.mark.parametrize("name,L,shape", [
    ("strassen_222_7", 1, (512, 512, 512)),
    ("strassen_222_7", 3, (9000, 9000, 9000)),
    ("fmm_424_26", 2, (9000, 9000, 9000)),
    ("fmm_423_20", 2, (16384, 16384, 2400)),
    ("fmm_333_23", 2, (4097, 1001, 30)),
    ("fmm_323_15", 1, (3, 2, 3)),
    ("fmm_424_26", 1, (5, 3, 9)),
])
def test_planner_peel_and_leaves(name, L, shape):
    m, k, n = shape
    a = algorithms.get(name)
    p = F.Plan(name, m, k, n, L, host_only=True)
    i = p.info
    fm, fk, fn = a.M ** L, a.K ** L, a.N ** L
    assert (i["m0"], i["k0"], i["n0"]) == (m // fm * fm, k // fk * fk, n // fn * fn)
    assert (i["leaf_m"], i["leaf_k"], i["leaf_n"]) == (m // fm, k // fk, n // fn)
    assert i["num_leaves"] == a.R ** L
    peels = (i["k0"] < k) + (i["n0"] < n) + (i["m0"] < m)
    assert i["num_gemm_problems"] == a.R ** L + peels
    # leaf flops: R^L leaf products plus the classical peel products
    lm, lk, ln = i["leaf_m"], i["leaf_k"], i["leaf_n"]
    m0, k0, n0 = i["m0"], i["k0"], i["n0"]
    expect = 2 * lm * lk * ln * a.R ** L + 2 * m0 * (k - k0) * n0 + 2 * m0 * k * (n - n0) \
        + 2 * (m - m0) * k * n
    assert i["leaf_flops"] == pytest.approx(expect, rel=1e-12)
    assert i["classical_flops"] == 2.0 * m * k * n


def _single(X, r):
    return sum(1 for v in X[:, r] if v) == 1


@pytest.mark.parametrize("name", ["strassen_222_7", "fmm_333_23", "fmm_424_26"])
@pytest.mark.parametrize("L", [1, 2])
@pytest.mark.parametrize("fuse", ["1", "2"])
def test_single_nonzero_columns_become_views(name, L, fuse, monkeypatch):
    """Leaf operands whose U (V) columns have one non-zero at every level are
    scaled views of A (B) (Section 3.1: no temporary for such columns).  With
    all levels formed in one pass every other leaf operand is written to the
    workspace; with one level per pass, an operand whose deeper levels are
    single-non-zero is a scaled view of an intermediate instead."""
    monkeypatch.setenv("FMM_FUSE", fuse)
    M, K, N, R, U, V, W = F.algorithm_coeffs(name)
    p = F.Plan(name, M ** L * 8, K ** L * 8, N ** L * 8, L, host_only=True)
    info = p.info
    for side, X, loc_in in ((0, U, F.LOC_A), (1, V, F.LOC_B)):
        views = ws_views = 0
        for leaf in range(R ** L):
            digits = [(leaf // R ** (L - 1 - j)) % R for j in range(L)]
            loc, off, row, col, ld, alpha = p.operand(side, leaf)
            if all(_single(X, d) for d in digits):
                assert loc == loc_in
                views += 1
                coef = np.prod([X[:, d][X[:, d] != 0][0] for d in digits])
                assert alpha == coef
            else:
                assert loc == F.LOC_WORKSPACE
                if L == 2 and fuse == "1" and _single(X, digits[1]):
                    ws_views += 1
                    assert alpha == X[:, digits[1]][X[:, digits[1]] != 0][0]
                else:
                    assert alpha == 1.0
        nmat = info["num_s_materialized"] if side == 0 else info["num_t_materialized"]
        assert nmat == R ** L - views - ws_views
    for leaf in range(R ** L):
        assert p.operand(2, leaf)[0] == F.LOC_WORKSPACE


def test_strassen_view_positions():
    """S_3 = A11 and S_4 = A22 (Section 2.1) are views at the right blocks."""
    p = F.Plan("strassen_222_7", 64, 64, 64, 1, host_only=True)
    assert p.operand(0, 2)[:4] == (F.LOC_A, 0, 0, 0)
    assert p.operand(0, 3)[:4] == (F.LOC_A, 0, 32, 32)
    # T_2 = B11, T_5 = B22
    assert p.operand(1, 1)[:4] == (F.LOC_B, 0, 0, 0)
    assert p.operand(1, 4)[:4] == (F.LOC_B, 0, 32, 32)


def test_workspace_and_addition_bytes_model():
    """Strassen, one level, 512^3 FP64: five S and five T blocks of 256x256 are
    written (two columns of U and of V have one non-zero), seven products of
    256x256; the streaming byte count is reads of A, B and the 7 products plus
    writes of the 10 formed operands and of C.  Workspace rows of 2 KB or more
    carry a 128-byte pad (a 256-wide FP64 block is stored with 272 columns)."""
    p = F.Plan("strassen_222_7", 512, 512, 512, 1, host_only=True)
    i = p.info
    blk = 256 * 256 * 8
    padded = 256 * (256 + 16) * 8
    assert i["num_s_materialized"] == 5 and i["num_t_materialized"] == 5
    assert i["workspace_bytes"] >= (5 + 5 + 7) * padded
    assert i["workspace_bytes"] < (5 + 5 + 7) * padded + 64 * 1024
    reads = 4 * blk + 4 * blk + 7 * blk
    writes = 5 * blk + 5 * blk + 4 * blk
    assert i["add_bytes"] == reads + writes


def test_workspace_row_padding():
    """FP64 workspace operands whose rows span 2 KB or more are stored 16
    elements wider (no power-of-two row stride across a leaf tile); narrower
    FP64 rows and FP32 rows keep the 16-element rounding only; views into A
    and B keep the caller's leading dimension."""
    with F.Plan("strassen_222_7", 512, 512, 512, 1, host_only=True) as p:
        ld_ws = {p.operand(0, r)[4] for r in range(7) if p.operand(0, r)[0] == F.LOC_WORKSPACE}
        ld_view = {p.operand(0, r)[4] for r in range(7) if p.operand(0, r)[0] == F.LOC_A}
        assert ld_ws == {256 + 16} and ld_view == {0}
    with F.Plan("strassen_222_7", 256, 256, 256, 1, host_only=True) as p:
        assert {p.operand(1, r)[4] for r in range(7) if p.operand(1, r)[0] == F.LOC_WORKSPACE} == {128}
    with F.Plan("strassen_222_7", 512, 512, 512, 1, F.F32, host_only=True) as p:
        assert {p.operand(0, r)[4] for r in range(7) if p.operand(0, r)[0] == F.LOC_WORKSPACE} == {256}


def test_zero_sizes_are_valid():
    for (m, k, n) in [(0, 5, 5), (5, 0, 5), (5, 5, 0), (0, 0, 0)]:
        p = F.Plan("strassen_222_7", m, k, n, 2, host_only=True)
        assert p.info["levels"] == 0


def test_host_only_plan_cannot_run():
    p = F.Plan("strassen_222_7", 64, 64, 64, 1, host_only=True)
    lib = ctypes.CDLL(F.library_path())
    lib.fmm_multiply.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p, ctypes.c_int64] * 3 + [ctypes.c_void_p]
    lib.fmm_multiply.restype = ctypes.c_int
    assert lib.fmm_multiply(p._p, 1, 64, 2, 64, 3, 64, None) == 1


@pytest.mark.parametrize("name,L", [("strassen_222_7", 1), ("strassen_222_7", 2), ("fmm_424_26", 2)])
def test_bf16x3_leaf_operands_are_split_not_viewed(name, L):
    """On the BF16x3 path every leaf operand is written as hi / lo bfloat16
    planes (4 bytes per element, like the FP32 value it replaces): no views of
    A or B, S planes row-major with rows padded to 8, T planes in k-octets."""
    a = algorithms.get(name)
    m, k, n = a.M ** L * 40, a.K ** L * 33, a.N ** L * 24
    p = F.Plan(name, m, k, n, L, dtype=F.F32_BF16X3, host_only=True)
    i = p.info
    assert i["num_s_materialized"] == a.R ** L and i["num_t_materialized"] == a.R ** L
    for leaf in range(a.R ** L):
        loc, off, row, col, ld, alpha = p.operand(0, leaf)
        assert loc == F.LOC_WORKSPACE and ld == 40 and alpha == 1.0  # round_up(33, 8)
        loc, off, row, col, ld, alpha = p.operand(1, leaf)
        assert loc == F.LOC_WORKSPACE and ld == 8 * 24 and alpha == 1.0
    # the plain FP32 path keeps its views
    q = F.Plan(name, m, k, n, L, dtype=F.F32, host_only=True).info
    assert q["num_s_materialized"] < a.R ** L


def test_argument_errors_before_any_device_call():
    """Entry points reject bad arguments with FMM_EINVAL (1) before touching a
    device; NULL handles are accepted where the header says so."""
    lib = F._lib
    vp = ctypes.c_void_p
    # batched multiply: zero requests is a no-op, a negative count an error
    assert lib.fmm_multiply_batched(None, None, None, None, None, None, None, 0, None) == 0
    assert lib.fmm_multiply_batched(None, None, None, None, None, None, None, -1, None) == 1
    # binding memory to a plan that was not made with defer_device_memory
    p = F.Plan("strassen_222_7", 64, 64, 64, 1, host_only=True)
    assert lib.fmm_plan_bind(p._p, vp(1 << 20), 1 << 30, None) == 1
    assert lib.fmm_plan_device_bytes(None) == 0
    # ranking: negative capacity is an error, zero capacity returns nothing
    cnt = ctypes.c_int(-1)
    assert lib.fmm_rank_candidates(64, 64, 64, 0, None, 0, 0.0, None, -1, ctypes.byref(cnt)) == 1
    assert lib.fmm_rank_candidates(64, 64, 64, 0, None, 0, 0.0, None, 0, ctypes.byref(cnt)) == 0 and cnt.value == 0
    # server options
    srv = vp()
    zero3 = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    for batch, inflight, streams, large in ((0, 2, 1, 0.0), (65, 2, 1, 0.0), (8, 0, 1, 0.0), (8, 2, 5, 0.0),
                                            (8, 2, -1, 0.0), (8, 2, 3, -1.0)):
        opts = F._ServerOptions(1 << 20, batch, inflight, 0, 0, zero3, streams, large)
        assert lib.fmm_server_create(ctypes.byref(srv), ctypes.byref(opts), None) == 1
    assert lib.fmm_server_arena_bytes(None) == 0
    assert lib.fmm_server_create(ctypes.byref(srv), None, None) == 1
    assert lib.fmm_server_submit(None, None, None) == 1
    n = ctypes.c_int(-1)
    assert lib.fmm_server_progress(None, 0, None, 0, ctypes.byref(n)) == 1 and n.value == 0
    assert lib.fmm_server_pending(None) == 0
    assert lib.fmm_server_destroy(None) == 0
    # recorded choices must name a valid plan
    from paper_1409_2908_amd import autotune
    for args in ((-1, 8, 8, 0, "strassen_222_7", 1, 0), (64, 64, 64, 0, "strassen_222_7", 1, 3),
                 (64, 64, 64, 5, "strassen_222_7", 1, 0), (64, 64, 64, 0, "strassen_222_7", -1, 0)):
        with pytest.raises(F.FmmError) as e:
            autotune.record(*args)
        assert e.value.code == 1


def test_leaf_form_choice_and_limits():
    """One-level FP64 / FP32 plans of Strassen-type base cases form their leaf
    operands inside the leaf GEMM when asked (never by default); deeper,
    BF16x3 and wide-column plans cannot, and asking for it there is an
    error."""
    with F.Plan("strassen_222_7", 512, 512, 512, 1, F.F64, host_only=True) as p:
        assert p.info["leaf_form"] == 0
    with F.Plan("strassen_222_7", 512, 512, 512, 1, F.F64, host_only=True, leaf_form=2) as p:
        assert p.info["leaf_form"] == 2
    with F.Plan("strassen_222_7", 512, 512, 512, 1, F.F64, host_only=True, leaf_form=1) as p:
        assert p.info["leaf_form"] == 0
    with F.Plan("fmm_333_23", 600, 600, 600, 1, F.F32, host_only=True) as p:
        assert p.info["leaf_form"] == 0  # columns of up to 7 non-zeros
    with pytest.raises(F.FmmError):
        F.Plan("fmm_333_23", 600, 600, 600, 1, F.F32, host_only=True, leaf_form=2)
    with F.Plan("strassen_222_7", 8192, 8192, 8192, 1, F.F64, host_only=True) as p:
        assert p.info["leaf_form"] == 0
    with F.Plan("strassen_222_7", 8192, 8192, 8192, 1, F.F64, host_only=True, leaf_form=2) as p:
        assert p.info["leaf_form"] == 2
    for args in (("strassen_222_7", 512, 512, 512, 2, F.F64), ("strassen_222_7", 512, 512, 512, 1, F.F32_BF16X3)):
        with F.Plan(*args, host_only=True) as p:
            assert p.info["leaf_form"] == 0
        with pytest.raises(F.FmmError):
            F.Plan(*args, host_only=True, leaf_form=2)
    with pytest.raises(F.FmmError):
        F.Plan("strassen_222_7", 512, 512, 512, 1, F.F64, host_only=True, leaf_form=3)
