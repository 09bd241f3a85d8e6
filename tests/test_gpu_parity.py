"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (relative Frobenius error against the classical binary64 oracle):
  FP64: 1e-12 for every algorithm and depth (a rounding-error analysis of
        L fast levels grows the bound by a small constant per level over the
        classical k*u; measured errors are ~1e-15).
  FP32: 2e-6 * 2^L (binary32 leaves, FP64 additions).
Integer-valued inputs ({-8..8}) are exact in every path and must match the
oracle bit for bit.  Stage kernels are bit-exact against the oracle's chains
in the same (ascending, level-by-level) order.
"""
import os

import numpy as np
import pytest

import fmm_inputs
from oracle import algorithms, classical, recursive
from gpu_util import relf, say, to_dev, to_host, ws_read, ws_write

pytestmark = pytest.mark.gpu

ALGS = ["strassen_222_7", "fmm_333_23", "fmm_323_15", "fmm_423_20", "fmm_424_26"]


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    import paper_1409_2908_amd as lib
    return lib


def _shape(alg, L, t=(3, 2, 3), r=(1, 1, 1)):
    a = algorithms.get(alg)
    return a.M ** L * t[0] + r[0], a.K ** L * t[1] + r[1], a.N ** L * t[2] + r[2]


def _run(F, alg, L, A, B, dtype):
    m, k = A.shape
    n = B.shape[1]
    with F.Plan(alg, m, k, n, L, dtype) as p:
        C = p.multiply(to_dev(A), to_dev(B))
        return to_host(C)


@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("L", [1, 2])
def test_fp64_parity_ragged(F, alg, L):
    a = algorithms.get(alg)
    # leaf blocks spanning several 128 x 128 tiles (L = 1) and ragged peels
    lm, lk, ln = (130, 150, 140) if L == 1 else (40, 50, 35)
    fm, fk, fn = a.M ** L, a.K ** L, a.N ** L
    m, k, n = fm * lm + fm - 1, fk * lk + 1, fn * ln + fn - 1
    say(f"case fp64 {alg} L={L} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(1, m, k, n, "uniform")
    C = _run(F, alg, L, A, B, F.F64)
    ref = classical.gemm(A, B)
    err = relf(C, ref)
    say(f"  relF={err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("L", [1, 2])
def test_integer_inputs_bit_exact(F, alg, L):
    m, k, n = _shape(alg, L, (5, 7, 6), (1, 2, 1))
    say(f"case int {alg} L={L} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(2, m, k, n, "integer")
    ref = classical.gemm(A, B)
    C = _run(F, alg, L, A, B, F.F64)
    assert np.array_equal(C, ref)
    C32 = _run(F, alg, L, A.astype(np.float32), B.astype(np.float32), F.F32)
    assert np.array_equal(C32.astype(np.float64), ref)


def test_config1_strassen_512(F):
    """Strassen, one level, 512^3 FP64: uniform inputs on five seeds within
    1e-12, integer inputs bit-exact."""
    for seed in range(5):
        A, B = fmm_inputs.operands(seed, 512, 512, 512, "uniform")
        C = _run(F, "strassen_222_7", 1, A, B, F.F64)
        err = relf(C, classical.gemm(A, B))
        say(f"config1 seed {seed} relF={err:.3e}")
        assert err <= 1e-12
    A, B = fmm_inputs.operands(0, 512, 512, 512, "integer")
    assert np.array_equal(_run(F, "strassen_222_7", 1, A, B, F.F64), classical.gemm(A, B))


@pytest.mark.parametrize("alg,L", [("strassen_222_7", 3), ("fmm_323_15", 3), ("fmm_424_26", 2)])
def test_fp64_deep_parity(F, alg, L):
    m, k, n = _shape(alg, L, (6, 5, 4), (3, 0, 2))
    say(f"case deep {alg} L={L} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(3, m, k, n, "uniform")
    C = _run(F, alg, L, A, B, F.F64)
    err = relf(C, classical.gemm(A, B))
    say(f"  relF={err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("alg", ["strassen_222_7", "fmm_424_26", "fmm_333_23"])
@pytest.mark.parametrize("L", [0, 1, 2])
def test_fp32_parity(F, alg, L):
    m, k, n = _shape(alg, L, (9, 8, 7), (1, 3, 2)) if L else (333, 444, 255)
    say(f"case fp32 {alg} L={L} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(4, m, k, n, "uniform", np.float32)
    C = _run(F, alg if L else "classical", L, A, B, F.F32)
    err = relf(C, classical.gemm(A, B))
    say(f"  relF={err:.3e}")
    assert err <= 2e-6 * 2 ** L


@pytest.mark.parametrize("alg,L", [("strassen_222_7", 2), ("strassen_222_7", 3), ("fmm_424_26", 2),
                                   ("fmm_333_23", 2), ("fmm_323_15", 3), ("fmm_423_20", 2)])
def test_fused_levels_bitwise_equal_unfused(F, alg, L, monkeypatch):
    """Forming two levels per pass is the same arithmetic in the same order as
    one level per pass, so the products agree bit for bit."""
    m, k, n = _shape(alg, L, (4, 3, 5), (1, 1, 1))
    say(f"case fuse {alg} L={L} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(5, m, k, n, "uniform")
    out = {}
    for fuse in ("1", "2"):
        monkeypatch.setenv("FMM_FUSE", fuse)
        out[fuse] = _run(F, alg, L, A, B, F.F64)
    assert np.array_equal(out["1"].view(np.int64), out["2"].view(np.int64))


def _leaf_operand(F, p, side, leaf, A, B, dtype):
    loc, off, row, col, ld, alpha = p.operand(side, leaf)
    return loc, off, row, col, ld, alpha


@pytest.mark.parametrize("alg,L,fuse,mult", [("strassen_222_7", 1, "1", 1), ("strassen_222_7", 2, "2", 1),
                                             ("strassen_222_7", 3, "2", 1), ("fmm_424_26", 2, "1", 1),
                                             ("fmm_333_23", 2, "2", 1), ("fmm_423_20", 1, "1", 1),
                                             ("strassen_222_7", 1, "1", 8), ("strassen_222_7", 2, "2", 8),
                                             ("fmm_424_26", 2, "1", 8), ("fmm_333_23", 1, "1", 8)])
def test_operand_formation_bit_exact(F, alg, L, fuse, mult, monkeypatch):
    """Every leaf operand S_rho, T_rho produced by the formation kernels equals
    the oracle's chain (ascending index, level by level) bit for bit; views
    equal alpha times the viewed block.  mult = 8 makes every block width a
    multiple of 4 with 16-byte aligned rows (the coarsened kernels)."""
    monkeypatch.setenv("FMM_FUSE", fuse)
    a = algorithms.get(alg)
    m, k, n = a.M ** L * 5 * mult, a.K ** L * 4 * mult, a.N ** L * 6 * mult
    say(f"case form {alg} L={L} fuse={fuse} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(6, m, k, n, "uniform")
    S = recursive.form_operands(a, L, A, "A")
    T = recursive.form_operands(a, L, B, "B")
    with F.Plan(alg, m, k, n, L, F.F64) as p:
        info = p.info
        dA, dB = to_dev(A), to_dev(B)
        C = p.run_stage(F.STAGE_FORM_S, dA, dB)
        p.run_stage(F.STAGE_FORM_T, dA, dB, C)
        lm, lk, ln = info["leaf_m"], info["leaf_k"], info["leaf_n"]
        for side, X, ref, (h, w) in ((0, A, S, (lm, lk)), (1, B, T, (lk, ln))):
            for leaf in range(a.R ** L):
                loc, off, row, col, ld, alpha = p.operand(side, leaf)
                if loc == F.LOC_WORKSPACE:
                    got = ws_read(p, off, h, w, ld, np.float64) * alpha
                else:
                    got = X[row:row + h, col:col + w] * alpha
                assert np.array_equal(got.view(np.int64), ref[leaf].view(np.int64)), (side, leaf)


@pytest.mark.parametrize("alg,L,shape,dtype_name", [
    ("fmm_424_26", 2, (592, 524, 2064), "F64"),     # leaf widths 131 (S) and 129 (T): odd, past one workgroup
    ("fmm_424_26", 2, (640, 512, 2048), "F64"),     # even widths 128 (S, T): every pair stored at once
    ("fmm_423_20", 2, (400, 260, 873), "F64"),      # leaf widths 65 and 97
    ("strassen_222_7", 2, (520, 1036, 772), "F32"),  # FP32 outputs, two positions per thread: widths 259, 193
    ("strassen_222_7", 1, (518, 1030, 774), "F32"),  # one level: widths 515, 387
    ("strassen_222_7", 2, (520, 1032, 776), "F32"),  # even widths 258, 194: 8-byte pair loads and stores
    ("strassen_222_7", 1, (518, 1028, 772), "F32"),  # even widths 514, 386
])
def test_two_position_formation_bit_exact(F, alg, L, shape, dtype_name, monkeypatch):
    """The formation kernels that give a lane or thread two adjacent positions
    (the two-level LDS pass of base cases with at most 8 blocks per side, and
    the register pass for FP32 outputs) on widths that are odd, a multiple
    of the workgroup's 128 positions, or past it (FP32 with even widths: the
    aligned-pair path): every leaf operand equals the oracle's chain bit for
    bit (FP32 outputs: the binary64 chain rounded once to binary32)."""
    monkeypatch.setenv("FMM_FUSE", str(L))
    a = algorithms.get(alg)
    m, k, n = shape
    np_dt = np.float64 if dtype_name == "F64" else np.float32
    say(f"case two-position form {alg} L={L} {dtype_name} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(7, m, k, n, "uniform", np_dt)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    fm, fk, fn = a.M ** L, a.K ** L, a.N ** L
    assert m % fm == 0 and k % fk == 0 and n % fn == 0
    S = recursive.form_operands(a, L, A64, "A")
    T = recursive.form_operands(a, L, B64, "B")
    with F.Plan(alg, m, k, n, L, getattr(F, dtype_name)) as p:
        info = p.info
        dA, dB = to_dev(A), to_dev(B)
        C = p.run_stage(F.STAGE_FORM_S, dA, dB)
        p.run_stage(F.STAGE_FORM_T, dA, dB, C)
        lm, lk, ln = info["leaf_m"], info["leaf_k"], info["leaf_n"]
        iv = np.int64 if dtype_name == "F64" else np.int32
        for side, X, ref, (h, w) in ((0, A, S, (lm, lk)), (1, B, T, (lk, ln))):
            for leaf in range(a.R ** L):
                loc, off, row, col, ld, alpha = p.operand(side, leaf)
                if loc != F.LOC_WORKSPACE:
                    continue
                got = ws_read(p, off, h, w, ld, np_dt) * np_dt(alpha)
                want = ref[leaf].astype(np_dt)
                assert np.array_equal(got.view(iv), want.view(iv)), (side, leaf)


@pytest.mark.parametrize("alg,L,fuse", [("strassen_222_7", 1, "1"), ("strassen_222_7", 2, "2"),
                                        ("fmm_424_26", 2, "2"), ("fmm_424_26", 2, "1"),
                                        ("fmm_333_23", 1, "1"), ("strassen_222_7", 3, "2")])
def test_combination_bit_exact(F, alg, L, fuse, monkeypatch):
    """The W-combination of seeded leaf products equals the oracle's
    deepest-level-first chains bit for bit."""
    monkeypatch.setenv("FMM_FUSE", fuse)
    a = algorithms.get(alg)
    m, k, n = a.M ** L * 3, a.K ** L * 2, a.N ** L * 5
    say(f"case combine {alg} L={L} fuse={fuse} m={m} k={k} n={n}")
    with F.Plan(alg, m, k, n, L, F.F64) as p:
        info = p.info
        lm, ln = info["leaf_m"], info["leaf_n"]
        Ms = []
        for leaf in range(a.R ** L):
            Mv = fmm_inputs.matrix(100 + leaf, 7, lm, ln, "uniform")
            Ms.append(Mv)
            loc, off, row, col, ld, alpha = p.operand(2, leaf)
            assert loc == F.LOC_WORKSPACE
            ws_write(p, off, Mv, ld)
        import torch
        dA = torch.zeros((m, k), dtype=torch.float64, device="cuda")
        dB = torch.zeros((k, n), dtype=torch.float64, device="cuda")
        C = p.run_stage(F.STAGE_COMBINE, dA, dB)
        got = to_host(C)
    ref = recursive.combine_products(a, L, Ms)
    assert np.array_equal(got.view(np.int64), ref.view(np.int64))


@pytest.mark.parametrize("alg,dtype_name,shape", [
    ("strassen_222_7", "F32", (148, 20, 264)),         # leaf width 66: aligned pairs, one partial workgroup
    ("strassen_222_7", "F32", (92, 20, 1032)),         # width 258: several workgroups and a partial one
    ("strassen_222_7", "F32", (148, 20, 260)),         # width 65: odd, the LDS kernel
    ("strassen_222_7", "F32_BF16X3", (148, 20, 1032)),
    ("winograd_222_7", "F32", (100, 20, 520)),
    ("classical_222_8", "F32", (60, 20, 264)),
])
def test_fp32_combination_bit_exact(F, alg, dtype_name, shape, monkeypatch):
    """Two fused levels of the W-combination of seeded FP32 leaf products (the
    register kernel for aligned pairs, the LDS kernel otherwise) equal the
    oracle's binary64 chains rounded once to binary32, bit for bit."""
    monkeypatch.setenv("FMM_FUSE", "2")
    a = algorithms.get(alg)
    m, k, n = shape
    say(f"case fp32 combine {alg} {dtype_name} m={m} k={k} n={n}")
    with F.Plan(alg, m, k, n, 2, getattr(F, dtype_name)) as p:
        info = p.info
        lm, ln = info["leaf_m"], info["leaf_n"]
        assert (lm * a.M ** 2, ln * a.N ** 2) == (m, n)
        Ms = []
        for leaf in range(a.R ** 2):
            Mv = fmm_inputs.matrix(400 + leaf, 7, lm, ln, "uniform").astype(np.float32)
            Ms.append(Mv.astype(np.float64))
            loc, off, row, col, ld, alpha = p.operand(2, leaf)
            assert loc == F.LOC_WORKSPACE
            ws_write(p, off, Mv, ld)
        import torch
        dA = torch.zeros((m, k), dtype=torch.float32, device="cuda")
        dB = torch.zeros((k, n), dtype=torch.float32, device="cuda")
        got = to_host(p.run_stage(F.STAGE_COMBINE, dA, dB))
    ref = recursive.combine_products(a, 2, Ms).astype(np.float32)
    assert got.dtype == np.float32
    assert np.array_equal(got.view(np.int32), ref.view(np.int32))


def test_classical_gemm_kernel(F):
    for (m, k, n) in [(1, 1, 1), (127, 129, 131), (300, 17, 513), (64, 1000, 64), (5, 3, 700)]:
        A, B = fmm_inputs.operands(7, m, k, n, "uniform")
        import torch
        C = to_host(F.gemm(to_dev(A), to_dev(B)))
        err = relf(C, classical.gemm(A, B))
        say(f"gemm {m}x{k}x{n} relF={err:.2e}")
        assert err <= 1e-14
        Ai, Bi = fmm_inputs.operands(7, m, k, n, "integer")
        assert np.array_equal(to_host(F.gemm(to_dev(Ai), to_dev(Bi))), classical.gemm(Ai, Bi))


def test_edge_cases(F):
    import torch
    # zero sizes
    for (m, k, n) in [(0, 4, 4), (4, 4, 0)]:
        with F.Plan("strassen_222_7", m, k, n, 1) as p:
            C = p.multiply(torch.zeros((m, k), dtype=torch.float64, device="cuda"),
                           torch.zeros((k, n), dtype=torch.float64, device="cuda"))
            assert C.shape == (m, n)
    with F.Plan("strassen_222_7", 5, 0, 6, 1) as p:
        C = torch.full((5, 6), 7.0, dtype=torch.float64, device="cuda")
        p.multiply(torch.zeros((5, 0), dtype=torch.float64, device="cuda"),
                   torch.zeros((0, 6), dtype=torch.float64, device="cuda"), C)
        assert to_host(C).tolist() == [[0.0] * 6] * 5
    # exactly the base case, one element per block
    A, B = fmm_inputs.operands(8, 2, 2, 2, "integer")
    assert np.array_equal(_run(F, "strassen_222_7", 1, A, B, F.F64), A @ B)
    A, B = fmm_inputs.operands(8, 4, 2, 4, "integer")
    assert np.array_equal(_run(F, "fmm_424_26", 1, A, B, F.F64), A @ B)
    # depth too large
    with pytest.raises(F.FmmError):
        F.Plan("strassen_222_7", 3, 16, 16, 2)
    # strided operands (leading dimensions larger than the column counts)
    m, k, n = 130, 66, 98
    A, B = fmm_inputs.operands(9, m, k, n, "uniform")
    bigA = torch.zeros((m, k + 7), dtype=torch.float64, device="cuda")
    bigB = torch.zeros((k, n + 5), dtype=torch.float64, device="cuda")
    bigC = torch.zeros((m, n + 3), dtype=torch.float64, device="cuda")
    bigA[:, :k] = to_dev(A)
    bigB[:, :n] = to_dev(B)
    with F.Plan("strassen_222_7", m, k, n, 1) as p:
        p.multiply(bigA[:, :k], bigB[:, :n], bigC[:, :n])
    assert relf(to_host(bigC)[:, :n], classical.gemm(A, B)) < 1e-14
    assert np.all(to_host(bigC)[:, n:] == 0)
    # C overlapping A is rejected
    with F.Plan("strassen_222_7", 8, 8, 8, 1) as p:
        X = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
        with pytest.raises(F.FmmError):
            p.multiply(X, torch.zeros((8, 8), dtype=torch.float64, device="cuda"), X)
    # wrong dtype
    with F.Plan("strassen_222_7", 8, 8, 8, 1) as p:
        with pytest.raises(TypeError):
            p.multiply(torch.zeros((8, 8), device="cuda"), torch.zeros((8, 8), device="cuda"))


def test_deterministic(F):
    A, B = fmm_inputs.operands(10, 1000, 1000, 1000, "uniform")
    with F.Plan("fmm_424_26", 1000, 1000, 1000, 2, F.F64) as p:
        dA, dB = to_dev(A), to_dev(B)
        c1 = to_host(p.multiply(dA, dB))
        c2 = to_host(p.multiply(dA, dB))
    assert np.array_equal(c1.view(np.int64), c2.view(np.int64))


def test_bench_configuration_sampled_rows(F):
    """The benchmark's own configuration (16384^3 FP64, the launch the
    benchmark times), checked on sampled rows including every block and peel
    boundary row against the oracle's row product."""
    import torch
    n = 16384
    alg, L = os.environ.get("FMM_BENCH_ALG", "fmm_424_26"), int(os.environ.get("FMM_BENCH_LEVELS", "2"))
    say(f"case bench-config {alg} L={L} n={n}")
    A, B = fmm_inputs.operands(0, n, n, n, "uniform")
    with F.Plan(alg, n, n, n, L, F.F64) as p:
        dA, dB = to_dev(A), to_dev(B)
        C = p.multiply(dA, dB)
        torch.cuda.synchronize()
        a = algorithms.get(alg)
        h = n // a.M ** L
        must = [0, n - 1] + [b * h for b in range(a.M ** L)] + [b * h - 1 for b in range(1, a.M ** L)]
        rows = fmm_inputs.sample_rows(1, n, 24, must)
        got = C[torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = classical.gemm_rows(A, B, rows)
    err = relf(got, ref)
    say(f"  sampled {len(rows)} rows relF={err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("dtype_name", ["F64", "F32"])
@pytest.mark.parametrize("alg,L,shape", [("classical", 0, (300, 211, 515)), ("classical", 0, (1, 1000, 129)),
                                         ("strassen_222_7", 1, (517, 260, 383)),
                                         ("fmm_424_26", 1, (1030, 777, 1029))])
def test_leaf_tile_shapes_agree(F, dtype_name, alg, L, shape):
    """The 64 x 64 and 128 x 128 leaf tiles accumulate every output element
    over the same K steps in the same order, so they agree bit for bit; both
    match the oracle (the FP64 and FP32 tolerances above)."""
    dtype = getattr(F, dtype_name)
    np_dt = np.float64 if dtype_name == "F64" else np.float32
    m, k, n = shape
    say(f"case leaf tiles {dtype_name} {alg} L={L} {m}x{k}x{n}")
    A, B = fmm_inputs.operands(17, m, k, n, "uniform", np_dt)
    out = {}
    for tile in (64, 128, 0):
        with F.Plan(alg, m, k, n, L, dtype, leaf_tile=tile) as p:
            out[tile] = to_host(p.multiply(to_dev(A), to_dev(B)))
    ref = classical.gemm(A, B)
    tol = 1e-12 if dtype_name == "F64" else 2e-6 * 2 ** L
    for tile in (64, 128):
        assert relf(out[tile], ref) <= tol, tile
    iv = np.int64 if dtype_name == "F64" else np.int32
    assert np.array_equal(out[64].view(iv), out[128].view(iv))
    assert np.array_equal(out[0].view(iv), out[64].view(iv))



@pytest.mark.parametrize("dtype_name,alg,L,shape", [
    ("F64", "classical", 0, (258, 1002, 390)),
    ("F64", "strassen_222_7", 1, (516, 1000, 772)),
    ("F64", "fmm_424_26", 1, (1032, 1004, 1032)),
    ("F32", "classical", 0, (260, 1004, 388)),
    ("F32", "strassen_222_7", 1, (520, 1000, 776)),
    ("F32", "fmm_424_26", 1, (1032, 1000, 1040)),
])
def test_direct_load_leaf_edges(F, dtype_name, alg, L, shape):
    """Shapes whose operands satisfy the direct-load kernels' alignment (FP64:
    even leading dimensions and K, N; FP32: multiples of 4, 16-byte rows), so
    leaf_tile 128 runs gemm_f64_dma_kernel / gemm_f32_dma_kernel, with partial
    128-row and 128-column tiles and a K tail that is not a multiple of the
    16-k step (10, 4, 6, 12, 4, 8 here).  The direct-load tiles must agree
    bit for bit with the register-staged 64 x 64 tiles and match the oracle."""
    dtype = getattr(F, dtype_name)
    np_dt = np.float64 if dtype_name == "F64" else np.float32
    m, k, n = shape
    say(f"case direct-load edges {dtype_name} {alg} L={L} {m}x{k}x{n}")
    A, B = fmm_inputs.operands(23, m, k, n, "uniform", np_dt)
    out = {}
    for tile in (128, 64, 0):
        with F.Plan(alg, m, k, n, L, dtype, leaf_tile=tile) as p:
            out[tile] = to_host(p.multiply(to_dev(A), to_dev(B)))
    ref = classical.gemm(A, B)
    tol = 1e-12 if dtype_name == "F64" else 2e-6 * 2 ** L
    assert relf(out[128], ref) <= tol
    iv = np.int64 if dtype_name == "F64" else np.int32
    assert np.array_equal(out[128].view(iv), out[64].view(iv))
    assert np.array_equal(out[0].view(iv), out[64].view(iv))
    Ai, Bi = fmm_inputs.operands(24, m, k, n, "integer", np_dt)
    with F.Plan(alg, m, k, n, L, dtype, leaf_tile=128) as p:
        Ci = to_host(p.multiply(to_dev(Ai), to_dev(Bi)))
    assert np.array_equal(Ci.astype(np.float64), classical.gemm(Ai.astype(np.float64), Bi.astype(np.float64)))


def test_fp64_error_per_depth(F):
    """The error of each square-configuration base case per depth at 4096^3
    (uniform inputs; 32 sampled rows, every top-level block boundary among
    them, against the oracle's row product), printed as a table and held to
    the FP64 gate."""
    import torch
    n = 4096
    A, B = fmm_inputs.operands(3, n, n, n, "uniform")
    dA, dB = to_dev(A), to_dev(B)
    rows = fmm_inputs.sample_rows(2, n, 32, [0, n - 1, n // 2, n // 3, n // 4, 3 * n // 4])
    ref = classical.gemm_rows(A, B, rows)
    sel = torch.from_numpy(rows).cuda()
    for alg in ("strassen_222_7", "fmm_333_23", "fmm_323_15", "fmm_424_26"):
        errs = []
        for L in (1, 2, 3):
            with F.Plan(alg, n, n, n, L, F.F64) as p:
                got = p.multiply(dA, dB)[sel].cpu().numpy()
            errs.append(relf(got, ref))
        say(f"error-per-depth {alg} n={n} L=1/2/3 relF " + " / ".join(f"{e:.2e}" for e in errs))
        assert max(errs) <= 1e-12, (alg, errs)


MIXED = [("fmm_424_26+strassen_222_7", ["fmm_424_26", "strassen_222_7"]),
         ("strassen_222_7+fmm_323_15", ["strassen_222_7", "fmm_323_15"]),
         ("fmm_333_23+fmm_423_20", ["fmm_333_23", "fmm_423_20"]),
         ("strassen_222_7+fmm_424_26+strassen_222_7", ["strassen_222_7", "fmm_424_26", "strassen_222_7"])]


@pytest.mark.parametrize("spec,names", MIXED)
def test_mixed_levels_parity(F, spec, names):
    """One base case per level (Section 5.2's composition): ragged sizes
    against the binary64 oracle (FP64 gate), integer inputs bit-exact."""
    algs = [algorithms.get(x) for x in names]
    L = len(algs)
    fm = int(np.prod([a.M for a in algs]))
    fk = int(np.prod([a.K for a in algs]))
    fn = int(np.prod([a.N for a in algs]))
    m, k, n = fm * 3 + 1, fk * 2 + 1, fn * 3 + 2
    say(f"case mixed {spec} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(23, m, k, n, "uniform")
    C = _run(F, spec, L, A, B, F.F64)
    err = relf(C, classical.gemm(A, B))
    say(f"  relF={err:.2e}")
    assert err <= 1e-12
    Ai, Bi = fmm_inputs.operands(23, m, k, n, "integer")
    assert np.array_equal(_run(F, spec, L, Ai, Bi, F.F64), classical.gemm(Ai, Bi))


@pytest.mark.parametrize("spec,names", MIXED[:2])
def test_mixed_levels_stages_bit_exact(F, spec, names):
    """Formation and combination of a mixed plan equal the oracle's per-level
    chains bit for bit (leaf operands, and C from seeded leaf products)."""
    algs = [algorithms.get(x) for x in names]
    L = len(algs)
    m = int(np.prod([a.M for a in algs])) * 3
    k = int(np.prod([a.K for a in algs])) * 2
    n = int(np.prod([a.N for a in algs])) * 3
    say(f"case mixed stages {spec} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(24, m, k, n, "uniform")
    S = recursive.form_operands(algs, L, A, "A")
    T = recursive.form_operands(algs, L, B, "B")
    with F.Plan(spec, m, k, n, L, F.F64) as p:
        info = p.info
        dA, dB = to_dev(A), to_dev(B)
        C = p.run_stage(F.STAGE_FORM_S, dA, dB)
        p.run_stage(F.STAGE_FORM_T, dA, dB, C)
        lm, lk, ln = info["leaf_m"], info["leaf_k"], info["leaf_n"]
        for side, X, ref, (h, w) in ((0, A, S, (lm, lk)), (1, B, T, (lk, ln))):
            for leaf in range(len(ref)):
                loc, off, row, col, ld, alpha = p.operand(side, leaf)
                if loc == F.LOC_WORKSPACE:
                    got = ws_read(p, off, h, w, ld, np.float64) * alpha
                else:
                    got = X[row:row + h, col:col + w] * alpha
                assert np.array_equal(got.view(np.int64), ref[leaf].view(np.int64)), (side, leaf)
        Ms = []
        for leaf in range(len(S)):
            Mv = fmm_inputs.matrix(300 + leaf, 7, lm, ln, "uniform")
            Ms.append(Mv)
            loc, off, row, col, ld, alpha = p.operand(2, leaf)
            ws_write(p, off, Mv, ld)
        C = p.run_stage(F.STAGE_COMBINE, dA, dB)
        got = to_host(C)
    ref = recursive.combine_products(algs, L, Ms)
    assert np.array_equal(got.view(np.int64), ref.view(np.int64))
