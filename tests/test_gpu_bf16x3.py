"""GPU parity of the FP32 paths: plain FP32 MFMA leaves and BF16x3 leaves.

Tolerances (relative Frobenius error):
  classical BF16x3 against the binary64 product: 2e-5.  Each operand keeps
          ~16 significant bits (2^-16 relative split error, the dropped lo*lo
          term is 2^-16 relative); FP32 accumulation adds ~2^-24 sqrt(k).
  classical BF16x3 against its emulation (same split, binary64 sums): 5e-6,
          which a dropped product term (~2^-9) or a truncating split exceeds.
  fast BF16x3 against the binary64 product: oracle.bf16x3.gate(alg, L, k) =
          e0 * g^L, e0 = 3 * 2^-16 + (2 + sqrt(k)) 2^-24 the per-term error
          bound of the split product and g the base case's root-mean-square
          error growth per level (1 for a classical step, 2 for Strassen, 5.6
          for <4,2,4>); the emulated fast algorithm stays within it by ~11x on
          these inputs (pinned on the CPU), a lost product term exceeds it.
  fast BF16x3 against the emulated fast algorithm (oracle.bf16x3.fmm: the
          same static peel, operands rounded once to FP32, emulated BF16x3
          leaves): 2e-6 * 2^L, the FP32 tolerance, as a second, tighter
          check: what remains is FP32 rounding of the operand sums and of the
          accumulation.
  plain FP32 against the binary64 product: 2e-6 * 2^L.
Integer inputs with small magnitude are exact in every path (bf16 holds
integers up to 256 exactly; FP32 sums stay below 2^24).
"""
import numpy as np
import pytest

import fmm_inputs
from oracle import algorithms, bf16x3, classical
from gpu_util import relf, say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    import paper_1409_2908_amd as lib
    return lib


def _run(F, alg, L, A, B, dtype):
    m, k = A.shape
    n = B.shape[1]
    with F.Plan(alg, m, k, n, L, dtype) as p:
        return to_host(p.multiply(to_dev(A), to_dev(B)))


@pytest.mark.parametrize("shape", [(256, 512, 384), (300, 333, 257), (129, 64, 1000), (1, 7, 5)])
def test_bf16x3_classical_matches_emulation(F, shape):
    m, k, n = shape
    say(f"case bf16x3 gemm {m}x{k}x{n}")
    A, B = fmm_inputs.operands(11, m, k, n, "uniform", np.float32)
    C = to_host(F.gemm(to_dev(A), to_dev(B), dtype=F.F32_BF16X3))
    emu = bf16x3.gemm(A, B)
    ref = classical.gemm(A, B)
    e_emu, e_ref = relf(C, emu), relf(C, ref)
    say(f"  vs emulation {e_emu:.2e}  vs fp64 {e_ref:.2e}")
    assert e_emu <= 5e-6
    assert e_ref <= 2e-5


@pytest.mark.parametrize("alg,L", [("classical", 0), ("strassen_222_7", 1), ("strassen_222_7", 2),
                                   ("fmm_424_26", 1), ("fmm_333_23", 1)])
def test_bf16x3_integer_bit_exact(F, alg, L):
    if alg == "classical":
        m, k, n = 200, 301, 150
    else:
        from oracle import algorithms
        a = algorithms.get(alg)
        m, k, n = a.M ** L * 9 + 1, a.K ** L * 7 + 1, a.N ** L * 8 + 2
    say(f"case bf16x3 int {alg} L={L} {m}x{k}x{n}")
    A, B = fmm_inputs.operands(12, m, k, n, "integer", np.float32)
    C = _run(F, alg, L, A, B, F.F32_BF16X3)
    assert np.array_equal(C.astype(np.float64), classical.gemm(A, B))


FAST_CASES = [(alg, L) for alg in ("strassen_222_7", "fmm_333_23", "fmm_323_15", "fmm_423_20", "fmm_424_26")
              for L in (1, 2)] + [("strassen_222_7", 3)]


@pytest.mark.parametrize("kind", ["normal_rowscaled", "uniform"])
@pytest.mark.parametrize("alg,L", FAST_CASES)
def test_bf16x3_fast_parity(F, alg, L, kind):
    a = algorithms.get(alg)
    m, k, n = a.M ** L * 40 + 3, a.K ** L * 35 + 1, a.N ** L * 30 + 2
    say(f"case bf16x3 {alg} L={L} {m}x{k}x{n} {kind}")
    A, B = fmm_inputs.operands(13, m, k, n, kind, np.float32)
    C = _run(F, alg, L, A, B, F.F32_BF16X3)
    ref = classical.gemm(A, B)
    err = relf(C, ref)
    gate = bf16x3.gate(a, L, k)
    # per-row view of the dynamic-range stress (reported)
    rows_s = fmm_inputs.scaled_rows(13, m, "A") if kind == "normal_rowscaled" else np.zeros(0, np.int64)
    unscaled = np.setdiff1d(np.arange(m), rows_s)
    row_err = np.linalg.norm(C - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
    emu = bf16x3.fmm(a, L, A, B)
    e_emu = relf(C, emu)
    say(f"  relF={err:.2e} gate={gate:.2e} (emulation {relf(emu, ref):.2e}) vs emulation {e_emu:.2e} "
        f"max row {row_err.max():.2e} unscaled-rows relF={relf(C[unscaled], ref[unscaled]):.2e}")
    assert err <= gate
    assert e_emu <= 2e-6 * 2 ** L
    C32 = _run(F, alg, L, A, B, F.F32)
    err32 = relf(C32, ref)
    say(f"  plain FP32 relF={err32:.2e}")
    assert err32 <= 2e-6 * 2 ** L


def test_bf16x3_views_and_peels(F):
    """Odd leaf k (element-wise A loads), single-non-zero views of A, peel strips."""
    m, k, n = 2 * 151 + 1, 2 * 149 + 1, 2 * 133 + 1
    A, B = fmm_inputs.operands(14, m, k, n, "uniform", np.float32)
    C = _run(F, "strassen_222_7", 1, A, B, F.F32_BF16X3)
    assert relf(C, classical.gemm(A, B)) <= 4e-5


def _bf16_bits(x32):
    return (np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)


@pytest.mark.parametrize("alg,L,kmul", [("strassen_222_7", 1, 9), ("strassen_222_7", 2, 9), ("fmm_424_26", 1, 9),
                                        ("fmm_333_23", 1, 9), ("fmm_423_20", 2, 9), ("strassen_222_7", 1, 16),
                                        ("strassen_222_7", 2, 12), ("fmm_424_26", 1, 20)])
def test_split_leaf_operands_bit_exact(F, alg, L, kmul):
    """On the BF16x3 path the formation kernels write every leaf operand as
    hi / lo bfloat16 planes: S row-major, T in k-octets (8 consecutive k of a
    column together).  Both planes must equal the split of the oracle's chain
    (binary64, ascending index, level by level) rounded once to FP32, bit for
    bit; leaf k = 9 exercises a partial octet, leaf k a multiple of 4 the
    coarsened S writer."""
    from oracle import recursive
    from gpu_util import ws_read
    a = algorithms.get(alg)
    m, k, n = a.M ** L * 5, a.K ** L * kmul, a.N ** L * 6
    say(f"case split operands {alg} L={L} {m}x{k}x{n}")
    A, B = fmm_inputs.operands(15, m, k, n, "normal_rowscaled", np.float32)
    S = recursive.form_operands(a, L, A.astype(np.float64), "A")
    T = recursive.form_operands(a, L, B.astype(np.float64), "B")
    with F.Plan(alg, m, k, n, L, F.F32_BF16X3) as p:
        info = p.info
        assert info["num_s_materialized"] == a.R ** L and info["num_t_materialized"] == a.R ** L
        dA, dB = to_dev(A), to_dev(B)
        C = p.run_stage(F.STAGE_FORM_S, dA, dB)
        p.run_stage(F.STAGE_FORM_T, dA, dB, C)
        lm, lk, ln = info["leaf_m"], info["leaf_k"], info["leaf_n"]
        for leaf in range(a.R ** L):
            loc, off, row, col, ld, alpha = p.operand(0, leaf)
            assert loc == F.LOC_WORKSPACE and alpha == 1.0 and ld % 8 == 0 and ld >= lk
            eh, el = bf16x3.split(S[leaf].astype(np.float32))
            hi = ws_read(p, off, lm, lk, ld, np.uint16)
            lo = ws_read(p, off + lm * ld, lm, lk, ld, np.uint16)
            bad_h = np.argwhere(hi != _bf16_bits(eh))
            bad_l = np.argwhere(lo != _bf16_bits(el))
            assert len(bad_h) == 0 and len(bad_l) == 0, (
                "S", leaf, len(bad_h), len(bad_l), bad_h[:4].tolist(), bad_l[:4].tolist(),
                S[leaf].flat[:3].tolist(), hi.flat[:3].tolist(), _bf16_bits(eh).flat[:3].tolist())
            loc, off, row, col, ld, alpha = p.operand(1, leaf)
            assert loc == F.LOC_WORKSPACE and alpha == 1.0 and ld == 8 * ln
            groups = (lk + 7) // 8
            th, tl = bf16x3.split(T[leaf].astype(np.float32))
            raw_h = ws_read(p, off, groups, ld, ld, np.uint16).reshape(groups, ln, 8)
            raw_l = ws_read(p, off + groups * ld, groups, ld, ld, np.uint16).reshape(groups, ln, 8)
            # element (kk, nn) of a plane is at group kk // 8, column nn, slot kk % 8
            got_h = raw_h.transpose(0, 2, 1).reshape(groups * 8, ln)[:lk]
            got_l = raw_l.transpose(0, 2, 1).reshape(groups * 8, ln)[:lk]
            assert np.array_equal(got_h, _bf16_bits(th)) and np.array_equal(got_l, _bf16_bits(tl)), ("T", leaf)


@pytest.mark.parametrize("alg,L", [("fmm_424_26", 2), ("fmm_333_23", 2), ("strassen_222_7", 2)])
@pytest.mark.parametrize("dtype_name", ["F32_BF16X3", "F32"])
def test_fp32_fused_levels_bitwise_equal_unfused(F, alg, L, dtype_name, monkeypatch):
    """With FP32 operands the operand sums and the W-combination are binary64
    chains rounded once to FP32 (and split once on the BF16x3 path), so two
    levels per pass -- the LDS kernels for wide base cases and the split-S
    outputs they write -- give the same bits as one level per pass."""
    dtype = getattr(F, dtype_name)
    a = algorithms.get(alg)
    m, k, n = a.M ** L * 5 + 1, a.K ** L * 7 + 2, a.N ** L * 3 + 1
    say(f"case fp32 fuse {dtype_name} {alg} L={L} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(21, m, k, n, "normal_rowscaled", np.float32)
    out = {}
    for fuse in ("1", "2"):
        monkeypatch.setenv("FMM_FUSE", fuse)
        out[fuse] = _run(F, alg, L, A, B, dtype)
    assert np.array_equal(out["1"].view(np.int32), out["2"].view(np.int32))


@pytest.mark.parametrize("alg,L,shape", [("classical", 0, (300, 211, 515)), ("classical", 0, (65, 1001, 130)),
                                         ("strassen_222_7", 1, (517, 262, 383)),
                                         ("fmm_424_26", 1, (1030, 778, 1029)),
                                         ("strassen_222_7", 1, (1030, 778, 1029)),
                                         ("strassen_222_7", 2, (2063, 1001, 2050))])
def test_bf16x3_leaf_tile_shapes_agree(F, alg, L, shape):
    """64 x 64, 128 x 128 and (split leaf operands) 256 x 256 BF16x3 tiles
    run the same three MFMA products over the same K steps, so they agree bit
    for bit (split leaf operands and FP32 operands split while staged, ragged
    tile edges, a partial last K step, peel strips); all match the emulation."""
    m, k, n = shape
    say(f"case bf16x3 leaf tiles {alg} L={L} {m}x{k}x{n}")
    A, B = fmm_inputs.operands(19, m, k, n, "normal_rowscaled", np.float32)
    out = {}
    for tile in (64, 128, 256, 0):
        with F.Plan(alg, m, k, n, L, F.F32_BF16X3, leaf_tile=tile) as p:
            out[tile] = to_host(p.multiply(to_dev(A), to_dev(B)))
    a = None if alg == "classical" else algorithms.get(alg)
    emu = bf16x3.gemm(A, B) if a is None else bf16x3.fmm(a, L, A, B)
    for tile in (64, 128, 256):
        assert relf(out[tile], emu) <= 2e-6 * 2 ** max(L, 1), tile
        assert np.array_equal(out[tile].view(np.int32), out[64].view(np.int32)), tile
    assert relf(out[0], classical.gemm(A, B)) <= bf16x3.gate(a, L, k) if a else 2e-5
    assert np.array_equal(out[0].view(np.int32), out[64].view(np.int32))


@pytest.mark.parametrize("spec,names", [("fmm_424_26+strassen_222_7", ["fmm_424_26", "strassen_222_7"]),
                                        ("strassen_222_7+fmm_333_23", ["strassen_222_7", "fmm_333_23"])])
@pytest.mark.parametrize("dtype_name", ["F32_BF16X3", "F32"])
def test_fp32_mixed_levels_parity(F, spec, names, dtype_name):
    """One base case per level on the FP32 paths: BF16x3 against the emulated
    mixed algorithm, plain FP32 against the binary64 product."""
    algs = [algorithms.get(x) for x in names]
    fm = int(np.prod([a.M for a in algs]))
    fk = int(np.prod([a.K for a in algs]))
    fn = int(np.prod([a.N for a in algs]))
    m, k, n = fm * 5 + 1, fk * 3 + 2, fn * 4 + 1
    say(f"case fp32 mixed {dtype_name} {spec} m={m} k={k} n={n}")
    A, B = fmm_inputs.operands(29, m, k, n, "normal_rowscaled", np.float32)
    C = _run(F, spec, 2, A, B, getattr(F, dtype_name))
    ref = classical.gemm(A, B)
    e_ref = relf(C, ref)
    if dtype_name == "F32_BF16X3":
        e = relf(C, bf16x3.fmm(algs, 2, A, B))
        say(f"  relF={e_ref:.2e} gate={bf16x3.gate(algs, 2, k):.2e} vs emulation {e:.2e}")
        assert e_ref <= bf16x3.gate(algs, 2, k)
    else:
        e = e_ref
        say(f"  relF={e:.2e}")
    assert e <= 2e-6 * 4
