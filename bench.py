"""Benchmark: recursive fast matrix multiplication on one MI355X.

One step = one fmm_multiply over the whole hot path (operand formation, the
grouped leaf GEMM launch, the W-combination) of a synthetic FP64 square
product with inputs resident in HBM.  Default workload: 16384^3 FP64,
uniform[-1,1) operands, the base case and depth given by --alg/--levels.

Prints one JSON line with the effective rate 2mkn/t, the same-GPU classical
GEMM rate, the leaf GEMM's roofline figures (live HIP events on the launch
stream), the error on sampled rows against the CPU oracle, and the oracle's
own rate on those rows as the CPU baseline.

--mode serving replays a Poisson request stream through the serving runtime;
--mode sweep prints timing tables of the other workloads (one JSON line each).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix peak
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def traffic_from_profile(kernel_tag):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if
    its kernel source hash matches the current source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
        import hashlib
        src = os.path.join(ROOT, rec["source"])
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if h != rec.get("source_sha256"):
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=16384, help="m = k = n")
    ap.add_argument("--alg", default="fmm_424_26")
    ap.add_argument("--levels", type=int, default=2)
    ap.add_argument("--fuse", type=int, default=0, help="levels per addition pass (0 = library default)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB device copy first (reference dispatch for HBM counters)")
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32", "bf16x3"],
                    help="f64: uniform[-1,1) FP64 operands; f32 / bf16x3: FP32 normal(0,1) operands with 10%% "
                         "of the rows of A and B scaled by 1e3, plain FP32 or BF16x3 leaves")
    ap.add_argument("--cpu-rows", type=int, default=384,
                    help="rows of the oracle CPU baseline sample (about 10 s of CPU work at 16384)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="multiply", choices=["multiply", "serving", "sweep"],
                    help="multiply: the one-line hot-path benchmark (default); serving: the request "
                         "stream; sweep: timing tables of the square, rectangular and BF16x3 shapes")
    ap.add_argument("--requests", type=int, default=10000, help="serving: stream length")
    ap.add_argument("--load", type=float, default=0.8, help="serving: offered load / measured capacity")
    ap.add_argument("--arena-gb", type=float, default=0.0,
                    help="serving: workspace arena (GB; 0 = the device's free memory less a reserve)")
    ap.add_argument("--streams", type=int, default=3, help="serving: server streams (1-4)")
    ap.add_argument("--large-gflop", type=float, default=0.0,
                    help="serving: 2mkn (GFLOP) from which a request is large (0: the library default)")
    ap.add_argument("--max-batch", type=int, default=8)
    ap.add_argument("--max-inflight", type=int, default=2)
    ap.add_argument("--sweep", default="square", choices=["square", "rect", "bf16x3", "latency"])
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on exactly one GPU; the fast-multiplication hot path is "
              "measured per GPU (--gpus 1).  Multi-GPU sharding is design-only.", file=sys.stderr)
        sys.exit(2)

    import torch
    import fmm_inputs
    import paper_1409_2908_amd as F

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.mode == "serving":
        return run_serving(args)
    if args.mode == "sweep":
        return run_sweep(args)
    n = args.n
    m = k = n
    dt = {"f64": F.F64, "f32": F.F32, "bf16x3": F.F32_BF16X3}[args.dtype]
    elt = torch.float64 if dt == F.F64 else torch.float32
    if dt == F.F64:
        log(f"[bench] generating {m}x{k} and {k}x{n} FP64 operands")
        A, B = fmm_inputs.operands(0, m, k, n, "uniform")
    else:
        log(f"[bench] generating {m}x{k} and {k}x{n} FP32 operands (row-scaled normal)")
        A, B = fmm_inputs.operands(0, m, k, n, "normal_rowscaled", np.float32)
    dA = torch.from_numpy(A).to(dev)
    dB = torch.from_numpy(B).to(dev)
    dC = torch.empty((m, n), dtype=elt, device=dev)
    stream = torch.cuda.current_stream()

    if args.calibrate_copy:
        # a plain copy of exactly 2^30 bytes: reads 1 GiB, writes 1 GiB
        src = torch.ones(2 ** 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    plan = F.Plan(args.alg, m, k, n, args.levels, dt, fuse_levels=args.fuse)
    info = plan.info
    log(f"[bench] plan {args.alg} L={args.levels}: leaf {info['leaf_m']}x{info['leaf_k']}x{info['leaf_n']}"
        f" x{info['num_leaves']}, workspace {info['workspace_bytes'] / 2**30:.2f} GiB")

    for _ in range(args.warmup):
        plan.multiply(dA, dB, dC)
    torch.cuda.synchronize()

    plan.enable_timing(max(args.steps, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.multiply(dA, dB, dC)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage_ms = plan.stage_ms()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    eff_tflops = 2.0 * m * k * n / (ms_per_step * 1e-3) / 1e12
    log(f"[bench] fast: {ms_per_step:.3f} ms/step, {eff_tflops:.2f} effective TFLOP/s, stages {stage_ms}")

    # same-GPU classical baseline: the same MFMA kernel on the one full problem
    def classical_rate(gdt):
        for _ in range(2):
            F.gemm(dA, dB, dC, dtype=gdt)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        csteps = max(3, min(args.steps, 5))
        ev0.record(stream)
        for _ in range(csteps):
            F.gemm(dA, dB, dC, dtype=gdt)
        ev1.record(stream)
        torch.cuda.synchronize()
        cms = ev0.elapsed_time(ev1) / csteps
        return cms, 2.0 * m * k * n / (cms * 1e-3) / 1e12

    classical_ms, classical_tflops = classical_rate(dt)
    log(f"[bench] classical MFMA GEMM: {classical_ms:.3f} ms, {classical_tflops:.2f} TFLOP/s")
    plain_fp32 = None
    if dt == F.F32_BF16X3:
        plain_fp32 = round(classical_rate(F.F32)[1], 3)
        log(f"[bench] plain FP32 classical MFMA GEMM: {plain_fp32} TFLOP/s")

    # the vendor BLAS on the same GPU (torch.matmul: rocBLAS / hipBLASLt),
    # called only, in the operands' own precision
    def vendor_rate():
        for _ in range(2):
            torch.matmul(dA, dB, out=dC)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        vsteps = max(3, min(args.steps, 5))
        ev0.record(stream)
        for _ in range(vsteps):
            torch.matmul(dA, dB, out=dC)
        ev1.record(stream)
        torch.cuda.synchronize()
        return 2.0 * m * k * n / (ev0.elapsed_time(ev1) / vsteps * 1e-3) / 1e12

    vendor_tflops = vendor_rate()
    log(f"[bench] vendor GEMM (torch.matmul, {'FP64' if dt == F.F64 else 'FP32'}): {vendor_tflops:.2f} TFLOP/s")

    # error on sampled rows + CPU baseline (the oracle on those rows)
    plan.multiply(dA, dB, dC)
    torch.cuda.synchronize()
    err = err_max_row = err_unscaled = None
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import classical as oracle_classical
        a = F.algorithm_coeffs(args.alg) if args.alg != "classical" else (1, 1, 1)
        h = m // (a[0] ** args.levels)
        must = [0, m - 1] + [b * h for b in range(a[0] ** args.levels)]
        rows = fmm_inputs.sample_rows(1, m, args.cpu_rows, must)
        got = dC[torch.from_numpy(rows).to(dev)].cpu().numpy()
        tc0 = time.perf_counter()
        ref = oracle_classical.gemm_rows(A, B, rows)
        tc1 = time.perf_counter()
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        # the worst single row, and (row-scaled inputs) the rows of C whose
        # row of A was not scaled, which the scaled rows' magnitude would
        # otherwise hide in the Frobenius norm
        row_err = np.linalg.norm(got - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
        err_max_row = float(row_err.max())
        if dt != F.F64:
            unscaled = ~np.isin(rows, fmm_inputs.scaled_rows(0, m, "A"))
            err_unscaled = float(np.linalg.norm(got[unscaled] - ref[unscaled]) / np.linalg.norm(ref[unscaled]))
        cpu_flops = 2.0 * len(rows) * k * n
        cpu = {"value": cpu_flops / (tc1 - tc0) / 1e12, "unit": "TFLOP/s",
               "cores": oracle_classical.num_threads(), "kind": "oracle",
               "sample": f"{len(rows)} rows of the {m}x{k}x{n} product ({cpu_flops / 1e9:.1f} GFLOP, "
                         f"{tc1 - tc0:.1f} s)"}
        log(f"[bench] sampled-row relF {err:.3e}; oracle {cpu['value'] * 1e3:.2f} GFLOP/s on {cpu['cores']} threads")

    leaf_ms = stage_ms[F.STAGE_LEAF]
    leaf_tflops = info["leaf_flops"] / (leaf_ms * 1e-3) / 1e12
    # the leaf launch's tile edge (the library's per-launch rule for FP64 /
    # FP32: 32 when there are at most half as many 64 x 64 tiles as compute
    # units, 64 for launches that form their operands or have fewer 128 x 128
    # tiles than units, else 128) and operand term slots (leaf_form)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    t128, rem = info["gemm_tiles"], info["gemm_tiles"] % (2 * cus)
    t64 = -(-info["leaf_m"] // 64) * -(-info["leaf_n"] // 64) * max(info["num_leaves"], 1)
    nt = info["leaf_form"]
    if 2 * t64 <= cus:
        tile = 32
    elif nt or t128 < cus or (t128 < 4 * cus and 0 < rem <= cus):
        tile = 64
    else:
        tile = 128
    e = 2 if dt == F.F64 else 4
    dma = (dt in (F.F64, F.F32) and tile == 128 and not nt and info["leaf_k"] % e == 0 and
           info["leaf_n"] % e == 0 and info["m0"] == m and info["k0"] == k and info["n0"] == n)
    if dma:
        # operands staged by direct loads (the library's rule: 16-byte aligned
        # rows, leading dimensions, K and N multiples of 16 bytes / element)
        if dt == F.F64:
            kernel, peak, tag = "gemm_f64_dma_kernel", FP64_PEAK_TFLOPS, "gemm_f64dma_t128"
        else:
            kernel, peak, tag = "gemm_f32_dma_kernel", FP32_PEAK_TFLOPS, "gemm_f32dma_t128"
    elif dt == F.F64:
        kernel, peak, tag = f"gemm_kernel<double, {tile}, {tile}, {nt}>", FP64_PEAK_TFLOPS, f"gemm_f64_t{tile}"
    elif dt == F.F32:
        kernel, peak, tag = f"gemm_kernel<float, {tile}, {tile}, {nt}>", FP32_PEAK_TFLOPS, f"gemm_f32_t{tile}"
    else:
        # three bf16 products per FP32 product, priced at the bf16 matrix peak;
        # the library's per-launch rule: split leaf operands with whole
        # k-octets run 256 x 256 tiles when there are two per compute unit
        leaf_k_octets = info["leaf_k"] % 8 == 0 and info["levels"] > 0
        t256 = -(-info["leaf_m"] // 256) * -(-info["leaf_n"] // 256) * info["num_leaves"]
        if leaf_k_octets and t256 >= 2 * cus:
            kernel, tag = "gemm_bf16x3_big_kernel", "gemm_bf16x3_t256"
        else:
            tile = 64 if t128 < cus else 128
            kernel, tag = f"gemm_bf16x3_kernel<{tile}>", f"gemm_bf16x3_t{tile}"
        peak = BF16_PEAK_TFLOPS
        leaf_tflops *= 3
    traffic = traffic_from_profile(tag)
    workload = (f"FP64 square {m}x{k}x{n}, uniform[-1,1)" if dt == F.F64 else
                f"FP32 square {m}x{k}x{n}, normal(0,1) with 10% of rows of A and B x1e3, "
                f"{'BF16x3' if dt == F.F32_BF16X3 else 'plain FP32'} leaves")
    out = {
        "metric": "effective TFLOP/s (2mkn/t) vs classical GEMM at fixed error; p50/p99 latency",
        "value": round(eff_tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"{workload}, {args.alg} at {args.levels} levels",
                   "m": m, "k": k, "n": n, "alg": args.alg, "levels": args.levels,
                   "fuse_levels": info["fuse_levels"]},
        "classical_same_gpu_tflops": round(classical_tflops, 3),
        "classical_plain_fp32_tflops": plain_fp32,
        "vendor_gemm_tflops": round(vendor_tflops, 3),
        "speedup_vs_classical": round(eff_tflops / classical_tflops, 4),
        "speedup_vs_vendor": round(eff_tflops / vendor_tflops, 4),
        "error_relF_sampled_rows": err,
        "error_max_row_relF": err_max_row,
        "error_relF_unscaled_rows": err_unscaled,
        "stage_ms": {"form_s": stage_ms[0], "form_t": stage_ms[1], "leaf_gemm": stage_ms[2],
                     "combine": stage_ms[3]},
        "roofline": {"bound": "mfma", "kernel": kernel,
                     "achieved": round(leaf_tflops, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(leaf_tflops / peak, 4), "traffic": traffic},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.close()


def oracle_check_kept(F, kept, rows_per_request=8, seed=500):
    """The kept served requests against the CPU oracle on sampled rows (first,
    last and seeded rows of each product): FP64 within 1e-12, BF16x3 within
    its error gate (oracle.bf16x3.gate for the request's plan).  Returns the
    largest error and the largest error / gate per dtype; raises if one is
    above its gate."""
    import torch
    import fmm_inputs
    from oracle import algorithms, bf16x3, classical
    worst = {}
    for idx, r in sorted(kept.items()):
        c = r["completion"]
        m, k = r["A"].shape
        rows = fmm_inputs.sample_rows(seed + idx, m, rows_per_request, [0, m - 1])
        ri = torch.from_numpy(rows).to(r["A"].device)
        Ar = r["A"][ri].double().cpu().numpy()
        got = r["C"][ri].double().cpu().numpy()
        ref = classical.gemm_rows(Ar, r["B"].double().cpu().numpy(), np.arange(len(rows)))
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        if r["dtype"] == F.F64:
            tol, name = 1e-12, "f64"
        else:
            names = c["alg"].split("+")
            algs = None if c["levels"] == 0 or c["alg"] == "classical" else (
                [algorithms.get(x) for x in names] if len(names) > 1 else algorithms.get(names[0]))
            tol, name = bf16x3.gate(algs, c["levels"], k), "bf16x3"
        if err > tol:
            raise AssertionError(f"request {idx} ({c['alg']} L={c['levels']}): relF {err:.3e} above {tol:.3e}")
        w = worst.setdefault(name, {"max_relF": 0.0, "max_relF_over_gate": 0.0, "checked": 0})
        w["max_relF"] = max(w["max_relF"], err)
        w["max_relF_over_gate"] = max(w["max_relF_over_gate"], err / tol)
        w["checked"] += 1
    return worst


def run_serving(args):
    """Config: a Poisson stream of FP64 / FP32 (BF16x3) requests, each of m, k, n
    log-uniform on [256, 8192].  Capacity is measured first with every request
    arriving at once; the stream then arrives at `load` x that capacity.  The
    same arrivals are served one at a time by the classical GEMM (FIFO, no
    batching) for comparison.  A seeded subset of the served requests is
    recomputed alone and must match the result from the mix bit for bit."""
    import torch
    import paper_1409_2908_amd as F
    from paper_1409_2908_amd import serving

    reqs = serving.make_requests(7, args.requests)
    log(f"[serving] {len(reqs)} requests; pools on device")
    pools = serving.Pools(8192 + 4096, seed=3)
    arena = int(args.arena_gb * 1e9)
    zeros = np.zeros(len(reqs))
    common = dict(arena_bytes=arena, max_batch=args.max_batch, max_inflight=args.max_inflight,
                  num_streams=args.streams, large_flops=args.large_gflop * 1e9)
    cap_fast, _ = serving.run_stream(reqs, zeros, pools, **common)
    log(f"[serving] capacity, fast path: {cap_fast}")
    cap_all, _ = serving.run_stream(reqs, zeros, pools, small_model=True, **common)
    log(f"[serving] capacity, the model's plan for small requests too: {cap_all}")
    cap_cl, _ = serving.run_stream(reqs, zeros, pools, arena_bytes=arena, max_batch=1, max_inflight=1,
                                   alg="classical", levels=0)
    log(f"[serving] capacity, one-at-a-time classical: {cap_cl}")
    rate = args.load * cap_fast["req_per_s"]
    arr = serving.poisson_arrivals(11, len(reqs), rate)
    keep = set(int(x) for x in np.random.default_rng(13).choice(len(reqs), min(200, len(reqs)), replace=False))
    fast, kept = serving.run_stream(reqs, arr, pools, keep=keep, **common)
    log(f"[serving] Poisson at {rate:.1f} req/s, fast path: {fast}")
    one = dict(common, num_streams=1)
    fast1, _ = serving.run_stream(reqs, arr, pools, **one)
    log(f"[serving] Poisson at {rate:.1f} req/s, fast path on one stream: {fast1}")
    cl, _ = serving.run_stream(reqs, arr, pools, arena_bytes=arena, max_batch=1, max_inflight=1,
                               alg="classical", levels=0)
    log(f"[serving] Poisson at {rate:.1f} req/s, one-at-a-time classical: {cl}")
    checked = serving.check_alone(kept)
    log(f"[serving] {checked} requests recomputed alone: bitwise equal")
    oracle_errors = oracle_check_kept(F, kept)
    log(f"[serving] {checked} requests against the CPU oracle on sampled rows: {oracle_errors}")
    cap_graph, _ = serving.run_stream(reqs, zeros, pools, use_graph=True, **common)
    log(f"[serving] capacity, fast path, one HIP graph per batch: {cap_graph}")
    fast_graph, kept_g = serving.run_stream(reqs, arr, pools, keep=keep, use_graph=True, **common)
    log(f"[serving] Poisson at {rate:.1f} req/s, fast path, one HIP graph per batch: {fast_graph}")
    checked_g = serving.check_alone(kept_g)
    log(f"[serving] {checked_g} graph-served requests recomputed alone: bitwise equal")
    out = {
        "metric": "serving throughput (requests/s, effective TFLOP/s) and p50/p99 latency",
        "value": round(fast["req_per_s"], 3), "unit": "requests/s", "n_gpus": 1,
        "higher_is_better": True, "data": "synthetic", "dtype": "f64+f32(bf16x3)",
        "config": {"workload": f"{len(reqs)} requests, m,k,n log-uniform [256,8192], FP64/FP32 1:1, "
                               f"Poisson at {args.load} x capacity", "arena_gb": fast["arena_gb"],
                   "streams": args.streams, "max_batch": args.max_batch, "max_inflight": args.max_inflight},
        "offered_req_per_s": round(rate, 3),
        "fast": fast, "fast_one_stream": fast1, "classical_one_at_a_time": cl,
        "capacity_fast": cap_fast, "capacity_classical": cap_cl, "capacity_model_for_small_requests": cap_all,
        "fast_graph": fast_graph, "capacity_fast_graph": cap_graph,
        "alone_vs_mix_checked": checked, "alone_vs_mix_checked_graph": checked_g,
        "oracle_sampled_rows": oracle_errors,
    }
    print(json.dumps(out), flush=True)


def run_sweep(args):
    """Timing tables (one JSON line per shape and candidate): the square FP64
    shapes with every base case at 1-3 levels, the rectangular FP64 shapes with
    the autotuner's pick, or FP32 BF16x3 Strassen at 1-3 levels against plain
    FP32.  Errors per depth come from the GPU tests, which alone use the
    oracle."""
    import torch
    import paper_1409_2908_amd as F
    from paper_1409_2908_amd import autotune

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def operands(m, k, n, elt):
        g = torch.Generator(device="cuda").manual_seed(0)
        A = torch.rand((m, k), dtype=elt, device="cuda", generator=g) * 2 - 1
        B = torch.rand((k, n), dtype=elt, device="cuda", generator=g) * 2 - 1
        return A, B, torch.empty((m, n), dtype=elt, device="cuda")

    def emit(rec):
        print(json.dumps(rec), flush=True)

    if args.sweep == "square":
        for n in (4096, 8192, 16384):
            A, B, C = operands(n, n, n, torch.float64)
            fl = 2.0 * n ** 3
            cms = timed(lambda: F.gemm(A, B, C))
            emit({"shape": [n, n, n], "alg": "classical", "levels": 0, "ms": cms, "tflops": fl / cms / 1e9})
            for alg in ("strassen_222_7", "winograd_222_7", "fmm_333_23", "fmm_323_15", "fmm_424_26", "fmm_334_29"):
                for L in (1, 2, 3):
                    try:
                        p = F.Plan(alg, n, n, n, L, F.F64)
                    except F.FmmError as e:
                        emit({"shape": [n, n, n], "alg": alg, "levels": L, "error": str(e)})
                        continue
                    ms = timed(lambda: p.multiply(A, B, C))
                    emit({"shape": [n, n, n], "alg": alg, "levels": L, "ms": ms, "tflops": fl / ms / 1e9,
                          "speedup": cms / ms, "workspace_gib": p.workspace_bytes / 2 ** 30})
                    p.close()
            del A, B, C
            torch.cuda.empty_cache()
    elif args.sweep == "rect":
        for (m, k, n) in ((16384, 1600, 16384), (16384, 16384, 2400), (9000, 9000, 9000)):
            A, B, C = operands(m, k, n, torch.float64)
            fl = 2.0 * m * k * n
            cms = timed(lambda: F.gemm(A, B, C))
            t = autotune.tune(m, k, n, F.F64, top=6)
            emit({"shape": [m, k, n], "classical_ms": cms, "classical_tflops": fl / cms / 1e9,
                  "tuned": {x: t[x] for x in ("alg", "levels", "fuse_levels", "leaf_tile", "ms", "tflops")},
                  "speedup": cms / t["ms"], "model_top": F.rank_candidates(m, k, n, F.F64)[0],
                  "candidates": [{x: c.get(x) for x in ("alg", "levels", "fuse_levels", "leaf_tile", "model_ms", "ms")}
                                 for c in t["candidates"]]})
            del A, B, C
            torch.cuda.empty_cache()
    elif args.sweep == "latency":
        # config 1: 512^3 FP64 Strassen one level is launch-bound; per-call wall
        # latency (enqueue + completion), eager vs graph replay vs classical
        n = 512
        A, B, C = operands(n, n, n, torch.float64)

        def lat(fn, reps=300):
            for _ in range(20):
                fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
            ts.sort()
            return {"p50_ms": ts[len(ts) // 2], "p99_ms": ts[int(len(ts) * 0.99)], "min_ms": ts[0]}

        emit({"shape": [n, n, n], "alg": "classical", "levels": 0, **lat(lambda: F.gemm(A, B, C))})
        for leaf_form in (1, 2):  # formation passes, or inside the leaf GEMM (the default here)
            for graph in (False, True):
                p = F.Plan("strassen_222_7", n, n, n, 1, F.F64, use_graph=graph, leaf_form=leaf_form)
                emit({"shape": [n, n, n], "alg": "strassen_222_7", "levels": 1, "graph": graph,
                      "leaf_form": p.info["leaf_form"], **lat(lambda: p.multiply(A, B, C))})
                p.close()
    else:
        for n in (8192, 16384):
            A, B, C = operands(n, n, n, torch.float32)
            fl = 2.0 * n ** 3
            for dt, name in ((F.F32, "fp32"), (F.F32_BF16X3, "bf16x3")):
                cms = timed(lambda: F.gemm(A, B, C, dtype=dt))
                emit({"shape": [n, n, n], "path": name, "alg": "classical", "levels": 0, "ms": cms,
                      "tflops": fl / cms / 1e9})
                for L in (1, 2, 3):
                    p = F.Plan("strassen_222_7", n, n, n, L, dt)
                    ms = timed(lambda: p.multiply(A, B, C))
                    emit({"shape": [n, n, n], "path": name, "alg": "strassen_222_7", "levels": L, "ms": ms,
                          "tflops": fl / ms / 1e9, "speedup_vs_same_path_classical": cms / ms})
                    p.close()
            del A, B, C
            torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
