"""Build the HIP library libfmm.so in-tree for gfx950 (MI355X).

Steps: regenerate csrc/fmm_tables.h and the per-base-case kernel sources
(csrc/gen/) from the base-case tables, compile every source with hipcc in
parallel, link one shared library next to this file.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfmm.so")
SOURCES = ["fmm_api.cpp", "fmm_plan.cpp", "fmm_tune.cpp", "fmm_serve.cpp", "fmm_add.hip", "fmm_gemm.hip",
           "fmm_gemm_bf16x3.hip", "fmm_gemm_f64dma.hip", "fmm_gemm_f32dma.hip"]
# plus one generated source per base case (csrc/gen/fmm_add_NN.hip), listed by gen_tables.generate()
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result", "-I" + os.path.join(HERE, "..", "include")]


def _compile(src, verbose):
    obj = os.path.join(BUILD, src.replace("/", "_") + ".o")
    # The addition kernels (csrc/gen/) round every multiply and add of a chain
    # separately, as the oracle's chains do: a contracted multiply-add differs
    # in the last bit once a coefficient or a view's scale is not 0 or +-2^e.
    extra = ["-ffp-contract=off"] if src.startswith("gen/") else []
    cmd = [HIPCC] + FLAGS + extra + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{out}")
    if verbose and out.strip():
        print(out)
    return obj


def build(verbose=False):
    # load the generator by path: importing the package would load the
    # (possibly stale) library this call is about to replace
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "fmm_gen_tables", os.path.join(HERE, "algorithms", "gen_tables.py"))
    gen_tables = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen_tables)
    _, generated = gen_tables.generate()
    sources = SOURCES + generated
    os.makedirs(BUILD, exist_ok=True)
    # the longest compiles (generated kernels of the widest base cases) first
    sources.sort(key=lambda s: (not s.startswith("gen/"), s), reverse=False)
    with cf.ThreadPoolExecutor(max_workers=min(os.cpu_count() or 8, 16)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), sources))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
