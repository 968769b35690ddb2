"""Build the HIP library libdnqs.so (gfx950) in-tree, next to this file."""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdnqs.so")
SOURCES = ["dnqs_api.hip", "k_hamiltonian.hip", "k_network.hip", "k_energy.hip", "k_pt2.hip", "k_pt2_part.hip", "k_pt2_reduce.hip", "k_gemm_x3.hip", "k_batch.hip", "k_optim.hip", "k_outsplit.hip", "k_sort.hip", "k_pset.hip", "k_lanczos.hip", "k_modes.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _compile(src, obj):
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    subprocess.check_call(cmd)


def build(verbose: bool = True) -> str:
    """Compile every source and link libdnqs.so (always rebuilds)."""
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    t0 = time.time()
    from concurrent.futures import ThreadPoolExecutor
    jobs = []
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as pool:
        for src in SOURCES:
            obj = os.path.join(bdir, src.replace(".hip", ".o"))
            objs.append(obj)
            jobs.append(pool.submit(_compile, src, obj))
        for j in jobs:
            j.result()
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
