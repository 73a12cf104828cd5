"""Build the HIP library ``lib/libode_ensemble.so`` for gfx950 with hipcc.

Each model's kernels are a separate translation unit, compiled in parallel,
then linked with the C ABI into one shared library.  ``python -m
paper_1810_03931_amd.build`` (or ``build()``) always recompiles.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB_DIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIB_DIR, "libode_ensemble.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


# Per-translation-unit flags: LLVM's scheduler tuned for instruction-level
# parallelism instead of occupancy, where a sweep's end is set by waves that
# run alone on their SIMD.
#  * Keller-Miksis is bound by a few long serial chains.  The schedule uses
#    258 registers, so one wave per SIMD instead of two; lock-step throughput
#    drops from 45% to 34% of the FP64 peak, but the sweep runs ~20% faster
#    (22-26 s against 27-32 s).
#  * Duffing and the relief valve keep two waves per SIMD (239 and 228
#    registers for the swept kernels).  Once a planned sweep's shorter wave
#    ends, the longer one runs alone, and it runs faster with this schedule:
#    758-771 against 779-786 ms, and 2432-2438 against 2488-2498 ms.
#  * The Lyapunov kernel (one wave per SIMD) gains nothing: 436 against 437 ms.
_ILP = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]
TU_FLAGS = {
    "kernels_keller_miksis.hip": _ILP,
    "kernels_duffing.hip": _ILP,
    "kernels_relief_valve.hip": _ILP,
}


def _compile(src, verbose):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    extra = TU_FLAGS.get(os.path.basename(src), [])
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *FLAGS, *extra, "-x", "hip", "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(OBJ, exist_ok=True)
    os.makedirs(LIB_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
