"""Build libjacobi.so (HIP, gfx950) in-tree with hipcc.

Every source is compiled for gfx950 only, with IEEE-exact arithmetic:
  -ffp-contract=off                 no FMA contraction (fixed rounding order)
  -fno-gpu-flush-denormals-to-zero  FP32 subnormals kept
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                    no packed FP32 instructions
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libjacobi.so")
BUILD_DIR = os.path.join(ROOT, "_build")
ARCH = "gfx950"

SOURCES = ["jacobi_abi.hip", "k_layout.hip", "k_sweep.hip", "k_march2d.hip", "k_march3d.hip",
           "k_residual.hip", "k_batch.hip", "k_deep.hip"]
# k_march2d.hip is compiled once per temporal depth (its kernels) and once
# more for the depth dispatch; each entry: (source, object name, defines)
MARCH2D_DEPTHS = list(range(1, 9)) + [10, 11, 12, 13, 14, 16]
UNITS = ([(s, os.path.splitext(s)[0], []) for s in SOURCES] +
         [("k_march2d.hip", "k_march2d_d%d" % d, ["-DJAC_MARCH2D_DEPTH=%d" % d])
          for d in MARCH2D_DEPTHS])
HEADERS = ["jacobi_internal.h", "kernels.h", "device_util.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _compile(unit, verbose, incremental=False):
    src, name, defines = unit
    obj = os.path.join(BUILD_DIR, name + ".o")
    if incremental and os.path.exists(obj):
        deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in HEADERS]
        deps.append(os.path.join(ROOT, "include", "jacobi.h"))
        if all(os.path.getmtime(d) <= os.path.getmtime(obj) for d in deps):
            return obj
    cmd = [HIPCC] + FLAGS + defines + ["-I", os.path.join(ROOT, "include"), "-c",
                                       os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s%s" % (src, r.stdout, r.stderr))
    return obj


def build(verbose: bool = False, jobs: int = 8, incremental: bool = False) -> str:
    """Compile every HIP source for gfx950 and link libjacobi.so.  Rebuilds
    every object unless incremental (then only objects older than their
    source or a header)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        # the largest units first, so they do not end up last in the queue
        units = sorted(UNITS, key=lambda u: -int(u[1].rsplit("_d", 1)[-1])
                       if u[1].startswith("k_march2d_d") else 0)
        objs = list(ex.map(lambda u: _compile(u, verbose, incremental), units))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, f) for f in SOURCES + HEADERS]
    deps.append(os.path.join(ROOT, "include", "jacobi.h"))
    return any(os.path.getmtime(p) > t for p in deps)


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
