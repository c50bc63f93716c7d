"""Host-side sanitizer runs (CPU only): the oracle and the C-ABI layer built
with AddressSanitizer and UndefinedBehaviorSanitizer and driven by the small C
programs in tests/sanitize/.  A report from either sanitizer, or a check that
fails, fails the test.  The device code is built as usual; only host code is
instrumented."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
CLANGXX = "/opt/rocm/llvm/bin/clang++"


def run_checked(cmd, env=None, timeout=300):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, "%s failed (%d):\n%s%s" % (cmd[0], r.returncode, r.stdout, r.stderr)
    for bad in ("AddressSanitizer", "runtime error:", "LeakSanitizer"):
        assert bad not in r.stderr, r.stderr
    return r


def test_oracle_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_check")
    run_checked(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off",
                 "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer", os.path.join(SAN, "oracle_check.c"),
                 os.path.join(ROOT, "oracle", "jacobi_oracle.c"), "-lm", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
    r = run_checked([exe], env=env)
    assert "oracle sanitize check: ok" in r.stdout


def _clang_rt_dir():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return os.path.dirname(hits[-1]) if hits else None


def test_c_abi_host_layer_under_asan_and_ubsan(tmp_path):
    objs = sorted(glob.glob(os.path.join(ROOT, "_build", "*.o")))
    others = [o for o in objs if os.path.basename(o) != "jacobi_abi.o"]
    rt = _clang_rt_dir()
    if not os.path.exists(HIPCC) or not os.path.exists(CLANG) or rt is None:
        pytest.skip("ROCm clang toolchain or its sanitizer runtime not available")
    if len(others) < 10:
        pytest.skip("library objects not built (run paper_2303_02543_amd/build.py)")
    abi_o = str(tmp_path / "jacobi_abi_san.o")
    # host code instrumented, device code as in the product build
    run_checked([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                 "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
                 "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-c",
                 os.path.join(ROOT, "paper_2303_02543_amd", "csrc", "jacobi_abi.hip"), "-o", abi_o])
    lib = str(tmp_path / "libjacobi_san.so")
    run_checked([CLANGXX, "-shared", "-fPIC", "-fsanitize=address", "-fsanitize=undefined",
                 "-shared-libsan", "-o", lib, abi_o] + others +
                ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    exe = str(tmp_path / "abi_check")
    run_checked([CLANG, "-O1", "-g", "-fsanitize=address", "-fsanitize=undefined",
                 "-fno-sanitize-recover=all", "-shared-libsan", "-I", os.path.join(ROOT, "include"),
                 os.path.join(SAN, "abi_check.c"), "-o", exe, "-L", str(tmp_path), "-ljacobi_san",
                 "-Wl,-rpath," + str(tmp_path), "-Wl,-rpath," + rt])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    r = run_checked([exe], env=env)
    assert "abi sanitize check: ok" in r.stdout
