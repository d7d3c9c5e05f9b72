"""Host sanitizers on the CPU (no GPU): the C oracle under AddressSanitizer
with UndefinedBehaviorSanitizer and, separately, ThreadSanitizer (its
stages, conversions and quotient run on POSIX threads); the library's
host-side ABI paths (argument checks, schedule registration and resolution,
size queries) under AddressSanitizer and UndefinedBehaviorSanitizer from
four threads.  Each driver exits non-zero on a failed check and the
sanitizers abort on the first report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r.stdout


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_c_oracle_under_sanitizers(tmp_path, san):
    exe = str(tmp_path / "orc")
    _run(["gcc", "-O1", "-g", "-std=c11", f"-fsanitize={san}", "-fno-sanitize-recover=all", "-pthread",
          os.path.join(ROOT, "oracle", "ntt_oracle.c"), os.path.join(NATIVE, "oracle_sanitize.c"), "-o", exe])
    out = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", TSAN_OPTIONS="halt_on_error=1"))
    assert "ok" in out


def test_abi_host_paths_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang++"
    build = os.path.join(ROOT, "paper_2509_22684_amd", "_build")
    if not (os.path.exists(hipcc) and os.path.exists(clang) and os.path.isdir(build)):
        pytest.skip("needs hipcc, the ROCm clang and the library's objects (python -m paper_2509_22684_amd.build)")
    objs = sorted(os.path.join(build, f) for f in os.listdir(build) if f.endswith(".o") and f != "api.cpp.o")
    api = str(tmp_path / "api.o")
    _run([hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2509_22684_amd", "csrc"),
          "-x", "hip", "-c", os.path.join(ROOT, "paper_2509_22684_amd", "csrc", "api.cpp"), "-o", api])
    drv = str(tmp_path / "driver.o")
    _run([clang, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-I", os.path.join(ROOT, "include"),
          "-c", os.path.join(NATIVE, "abi_sanitize.cpp"), "-o", drv])
    exe = str(tmp_path / "abi")
    _run([hipcc, "--offload-arch=gfx950", "-fsanitize=address,undefined", "-fno-gpu-sanitize", drv, api, *objs,
          "-o", exe, "-pthread"])
    out = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0",
                               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1"))
    assert "ok" in out
