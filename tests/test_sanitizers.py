"""Host-side sanitizer runs (CPU only; GPU code is never built with them).

* The CPU oracle, built with AddressSanitizer and UndefinedBehaviorSanitizer
  together with tests/sanitize/oracle_driver.c, runs every exported routine
  on a small ragged batch.
* The C ABI's host code (cme_api.hip, sanitizers on its host pass only),
  linked with the library's other objects and tests/sanitize/abi_driver.cpp,
  runs every entry point through its argument validation; without a GPU a
  valid request ends at the device query.
Any sanitizer report aborts the driver (no recovery), so the test fails."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
BUILD = os.path.join(ROOT, "paper_1307_3428_amd", "_build")
ROCM = "/opt/rocm"
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-fcx-limited-range",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
          "-o", exe, os.path.join(ROOT, "oracle", "cme_oracle.c"),
          os.path.join(HERE, "oracle_driver.c"), "-lm"])
    r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout and "runtime error" not in r.stderr


def test_abi_host_validation_under_asan_and_ubsan(tmp_path):
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not available")
    others = [os.path.join(BUILD, f) for f in sorted(os.listdir(BUILD))
              if f.endswith(".o") and f != "cme_api.o"] if os.path.isdir(BUILD) else []
    if not others:
        pytest.skip("library objects not built (run __graft_entry__.build())")
    api = str(tmp_path / "cme_api_san.o")
    # sanitizers on the host pass only
    _run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
          "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1307_3428_amd", "csrc"),
          "-c", os.path.join(ROOT, "paper_1307_3428_amd", "csrc", "cme_api.hip"), "-o", api])
    drv = str(tmp_path / "abi_driver.o")
    _run([clang, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
          "-I", os.path.join(ROOT, "include"), "-c", os.path.join(HERE, "abi_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "abi_san")
    _run([clang, "-fsanitize=address,undefined", drv, api, *others,
          "-L", os.path.join(ROCM, "lib"), "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", exe])
    env = dict(SAN_ENV, HIP_VISIBLE_DEVICES="")  # host paths only, also on a GPU machine
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout and "runtime error" not in r.stderr
