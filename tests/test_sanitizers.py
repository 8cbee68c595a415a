"""CPU runs under AddressSanitizer and UndefinedBehaviorSanitizer:

* the oracle's own tests (tests/test_oracle_*.py) against a sanitized build of
  oracle/tv_oracle.c (gcc, libasan preloaded into the test process);
* the host side of the C ABI: a host-only build of the library (device code is
  a stub, so no kernel can launch) driven by tests/sanitize/abi_host_check.c,
  which makes only host queries and calls with argument errors.

Both abort on the first memory or undefined-behaviour error.  Skipped where the
compilers are missing."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = os.environ.get("CLANG", "/opt/rocm/llvm/bin/clang")


def _env(**kw):
    env = dict(os.environ)
    env.update(ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.update(kw)
    return env


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_tests_under_asan_ubsan():
    sys.path.insert(0, ROOT)
    import oracle
    lib = oracle.build(force=True, sanitize=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    assert os.path.isabs(asan) and os.path.exists(asan), asan
    tests = sorted(os.path.join(ROOT, "tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_") and f.endswith(".py"))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + tests,
                       cwd=ROOT, env=_env(LD_PRELOAD=asan, ORACLE_LIBRARY=lib), capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "passed" in r.stdout


@pytest.mark.skipif(not (os.path.exists("/opt/rocm/bin/hipcc") and os.path.exists(CLANG)),
                    reason="hipcc or clang missing")
def test_host_abi_under_asan_ubsan():
    from paper_1502_07770_amd import build_lib
    lib = build_lib.build_host_sanitized()
    rt = os.path.dirname(subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                        capture_output=True, text=True).stdout.strip())
    exe = os.path.join(build_lib.SAN, "abi_host_check")
    cmd = [CLANG, "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-shared-libsan", "-g",
           "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "sanitize", "abi_host_check.c"), "-L" + build_lib.SAN, "-ltvchain_san",
           "-Wl,-rpath," + build_lib.SAN, "-Wl,-rpath," + rt, "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], env=_env(), capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "host ABI checks passed" in r.stdout
    assert os.path.exists(lib)


@pytest.mark.skipif(not (os.path.exists("/opt/rocm/bin/hipcc") and os.path.exists(CLANG)),
                    reason="hipcc or clang missing")
def test_nc_lane_bodies_under_asan_ubsan():
    """The non-convex lane kernels' per-chain bodies on the CPU with every array
    a separate exactly-sized heap block (tests/sanitize/nc_host_check.hip)."""
    from paper_1502_07770_amd import build_lib
    exe = build_lib.build_host_check(os.path.join(ROOT, "tests", "sanitize", "nc_host_check.hip"))
    r = subprocess.run([exe], env=_env(), capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "nc lane checks passed" in r.stdout
