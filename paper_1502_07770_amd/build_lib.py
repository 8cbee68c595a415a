"""Build libtvchain.so (HIP, gfx950) in-tree with hipcc.

Every ``*.hip`` file under ``csrc/`` is compiled for gfx950 with packed-FP32
instruction selection disabled (the files listed in PARTS once per part),
then linked into one shared library next to this file.  ``python -m paper_1502_07770_amd.build_lib`` runs it.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
ROOT = os.path.dirname(PKG)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libtvchain.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    "-I" + os.path.join(ROOT, "include"),
]


def _deps(src: str, seen=None) -> set:
    """The file and every local header it includes, transitively."""
    seen = set() if seen is None else seen
    if src in seen or not os.path.exists(src):
        return seen
    seen.add(src)
    with open(src) as fh:
        for line in fh:
            m = re.match(r'\s*#\s*include\s+"([^"]+)"', line)
            if m:
                for d in (os.path.dirname(src), CSRC, os.path.join(ROOT, "include")):
                    h = os.path.join(d, m.group(1))
                    if os.path.exists(h):
                        _deps(h, seen)
                        break
    return seen


# Sources compiled once per part (-DTVC_PART=k), each part instantiating a
# subset of their kernels, so the longest single compilation is shorter.
PARTS = {"chain_kernels.hip": 4, "tv2d_kernels.hip": 4, "tv2d_batched.hip": 2, "chain_l1.hip": 2}


def _units(srcs):
    """(source, part) pairs to compile; part 0 is a whole source."""
    out = []
    for f in srcs:
        n = PARTS.get(os.path.basename(f), 0)
        out += [(f, k) for k in range(1, n + 1)] if n else [(f, 0)]
    return out


def _compile(unit, incremental: bool = False) -> str:
    src, part = unit
    obj = os.path.join(BUILD, os.path.basename(src) + (".p%d" % part if part else "") + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if all(t > os.path.getmtime(d) for d in _deps(src)):
            return obj
    cmd = [HIPCC] + FLAGS + (["-DTVC_PART=%d" % part] if part else []) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (or, with incremental, those older than their
    object file or any header) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    units = _units(sorted(glob.glob(os.path.join(CSRC, "*.hip"))))
    # longest first: the split sources and the 2D ones dominate
    units.sort(key=lambda u: -os.path.getsize(u[0]) * (2 if u[1] == 0 else 1))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(units))) as ex:
        objs = list(ex.map(lambda u: _compile(u, incremental), units))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, file=sys.stderr)
    return LIB


# Host-only build with AddressSanitizer and UndefinedBehaviorSanitizer on the
# host code, for checking the C ABI's host side on a CPU.  Its device code is a
# one-kernel stub fatbinary, so none of the library's kernels can launch from it.
SAN = os.path.join(BUILD, "san")
SAN_LIB = os.path.join(SAN, "libtvchain_san.so")
SAN_HOST_FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"),
                  "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
# the link names only host objects (clang++, not hipcc)
SAN_LINK = [os.environ.get("CLANGXX", "/opt/rocm/llvm/bin/clang++"), "-shared", "-shared-libsan",
            "-fsanitize=address,undefined"]


def build_host_sanitized() -> str:
    """Build SAN_LIB (see above) and return its path."""
    os.makedirs(SAN, exist_ok=True)
    stub_src = os.path.join(SAN, "stub.hip")
    stub_fb = os.path.join(SAN, "stub.hipfb")
    with open(stub_src, "w") as fh:
        fh.write("#include <hip/hip_runtime.h>\n__global__ void tvc_host_check_stub(int *p) { if (p) p[0] = 0; }\n")
    r = subprocess.run([HIPCC, "--cuda-device-only", "--offload-arch=gfx950", "-O1", stub_src, "-o", stub_fb],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("stub fatbinary failed:\n%s" % r.stderr)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))

    def host_obj(src):
        obj = os.path.join(SAN, os.path.basename(src) + ".o")
        cmd = [HIPCC, "--cuda-host-only", "-Xclang", "-fcuda-include-gpubinary", "-Xclang", stub_fb] + \
            SAN_HOST_FLAGS + ["-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("host compile failed for %s:\n%s" % (src, r.stderr))
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(host_obj, srcs))
    cmd = SAN_LINK + objs + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", SAN_LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitized link failed:\n%s" % r.stderr)
    return SAN_LIB


def build_host_check(src: str) -> str:
    """Compile a host-only sanitized program from a HIP source (kernels become
    stubs over the stub fatbinary of build_host_sanitized) and return its path."""
    if not os.path.exists(os.path.join(SAN, "stub.hipfb")):
        build_host_sanitized()
    obj = os.path.join(SAN, os.path.basename(src) + ".o")
    exe = os.path.join(SAN, os.path.splitext(os.path.basename(src))[0])
    cmd = [HIPCC, "--cuda-host-only", "-Xclang", "-fcuda-include-gpubinary", "-Xclang",
           os.path.join(SAN, "stub.hipfb")] + SAN_HOST_FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("host compile failed for %s:\n%s" % (src, r.stderr))
    rt = subprocess.run([SAN_LINK[0], "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    cmd = SAN_LINK[:1] + SAN_LINK[2:] + ["-shared-libsan", obj, "-L/opt/rocm/lib", "-lamdhip64",
                                         "-Wl,-rpath,/opt/rocm/lib", "-Wl,-rpath," + os.path.dirname(rt), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitized link failed:\n%s" % r.stderr)
    return exe


if __name__ == "__main__":
    if "--host-sanitized" in sys.argv:
        print("built", build_host_sanitized(), file=sys.stderr)
    else:
        build(verbose=True, incremental="--incremental" in sys.argv)
