"""Build libddcc.so in-tree with hipcc for gfx950.

python -m paper_2311_10314_amd.build [-j JOBS] [-v] [--host-check]

--host-check also builds _build/sanitize/host_check: the host side of the
C ABI (api.cpp, adjoint_api.cpp) with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code only, linked with the normal
kernel objects and the checks of tests/host_check.c.
"""
import argparse
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libddcc.so")
SOURCES = ["api.cpp", "adjoint_api.cpp", "step2d.hip", "step3d.hip",
           "util.hip", "adjoint2d.hip"]
HOST_SOURCES = ["api.cpp", "adjoint_api.cpp"]
KERNEL_OBJECTS = ["step2d.o", "step3d.o", "util.o", "adjoint2d.o"]
SANITIZE = os.path.join(BUILD, "sanitize")
HOST_CHECK = os.path.join(SANITIZE, "host_check")
LLVM = os.environ.get("ROCM_LLVM", "/opt/rocm/llvm/bin")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 instructions stay off: the compiler would otherwise pair
# independent float operations into v_pk_* forms.
COMMON = ["-O3", "-std=c++20", "--offload-arch=" + ARCH, "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def _compile(src, verbose):
    out = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", os.path.join(CSRC, src),
                              "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s%s" % (src, r.stdout,
                                                          r.stderr))
    return out


def build(jobs=4, verbose=False):
    """Compile every HIP source and link the shared library (always
    recompiles)."""
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("%s failed:\n%s%s" % (cmd[0], r.stdout, r.stderr))


def build_host_check(verbose=False):
    """The sanitizer build of the host code (the kernel objects of build()
    must exist): host-only -fsanitize on the hipcc lines, the C driver and
    the link on lines that name no HIP source."""
    os.makedirs(SANITIZE, exist_ok=True)
    objs = []
    for src in HOST_SOURCES:
        out = os.path.join(SANITIZE, os.path.splitext(src)[0] + ".o")
        _run([HIPCC, "-O1", "-g", "-std=c++20", "--offload-arch=" + ARCH,
              "-fPIC", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
              "-fsanitize=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
              "-Wno-unused-command-line-argument", "-x", "hip", "-c",
              os.path.join(CSRC, src), "-o", out], verbose)
        objs.append(out)
    drv = os.path.join(SANITIZE, "host_check.o")
    _run([os.path.join(LLVM, "clang"), "-O1", "-g", "-std=c11",
          "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-c",
          os.path.join(os.path.dirname(HERE), "tests", "host_check.c"), "-o",
          drv], verbose)
    kernels = [os.path.join(BUILD, o) for o in KERNEL_OBJECTS]
    _run([os.path.join(LLVM, "clang++"), "-fsanitize=address,undefined", drv]
         + objs + kernels + ["-L/opt/rocm/lib", "-lamdhip64",
                             "-Wl,-rpath,/opt/rocm/lib", "-o", HOST_CHECK],
         verbose)
    return HOST_CHECK


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=4)
    ap.add_argument("-v", "--verbose", action="store_true")
    ap.add_argument("--host-check", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.verbose))
    if a.host_check:
        print(build_host_check(a.verbose))


if __name__ == "__main__":
    sys.exit(main())
