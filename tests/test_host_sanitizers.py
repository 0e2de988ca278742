"""The host side of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; the kernels are the normal
build): tests/host_check.c drives every validation path of include/ddcc.h
and, on a GPU, one small run through each entry point family. No GPU is
needed for the first part."""
import os
import shutil
import subprocess

import pytest

from paper_2311_10314_amd import build as B


def _host_check():
    if not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    if not all(os.path.exists(os.path.join(B.BUILD, o))
               for o in B.KERNEL_OBJECTS):
        B.build()
    return B.build_host_check()


def _run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return subprocess.run([exe, *args], capture_output=True, text=True,
                          env=env, timeout=600)


def test_validation_paths_are_clean_under_sanitizers():
    r = _run(_host_check())
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr[-4000:]
