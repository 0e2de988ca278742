"""Host-side accounting of bench.py (no GPU): the algorithmic bytes per
node update that the roofline objects divide by, the source hash that
keys the committed counter traffic, and the one-GPU guard.

The byte counts are written out here per component, from the storage the
step must move: every population read once and written once in the
population type; the history (phi C_i u: N d values, the symmetric flux
tensor: d(d+1)/2, P: 1) read and written once; the antisymmetric flux
tensor T (d(d-1)/2) read and written once; psi and the N - 1 wetting
weights read once, in the field type.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _count(N, d, Qf, Qg, pop_bytes, field_bytes, rest64=False):
    moving_and_rest = (N * Qf + Qg) * pop_bytes * 2
    if rest64:  # the N rest populations kept in float64 instead
        moving_and_rest += N * (8 - pop_bytes) * 2
    history = (N * d + d * (d + 1) // 2 + 1) * field_bytes * 2
    T = (d * (d - 1) // 2) * field_bytes * 2
    static = (1 + (N - 1)) * field_bytes
    return moving_and_rest + history + T + static


@pytest.mark.parametrize("case,N,d,Qf,Qg,prec,pop,field,expect", [
    # the 3D impact workload: D3Q15 phase sets, D3Q19 flow set
    ("sphere3d", 2, 3, 15, 19, "fp32", 4, 4, 528),
    ("sphere3d", 2, 3, 15, 19, "fp64", 8, 8, 1056),
    ("sphere3d", 2, 3, 15, 19, "fp16", 2, 4, 332),
    ("sphere3d", 2, 3, 15, 19, "bf16", 2, 4, 332),
    # the 2D porous box (N = 3) and the disk / batch boxes (N = 2), D2Q9
    ("porous2d", 3, 2, 9, 9, "fp32", 4, 4, 388),
    ("porous2d", 3, 2, 9, 9, "fp64", 8, 8, 776),
    ("disk2d", 2, 2, 9, 9, "fp32", 4, 4, 296),
    ("disk2d", 2, 2, 9, 9, "fp64", 8, 8, 592),
])
def test_algorithmic_bytes_per_node(case, N, d, Qf, Qg, prec, pop, field,
                                    expect):
    assert _count(N, d, Qf, Qg, pop, field) == expect
    assert bench.algorithmic_bytes_per_node(N, d, Qf, Qg, prec) == expect
    assert (bench.algorithmic_bytes_per_node(N, d, Qf, Qg, prec, True)
            == _count(N, d, Qf, Qg, pop, field, rest64=True))


def test_float64_rest_planes_add_what_they_should():
    # 3D FP32 N = 2: two rest planes of 8 instead of 4 bytes, read and
    # written: 16 B more; 2D FP32 N = 3: 24 B more; FP64: nothing
    assert bench.algorithmic_bytes_per_node(2, 3, 15, 19, "fp32", True) == 544
    assert bench.algorithmic_bytes_per_node(3, 2, 9, 9, "fp32", True) == 412
    assert bench.algorithmic_bytes_per_node(3, 2, 9, 9, "fp64", True) == 776


def test_source_hash_ignores_comments_and_spacing():
    a = "int f(int x) {  // returns x\n  return x + 1; /* one */\n}\n"
    b = "int f(int x)\n{\n return x + 1;\n}"
    c = "int f(int x) { return x + 2; }"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)


def test_counter_traffic_is_keyed_by_the_current_sources():
    # every committed entry names the kernels it was taken on; an entry is
    # reported only while its hash matches the sources
    import json
    with open(bench.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    for key, e in t.items():
        kind, prec = key.split("_")
        assert e["kernel"] == bench.KERNEL_TAGS[(kind, prec)]
        live = e["kernel_hash"] == bench.kernel_source_hash(kind)
        assert (bench.measured_traffic(kind, prec) is not None) == live


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
