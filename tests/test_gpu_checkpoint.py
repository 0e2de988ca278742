"""Checkpoint and resume (ddcc_save / ddcc_load): a run of 2k steps equals,
bit for bit, k steps, a checkpoint, a fresh context restored from it and k
more steps, in every storage type and in 2D and 3D (the 3D box also in the
streaming step mode)."""
import numpy as np
import pytest

from paper_2311_10314_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "2d_n3": lambda: W.random_small(2, 3, (37, 100), seed=2),
    "3d_n2": lambda: W.random_small(3, 2, (12, 10, 70), seed=31),
    "3d_streaming": lambda: W.random_small(3, 2, (64, 72, 96), seed=42),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_resume_from_checkpoint_is_exact(case, precision):
    from paper_2311_10314_amd.ddcc import Sim
    wl = CASES[case]()
    k = 7
    print("case", case, wl.shape, precision, flush=True)
    a = Sim.from_workload(wl, precision)
    a.step(2 * k)
    ref = a.read_moments()
    a.close()
    b = Sim.from_workload(wl, precision)
    b.step(k)
    state = b.save()
    b.close()
    c = Sim.from_workload(wl, precision)
    c.step(3)                     # a different state, overwritten by load
    c.load(state)
    assert c.time == k
    c.step(k)
    got = c.read_moments()
    assert c.time == 2 * k
    c.close()
    for x, y in zip(got, ref):
        assert np.array_equal(x, y)
