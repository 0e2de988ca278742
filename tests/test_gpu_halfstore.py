"""16-bit population storage (DDCC_FP16, DDCC_BF16) against the FP64 oracle.

The moving populations are stored in 16 bits (g_0 as the deviation
g_0 - rho0), history, T and geometry in float32, arithmetic in float32. The
bars follow from the unit roundoff u_s of the storage type (2^-11 for IEEE
half, 2^-8 for bfloat16):
  * one step from a common state: every moving population within
    u_s |f| (+ float32 arithmetic, + half the subnormal spacing) of the
    oracle's step;
  * short runs: C_i within 10 u_s and u within 50 u_s (relative L-inf);
  * per-phase mass: the float64 rest populations take back each node's
    storage rounding, so the drift stays at the float32-arithmetic level
    (< 1e-10), not at u_s.
"""
import numpy as np
import pytest

from paper_2311_10314_amd import workloads as W
from tests.helpers import gpu_state_to_oracle, oracle_run, rel_linf

pytestmark = pytest.mark.gpu

UNIT = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}
# Below the smallest normal number (2^-14 for IEEE half) the spacing is
# absolute: rounding to nearest errs by up to half of it.
SUB = {"fp16": 2.0 ** -25, "bf16": 2.0 ** -134}


def _run(wl, steps, precision):
    from paper_2311_10314_amd.ddcc import Sim
    sim = Sim.from_workload(wl, precision)
    m0 = sim.mass()
    sim.step(steps)
    C, u, P = sim.read_moments()
    drift = np.abs(sim.mass() - m0) / np.abs(m0)
    return sim, dict(C=C, u=u, P=P), drift


def _errors(g, o):
    return dict(C=max(rel_linf(g["C"][i], o["C"][i]) for i in range(len(o["C"]))),
                u=rel_linf(g["u"], o["u"]))


CASES_2D = [("random_2d_n2", lambda: W.random_small(2, 2, (20, 70), seed=1)),
            ("random_2d_n3", lambda: W.random_small(2, 3, (37, 100), seed=2))]


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
@pytest.mark.parametrize("case", [c[0] for c in CASES_2D])
def test_short_run_2d(case, precision):
    wl = dict(CASES_2D)[case]()
    print("case", case, wl.shape, precision, flush=True)
    o = oracle_run(wl, 60)
    sim, g, drift = _run(wl, 60, precision)
    sim.close()
    e = _errors(g, o)
    us = UNIT[precision]
    print("%s 60 steps C %.2e u %.2e (u_s %.1e) drift %.1e" % (
        precision, e["C"], e["u"], us, drift.max()), flush=True)
    assert e["C"] < 10 * us and e["u"] < 50 * us
    assert drift.max() < 1e-10


def _one_step_check(wl, precision, warm):
    import oracle
    from paper_2311_10314_amd.ddcc import Sim
    sim = Sim.from_workload(wl, precision)
    sim.step(warm)
    st = gpu_state_to_oracle(wl, sim)
    prm, geo, _ = oracle.from_workload(wl)
    st1 = oracle.step(prm, geo, st)
    sim.step(1)
    g1 = gpu_state_to_oracle(wl, sim)
    sim.close()
    us = UNIT[precision]
    moving_f = np.abs(g1.f[:, 1:] - st1.f[:, 1:])
    scale_f = np.abs(st1.f[:, 1:]).max()
    bound_f = us * np.abs(st1.f[:, 1:]) + 2e-5 * scale_f + SUB[precision]
    g_err = np.abs(g1.g - st1.g)
    dev = st1.g.copy()
    dev[0] -= wl.params["rho0"]        # g_0 is stored as g_0 - rho0
    bound_g = us * np.abs(dev) + 2e-5 * np.abs(dev).max() + SUB[precision]
    print("%s one step: max f excess %.2e, max g excess %.2e" % (
        precision, (moving_f - bound_f).max(), (g_err - bound_g).max()),
        flush=True)
    assert np.all(moving_f <= bound_f)
    assert np.all(g_err <= bound_g)
    # rest populations: exact mass bookkeeping, so phi C_i (the node sums)
    # matches the oracle up to the moving populations' rounding
    psiC_g = g1.f.sum(axis=1)
    psiC_o = st1.f.sum(axis=1)
    bound_c = us * np.abs(st1.f[:, 1:]).sum(axis=1) + 2e-5
    assert np.all(np.abs(psiC_g - psiC_o) <= bound_c)


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_one_step_populations_2d(precision):
    wl = W.random_small(2, 3, (37, 100), seed=2)
    _one_step_check(wl, precision, 30)


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_sphere_droplet_32_3d(precision):
    wl = W.droplet_impact_sphere_3d(n=32)
    o = oracle_run(wl, 40)
    sim, g, drift = _run(wl, 40, precision)
    sim.close()
    e = _errors(g, o)
    us = UNIT[precision]
    print("sphere32 %s 40 steps C %.2e u %.2e drift %.1e" % (
        precision, e["C"], e["u"], drift.max()), flush=True)
    assert e["C"] < 10 * us and e["u"] < 50 * us
    assert drift.max() < 1e-10


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_one_step_populations_3d(precision):
    wl = W.random_small(3, 2, (12, 10, 70), seed=11)
    _one_step_check(wl, precision, 20)
