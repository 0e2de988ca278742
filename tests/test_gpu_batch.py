"""Batches of independent 2D instances (ddcc_batch_*) on the GPU.

Each instance of a batch must evolve exactly as a single context of its own
size: the batch kernel runs the same per-node arithmetic on (instance, tile)
work items. Checked against the FP64 oracle (1e-10) and against single
contexts (1e-13), with and without graph replay and after autotuning.
"""
import numpy as np
import pytest

from paper_2311_10314_amd import workloads as W
from tests.helpers import oracle_run, rel_linf

pytestmark = pytest.mark.gpu


def small_batch():
    """Ragged shapes sharing N = 2 and the method parameters."""
    return [W.random_small(2, 2, (20, 70), seed=1),
            W.random_small(2, 2, (9, 13), seed=4),
            W.random_small(2, 2, (33, 64), seed=7),
            W.random_small(2, 2, (64, 5), seed=8)]


def _single(wl, steps, precision):
    from paper_2311_10314_amd.ddcc import Sim
    s = Sim.from_workload(wl, precision)
    s.step(steps)
    out = s.read_moments()
    s.close()
    return out


def _errs(a, b):
    return max(max(rel_linf(a[0][i], b[0][i]) for i in range(len(b[0]))),
               rel_linf(a[1], b[1]))


def test_batch_matches_oracle_and_single_fp64():
    from paper_2311_10314_amd.ddcc import Batch
    wls = small_batch()
    b = Batch.from_workloads(wls, "fp64")
    m0 = [b.mass(i) for i in range(len(wls))]
    b.step(40)
    for i, wl in enumerate(wls):
        got = b.read_moments(i)
        o = oracle_run(wl, 40)
        e_o = _errs(got, (o["C"], o["u"]))
        e_s = _errs(got, _single(wl, 40, "fp64"))
        drift = np.abs(b.mass(i) - m0[i]) / np.abs(m0[i])
        print("instance %d %s: vs oracle %.2e, vs single %.2e, drift %.1e" % (
            i, wl.shape, e_o, e_s, drift.max()), flush=True)
        assert e_o < 1e-10 and e_s < 1e-13 and drift.max() < 1e-12
    b.close()


@pytest.mark.parametrize("ty", [4, 8, 16])
def test_batch_tile_heights_agree(ty):
    from paper_2311_10314_amd.ddcc import Batch
    wls = small_batch()
    ref = Batch.from_workloads(wls, "fp64")
    ref.step(15)
    b = Batch.from_workloads(wls, "fp64")
    b.set_tile(ty)
    b.step(15)
    for i in range(len(wls)):
        assert _errs(b.read_moments(i), ref.read_moments(i)) < 1e-13
    b.close()
    ref.close()


def test_batch_graph_replay_equals_direct():
    """Graphs of 4 steps (captured once, replayed), plus direct steps for
    the remainder, give the same state as 10 direct steps; a second call
    replays the graph of the other level parity."""
    from paper_2311_10314_amd.ddcc import Batch
    wls = small_batch()
    d = Batch.from_workloads(wls, "fp32")
    d.step(10)
    d.step(7)
    g = Batch.from_workloads(wls, "fp32")
    g.set_graph(4)
    g.step(10)
    g.step(7)
    assert g.time == d.time == 17
    for i in range(len(wls)):
        a, c = g.read_moments(i), d.read_moments(i)
        assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    g.close()
    d.close()


def test_batch_autotune_keeps_state():
    from paper_2311_10314_amd.ddcc import Batch
    wls = small_batch()
    a = Batch.from_workloads(wls, "fp32")
    a.step(5)
    ty = a.autotune(3)
    assert ty in (4, 8, 16)
    assert a.time == 5
    a.step(5)
    c = Batch.from_workloads(wls, "fp32")
    c.set_tile(ty)
    c.step(10)
    for i in range(len(wls)):
        x, y = a.read_moments(i), c.read_moments(i)
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
    a.close()
    c.close()


def test_batched_workload_fp32_mass_and_single():
    """Eight instances of the uneven batched workload in FP32: per-phase
    mass drift below 1e-6 after 200 steps, and the same result as single
    contexts."""
    from paper_2311_10314_amd.ddcc import Batch
    wls = W.batched_instances(8)
    b = Batch.from_workloads(wls, "fp32")
    b.set_graph(50)
    m0 = [b.mass(i) for i in range(len(wls))]
    b.step(200)
    for i, wl in enumerate(wls):
        drift = np.abs(b.mass(i) - m0[i]) / np.abs(m0[i])
        e_s = _errs(b.read_moments(i), _single(wl, 200, "fp32"))
        print("instance %d %s: drift %.1e vs single %.1e" % (
            i, wl.shape, drift.max(), e_s), flush=True)
        assert drift.max() < 1e-6 and e_s < 1e-5
    b.close()


def test_full_batched_workload_every_instance():
    """The whole 256-instance workload in FP32 as the bench runs it
    (autotuned tile, HIP-graph step loop; at 5.5 M nodes the batch runs the
    streaming step mode): after 20 steps every instance equals a single
    context of its own (plain mode, at most 65 536 nodes) to 1e-6 (measured:
    bit for bit), and its phase masses are conserved to 1e-6."""
    from paper_2311_10314_amd.ddcc import Batch
    wls = W.batched_instances(256)
    b = Batch.from_workloads(wls, "fp32")
    b.autotune(3)
    b.set_graph(10)
    m0 = [b.mass(i) for i in range(len(wls))]
    b.step(20)
    worst, wi, wdrift = 0.0, -1, 0.0
    for i, wl in enumerate(wls):
        e = _errs(b.read_moments(i), _single(wl, 20, "fp32"))
        d = float((np.abs(b.mass(i) - m0[i]) / np.abs(m0[i])).max())
        wdrift = max(wdrift, d)
        if e > worst:
            worst, wi = e, i
    b.close()
    print("256 instances: worst difference to single contexts %.1e "
          "(instance %d), worst mass drift %.1e" % (worst, wi, wdrift),
          flush=True)
    assert worst <= 1e-6 and wdrift < 1e-6


def _samples():
    """Parameter samples: the same N = 2 method with different densities,
    viscosities, surface tension, mobility and body force per instance."""
    return [W.random_small(2, 2, (20, 70), seed=1),
            W.random_small(2, 2, (33, 64), seed=7, rho=[1.0, 10.0],
                           nu=[0.05, 0.15], m0=0.02,
                           sigma=[[0.0, 0.005], [0.005, 0.0]]),
            W.random_small(2, 2, (9, 13), seed=4, rho=[4.0, 0.5],
                           force=[1e-5, 0.0]),
            W.random_small(2, 2, (64, 5), seed=8, nu=[0.3, 0.02], m0=0.1)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_parameter_samples(precision):
    """Each instance with its own parameters (ddcc_batch_set_params) evolves
    as a single context with those parameters (within 1e-13 in FP64, 2e-6
    in FP32: the two kernels are compiled separately) and, in FP64, within
    1e-10 of the oracle; with a graph step loop too."""
    from paper_2311_10314_amd.ddcc import Batch
    wls = _samples()
    assert len({repr(w.params) for w in wls}) == len(wls)
    b = Batch.from_workloads(wls, precision)
    b.step(12)
    b.set_graph(4)
    b.step(8)
    for i, wl in enumerate(wls):
        got = b.read_moments(i)
        single = _single(wl, 20, precision)
        e_s = _errs(got, single)
        print("instance %d %s: vs single %.2e" % (i, precision, e_s),
              flush=True)
        assert e_s < (1e-13 if precision == "fp64" else 2e-6)
        if precision == "fp64":
            o = oracle_run(wl, 20)
            e = _errs(got, (o["C"], o["u"]))
            print("instance %d: vs oracle %.2e" % (i, e), flush=True)
            assert e < 1e-10
    b.close()


def test_batch_parameters_must_match_the_batch():
    from paper_2311_10314_amd.ddcc import (DDCC_E_INVAL, Batch, DDCCError,
                                           make_params)
    wls = _samples()[:2]
    b = Batch.from_workloads(wls, "fp32")
    other = make_params(2, wls[0].shape, 3, "D2Q9", "D2Q9", "fp32",
                        **W.random_small(2, 3, (20, 70), seed=1).params)
    with pytest.raises(DDCCError) as e:
        b.set_params(0, other)
    assert e.value.code == DDCC_E_INVAL
    bad = make_params(2, wls[0].shape, 2, "D2Q9", "D2Q9", "fp32",
                      **dict(wls[0].params, rho=[1.0, -1.0]))
    with pytest.raises(DDCCError) as e:
        b.set_params(1, bad)
    assert e.value.code == DDCC_E_INVAL
    b.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_full_batched_workload_2000_steps(precision, tol):
    """The whole 256-instance workload over its 2000 steps (graph step
    loop; streaming step mode), two of its smallest instances against
    oracle runs of the same length: C_i and u within the bar, P where
    psi >= 1e-2, mass drift 1e-12 (FP64) and 1e-6 (FP32)."""
    from paper_2311_10314_amd.ddcc import Batch
    steps = 2000
    wls = W.batched_instances(256)
    pick = sorted(range(256), key=lambda i: wls[i].nodes)[:2]
    refs = {i: oracle_run(wls[i], steps) for i in pick}
    b = Batch.from_workloads(wls, precision)
    b.set_graph(50)
    m0 = {i: b.mass(i) for i in pick}
    b.step(steps)
    for i in pick:
        C, u, P = b.read_moments(i)
        o = refs[i]
        fl = wls[i].psi >= 1e-2
        eC = max(rel_linf(C[j], o["C"][j]) for j in range(len(C)))
        eu = rel_linf(u, o["u"])
        eP = rel_linf(P[fl], o["P"][fl])
        drift = float(np.max(np.abs(b.mass(i) - m0[i]) / np.abs(m0[i])))
        print("%s instance %d %s after %d: C %.2e u %.2e P %.2e drift %.2e"
              % (precision, i, wls[i].shape, steps, eC, eu, eP, drift),
              flush=True)
        assert eC < tol and eu < tol and eP < tol
        assert drift < (1e-12 if precision == "fp64" else 1e-6)
    b.close()
