"""Degenerate and edge inputs on the GPU, against the oracle.

* Grids of one or two nodes along an axis (every neighbour is the node
  itself or its only partner through the periodic wrap) and ragged tiles,
  2D and 3D.
* Reduction consistency on the GPU: with the third phase absent at t = 0 an
  N = 3 run keeps phi C_3 at zero and follows the N = 2 run (mu_3 vanishes
  identically since g' is odd about 1/2, eq. 2.14). In 3D float contexts
  the C_i reach the chemical potential as a float32 field, so C_1 + C_2 = 1
  and mu_3 = 0 hold to float32 rounding and phi C_3 stays at that level.
* Zero-step calls: step(0) changes nothing; an adjoint sweep of 0 steps
  returns the objective of the current state and zero gradients.
"""
import numpy as np
import pytest

from paper_2311_10314_amd import workloads as W
from tests.helpers import oracle_run, rel_linf

pytestmark = pytest.mark.gpu

SHAPES = [(2, (1, 70)), (2, (9, 1)), (2, (2, 2)), (2, (1, 1)), (2, (3, 130)),
          (3, (1, 3, 66)), (3, (2, 1, 5)), (3, (3, 2, 1))]


@pytest.mark.parametrize("dim,shape", SHAPES)
def test_degenerate_grid(dim, shape):
    from paper_2311_10314_amd.ddcc import Sim
    wl = W.random_small(dim, 2, shape, seed=31)
    print("grid", shape, flush=True)
    sim = Sim.from_workload(wl, "fp64")
    sim.step(6)
    C, u, P = sim.read_moments()
    m = sim.mass()
    sim.close()
    o = oracle_run(wl, 6)
    eC = max(rel_linf(C[i], o["C"][i]) for i in range(2))
    eu = rel_linf(u, o["u"])
    print("grid %s: C %.2e u %.2e" % (shape, eC, eu), flush=True)
    assert eC < 1e-10 and eu < 1e-10
    assert np.all(np.abs(m - o["mass0"]) <= 1e-12 * np.abs(o["mass0"]))


def _absent_phase_case(N):
    n = 40
    x, y = W._grid((n, n))
    psi = W.psi_from_distance(W.periodic_distance((x, y), (n / 2, n / 2),
                                                  (n, n)) - 8.0)
    C1 = W.droplet(W.periodic_distance((x, y), (n / 2, n / 2 + 11), (n, n)),
                   8.0, 5.0)
    if N == 2:
        prm = W.default_params(2, 2, rho=[1.0, 3.0], nu=[0.1, 0.2])
        ct = np.full((1, n, n), 0.5)
        C0 = np.array([C1, 1 - C1])
    else:
        prm = W.default_params(2, 3, rho=[1.0, 3.0, 7.0], nu=[0.1, 0.2, 0.3])
        ct = np.array([np.full((n, n), 0.5), np.zeros((n, n))])
        C0 = np.array([C1, 1 - C1, np.zeros((n, n))])
    return W.Workload("absent_phase", 2, (n, n), "D2Q9", "D2Q9", prm, psi, ct,
                      C0, np.zeros((2, n, n)), np.zeros((n, n)), 200)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_absent_phase_stays_zero(precision, tol):
    from paper_2311_10314_amd.ddcc import Sim
    out = {}
    for N in (2, 3):
        sim = Sim.from_workload(_absent_phase_case(N), precision)
        sim.step(200)
        out[N] = sim.read_moments() + (sim.mass(),)
        sim.close()
    C2, u2, _, _ = out[2]
    C3, u3, _, m3 = out[3]
    print("%s: max C_3 %.1e, phase-3 mass %.1e, C_1 %.2e, u %.2e" % (
        precision, np.abs(C3[2]).max(), abs(m3[2]), rel_linf(C3[0], C2[0]),
        rel_linf(u3, u2)), flush=True)
    assert np.abs(C3[2]).max() < 1e-14 and abs(m3[2]) < 1e-12
    assert rel_linf(C3[0], C2[0]) < tol and rel_linf(u3, u2) < tol
    assert np.abs(u2).max() > 1e-5


def _absent_phase_case_3d(N):
    n = 32
    x, y, z = W._grid((n, n, n))
    c = (n / 2, n / 2, n / 2)
    psi = W.psi_from_distance(W.periodic_distance((x, y, z), c, (n, n, n))
                              - 7.0)
    C1 = W.droplet(W.periodic_distance((x, y, z), (n / 2, n / 2, n / 2 + 10),
                                       (n, n, n)), 7.0, 5.0)
    if N == 2:
        prm = W.default_params(3, 2, rho=[1.0, 3.0], nu=[0.1, 0.2])
        ct = np.full((1, n, n, n), 0.5)
        C0 = np.array([C1, 1 - C1])
    else:
        prm = W.default_params(3, 3, rho=[1.0, 3.0, 7.0], nu=[0.1, 0.2, 0.3])
        ct = np.array([np.full((n, n, n), 0.5), np.zeros((n, n, n))])
        C0 = np.array([C1, 1 - C1, np.zeros((n, n, n))])
    return W.Workload("absent_phase_3d", 3, (n, n, n), "D3Q15", "D3Q19", prm,
                      psi, ct, C0, np.zeros((3, n, n, n)), np.zeros((n, n, n)),
                      100)


@pytest.mark.parametrize("precision,c3_bar,tol", [("fp64", 1e-14, 1e-12),
                                                   ("fp32", 1e-7, 1e-5)])
def test_absent_phase_stays_zero_3d(precision, c3_bar, tol):
    """32^3, a droplet beside a solid sphere, 100 steps: the absent third
    phase stays at zero (FP64 to round-off, FP32 to the float32 rounding of
    the C field: measured 2e-8) and the N = 3 run follows the N = 2 run."""
    from paper_2311_10314_amd.ddcc import Sim
    out = {}
    for N in (2, 3):
        sim = Sim.from_workload(_absent_phase_case_3d(N), precision)
        sim.step(100)
        out[N] = sim.read_moments() + (sim.mass(),)
        sim.close()
    C2, u2, _, _ = out[2]
    C3, u3, _, m3 = out[3]
    print("3D %s: max C_3 %.1e, phase-3 mass %.1e, C_1 %.2e, u %.2e" % (
        precision, np.abs(C3[2]).max(), abs(m3[2]), rel_linf(C3[0], C2[0]),
        rel_linf(u3, u2)), flush=True)
    assert np.abs(C3[2]).max() < c3_bar and abs(m3[2]) < 1e-10
    assert rel_linf(C3[0], C2[0]) < tol and rel_linf(u3, u2) < tol
    assert np.abs(u2).max() > 1e-5


def test_zero_steps():
    from paper_2311_10314_amd.ddcc import Sim
    from tests.helpers import unpack_state
    wl = W.random_small(2, 2, (20, 70), seed=1)
    sim = Sim.from_workload(wl, "fp64")
    sim.step(3)
    before = unpack_state(sim, sim.save())
    sim.step(0)
    assert sim.time == 3
    J0 = sim.objective()
    J, gc, gp = sim.adjoint(0, 5)
    after = unpack_state(sim, sim.save())
    for key in ("f", "g", "hist", "T"):
        assert np.array_equal(before[key], after[key])
    assert sim.time == 3 and J == J0
    assert not gc.any() and not gp.any()
    sim.close()
