"""Parity of the 3D HIP path (D3Q15 phase sets, D3Q19 flow set) with the
FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from paper_2311_10314_amd import workloads as W
from tests.helpers import gpu_state_to_oracle, oracle_run, rel_linf

pytestmark = pytest.mark.gpu


def cases3d():
    return [W.random_small(3, 2, (12, 10, 70), seed=31),
            W.random_small(3, 3, (9, 13, 20), seed=32),
            W.random_small(3, 2, (21, 6, 7), seed=33)]


def gpu_run(wl, steps, precision="fp64", tile=None):
    from paper_2311_10314_amd.ddcc import Sim
    sim = Sim.from_workload(wl, precision)
    if tile:
        sim.set_tile(0, tile)
    m0 = sim.mass()
    sim.step(steps)
    C, u, P = sim.read_moments()
    return dict(C=C, u=u, P=P, mass0=m0, mass=sim.mass(), sim=sim)


def _err(g, o):
    return dict(C=max(rel_linf(g["C"][i], o["C"][i])
                      for i in range(len(o["C"]))),
                u=rel_linf(g["u"], o["u"]), P=rel_linf(g["P"], o["P"]))


@pytest.mark.parametrize("k", range(3))
def test_init_3d_fp64(k):
    wl = cases3d()[k]
    print("case", wl.name, wl.shape, flush=True)
    e = _err(gpu_run(wl, 0), oracle_run(wl, 0))
    print("init", e, flush=True)
    assert e["C"] < 1e-13 and e["u"] < 1e-12 and e["P"] < 1e-10


@pytest.mark.parametrize("k", range(3))
def test_one_step_3d_fp64(k):
    wl = cases3d()[k]
    print("case", wl.name, wl.shape, flush=True)
    o = oracle_run(wl, 1)
    g = gpu_run(wl, 1)
    st = gpu_state_to_oracle(wl, g["sim"])
    ef = np.abs(st.f - o["state"].f).max() / np.abs(o["state"].f).max()
    eg = np.abs(st.g - o["state"].g).max() / np.abs(o["state"].g).max()
    e = _err(g, o)
    print("one step f %.2e g %.2e" % (ef, eg), e, flush=True)
    assert ef < 1e-13 and eg < 1e-13 and max(e.values()) < 1e-10


@pytest.mark.parametrize("k", range(3))
def test_short_run_3d_fp64(k):
    wl = cases3d()[k]
    print("case", wl.name, wl.shape, flush=True)
    o = oracle_run(wl, 30)
    g = gpu_run(wl, 30)
    e = _err(g, o)
    print("30 steps", e, flush=True)
    assert max(e.values()) < 1e-10
    drift = np.abs(g["mass"] - g["mass0"]) / np.abs(g["mass0"])
    assert drift.max() < 1e-12


def test_tile_invariance_3d():
    wl = cases3d()[0]
    a = gpu_run(wl, 10, tile=2)
    b = gpu_run(wl, 10, tile=4)
    assert np.array_equal(a["C"], b["C"]) and np.array_equal(a["u"], b["u"])


@pytest.mark.parametrize("k", range(3))
def test_short_run_3d_fp32(k):
    wl = cases3d()[k]
    o = oracle_run(wl, 30)
    g = gpu_run(wl, 30, "fp32")
    e = _err(g, o)
    print("fp32 30 steps", e, flush=True)
    assert max(e.values()) < 1e-5
    drift = np.abs(g["mass"] - g["mass0"]) / np.abs(g["mass0"])
    assert drift.max() < 1e-6


def test_autotune_3d_keeps_the_state():
    from paper_2311_10314_amd.ddcc import Sim
    wl = cases3d()[1]
    a = Sim.from_workload(wl, "fp32")
    b = Sim.from_workload(wl, "fp32")
    a.step(3)
    b.step(3)
    assert b.autotune(2) in (2, 4)
    a.step(4)
    b.step(4)
    ca, ua, _ = a.read_moments()
    cb, ub, _ = b.read_moments()
    assert np.array_equal(ca, cb) and np.array_equal(ua, ub)
    a.close()
    b.close()


def test_long_run_3d_1000_steps():
    """1000 steps of a 12 x 14 x 20 box (N = 2, two solid blobs, random
    per-node angles and velocities) in FP64 and FP32 against one oracle run:
    relative L-inf of C_i and u within 1e-10 (FP64) and 1e-5 (FP32), phase
    mass drift within 1e-12 and 1e-6."""
    wl = W.random_small(3, 2, (12, 14, 20), seed=34)
    print("random 3D 12x14x20 N=2, 1000 steps", flush=True)
    o = oracle_run(wl, 1000)
    for precision, tol, dtol in (("fp64", 1e-10, 1e-12), ("fp32", 1e-5, 1e-6)):
        g = gpu_run(wl, 1000, precision)
        e = _err(g, o)
        drift = float((np.abs(g["mass"] - g["mass0"]) /
                       np.abs(g["mass0"])).max())
        g["sim"].close()
        print("%s 1000 steps" % precision, e, "drift %.1e" % drift, flush=True)
        assert max(e.values()) < tol
        assert drift < dtol


def _two_wall_box():
    """12 x 10 x 24 box, N = 3, two spherical solids, each wall its own
    psi_k and its own random per-node angles (Section 4.5 in 3D)."""
    wl = W.random_small(3, 3, (12, 10, 24), seed=35)
    rng = np.random.default_rng(36)
    coords = W._grid(wl.shape)
    walls = []
    for c, r in (((5.0, 3.0, 4.0), 3.5), ((17.0, 7.0, 8.0), 4.0)):
        psi_k = W.psi_from_distance(
            W.periodic_distance(coords, c, wl.shape) - r)
        ct_k = rng.uniform(-0.8, 0.8, size=(2,) + wl.shape)
        walls.append((psi_k, ct_k))
    wl.psi = walls[0][0] * walls[1][0]
    wl.cos_theta_iN = walls[0][1]
    wl.walls = walls
    return wl


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_two_walls_3d(precision, tol):
    """Several walls in 3D: the library's static wetting weights
    sum_k cos theta^k_iN |grad psi_k| (19-point stencil on each psi_k)
    against the oracle's per-wall sum, 60 steps."""
    wl = _two_wall_box()
    o = oracle_run(wl, 60)
    g = gpu_run(wl, 60, precision)
    e = _err(g, o)
    drift = float((np.abs(g["mass"] - g["mass0"]) / np.abs(g["mass0"])).max())
    print("two walls 3D %s 60 steps" % precision, e, "drift %.1e" % drift,
          flush=True)
    assert e["C"] < tol and e["u"] < tol
    assert drift < (1e-12 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_sphere_droplet_32(precision, tol):
    """32^3 version of the sphere / impacting-droplet case (sizes scaled by
    1/8), 40 steps against the oracle."""
    wl = W.droplet_impact_sphere_3d(n=32)
    o = oracle_run(wl, 40)
    g = gpu_run(wl, 40, precision)
    e = _err(g, o)
    fl = wl.psi >= 1e-3
    eP = rel_linf(g["P"][fl], o["P"][fl])
    print("sphere32 %s" % precision, e, "P(psi>=1e-3) %.2e" % eP, flush=True)
    assert e["C"] < tol and e["u"] < tol and eP < tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_sphere_droplet_64_one_step(precision, tol):
    """64^3 sphere case: GPU state after 50 steps, advanced one step by the
    oracle, matches the GPU's next step at every node."""
    import oracle
    from paper_2311_10314_amd.ddcc import Sim
    wl = W.droplet_impact_sphere_3d(n=64)
    sim = Sim.from_workload(wl, precision)
    sim.step(50)
    st = gpu_state_to_oracle(wl, sim)
    prm, geo, _ = oracle.from_workload(wl)
    st1 = oracle.step(prm, geo, st)
    Co, uo, Po = oracle.moments(prm, geo, st1)
    sim.step(1)
    C, u, P = sim.read_moments()
    g1 = gpu_state_to_oracle(wl, sim)
    eC = max(rel_linf(C[i], Co[i]) for i in range(2))
    eu = rel_linf(u, uo)
    fl = wl.psi >= 1e-3
    eP = rel_linf(P[fl], Po[fl])
    ef = np.abs(g1.f - st1.f).max() / np.abs(st1.f).max()
    eg = np.abs(g1.g - st1.g).max() / np.abs(st1.g).max()
    print("sphere64 %s one step: C %.2e u %.2e P %.2e f %.2e g %.2e" % (
        precision, eC, eu, eP, ef, eg), flush=True)
    assert max(eC, eu, ef, eg) < tol and eP < 100 * tol


# ---- D3Q7 phase sets (the paper's own 3D phase lattice) -------------------
def _d3q7_case(seed=21):
    return W.random_small(3, 2, (10, 12, 66), seed=seed, lattice_f="D3Q7",
                          d0=0.3)


def test_d3q7_one_step_fp64():
    """D3Q7 phase sets with the D3Q19 flow set, d0 = 0.3: one step of the
    populations and 30 steps of the moments against the oracle."""
    from paper_2311_10314_amd.ddcc import Sim
    import oracle
    wl = _d3q7_case()
    sim = Sim.from_workload(wl, "fp64")
    st = gpu_state_to_oracle(wl, sim)
    prm, geo, _ = oracle.from_workload(wl)
    st1 = oracle.step(prm, geo, st)
    sim.step(1)
    g1 = gpu_state_to_oracle(wl, sim)
    ef = np.abs(g1.f - st1.f).max() / np.abs(st1.f).max()
    eg = np.abs(g1.g - st1.g).max() / np.abs(st1.g).max()
    print("d3q7 one step f %.2e g %.2e" % (ef, eg), flush=True)
    assert ef < 1e-13 and eg < 1e-13
    sim.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_d3q7_short_run(precision, tol):
    wl = _d3q7_case(22)
    o = oracle_run(wl, 30)
    g = gpu_run(wl, 30, precision)
    e = _err(g, o)
    print("d3q7 %s 30 steps" % precision, e, flush=True)
    assert max(e.values()) < tol
    drift = np.abs(g["mass"] - g["mass0"]) / np.abs(g["mass0"])
    assert drift.max() < (1e-12 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("N,shape,precisions", [
    (3, (64, 72, 96), ("fp64", "fp32")),
    (2, (61, 66, 70), ("fp64",))])
def test_streaming_steps(N, shape, precisions):
    """Boxes that move more per step than the memory-side cache holds run
    the streaming step mode: 64 x 72 x 96 with three phases (about 290 MiB
    per step in FP32, 560 MiB in FP64), and 61 x 66 x 70 with two (FP64,
    about 280 MiB; nz = 61, ny = 66 and nx = 70 leave the last z column, tile
    row and tile partly filled). 2 steps
    against one oracle run, FP64 within 1e-12, FP32 within 2e-6 (C, u, and P
    where psi >= 1e-2)."""
    wl = W.random_small(3, N, shape, seed=41)
    print("random 3D %s N=%d, 2 steps" % ("x".join(map(str, shape)), N),
          flush=True)
    o = oracle_run(wl, 2)
    fl = np.asarray(wl.psi) >= 1e-2
    for precision in precisions:
        tol = 1e-12 if precision == "fp64" else 2e-6
        g = gpu_run(wl, 2, precision)
        g["sim"].close()
        e = _err(g, o)
        eP = rel_linf(g["P"][fl], o["P"][fl])
        print("%s 2 steps" % precision, e, "P(psi>=1e-2) %.2e" % eP,
              flush=True)
        assert e["C"] < tol and e["u"] < tol and eP < 100 * tol
