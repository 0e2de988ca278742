"""ddcc_mass_noalloc, the mass check that allocates nothing, against
ddcc_mass on the same contexts: two calls in a row on one GPU, the second
on a smaller context (fewer blocks and phases), so the second must not see
what the first left in the shared static workspace."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(shape, nphase, seed, precision, steps):
    from paper_2311_10314_amd import workloads as W
    from paper_2311_10314_amd.ddcc import Sim
    wl = W.random_small(len(shape), nphase, shape, seed=seed)
    sim = Sim.from_workload(wl, precision)
    sim.step(steps)
    return sim


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mass_noalloc_matches_mass_on_two_calls(precision):
    import torch
    from paper_2311_10314_amd import ddcc as d
    big = _case((300, 260), 3, 11, precision, 5)       # 78 000 nodes: 305 blocks
    small = _case((20, 70), 2, 12, precision, 3)       # 1 400 nodes: 6 blocks
    for sim in (big, small):
        out = torch.full((sim.nphase,), float("nan"), dtype=torch.float64,
                         device="cuda")
        flag = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        print("mass_noalloc %s shape %s N=%d" % (precision, sim.shape,
                                                sim.nphase), flush=True)
        sim.mass_noalloc(out, flag)
        sim.sync()
        got = out.cpu().numpy()
        ref = sim.mass()
        assert np.array_equal(got, ref), (got, ref)
        assert int(flag.item()) == 0
        # the flag output may be omitted
        out2 = torch.zeros((sim.nphase,), dtype=torch.float64, device="cuda")
        sim.mass_noalloc(out2)
        sim.sync()
        assert np.array_equal(out2.cpu().numpy(), ref)
    big.close()
    small.close()


def test_mass_noalloc_argument_errors():
    import torch
    from paper_2311_10314_amd import ddcc as d
    from paper_2311_10314_amd import workloads as W
    from paper_2311_10314_amd.ddcc import Sim
    assert d.ddcc_mass_noalloc(None, None, None) == d.DDCC_E_INVAL
    wl = W.random_small(2, 2, (9, 13), seed=4)
    p = d.make_params(wl.dim, wl.shape, wl.nphase, wl.lattice_f, wl.lattice_g,
                      "fp64", **wl.params)
    sim = Sim(p)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    # before init_fields
    assert d.ddcc_mass_noalloc(sim._h, ctypes.c_void_p(out.data_ptr()),
                               None) == d.DDCC_E_STATE
    sim.init_geometry(wl.psi, wl.cos_theta_iN)
    sim.init_fields(wl.C0, wl.u0, wl.P0)
    assert d.ddcc_mass_noalloc(sim._h, None, None) == d.DDCC_E_INVAL
    sim.mass_noalloc(out)
    sim.sync()
    assert np.array_equal(out.cpu().numpy(), sim.mass())
    sim.close()
