"""Error paths of a live context through the C ABI: every call that is out of
order or gets invalid input returns its DDCC_E_* code with a message, and
leaves the context usable. The non-finite check of the mass diagnostic is
driven by a checkpoint with a NaN written into it on the host (no kernel is
made to fault)."""
import numpy as np
import pytest

from paper_2311_10314_amd import workloads as W

pytestmark = pytest.mark.gpu


def _codes():
    from paper_2311_10314_amd import ddcc
    return ddcc


def _expect(code, fn, *args):
    d = _codes()
    with pytest.raises(d.DDCCError) as e:
        fn(*args)
    assert e.value.code == code, (e.value.code, str(e.value))
    return e.value


def _fresh(wl, precision="fp64"):
    d = _codes()
    p = d.make_params(wl.dim, wl.shape, wl.nphase, wl.lattice_f,
                      wl.lattice_g, precision, **wl.params)
    return d.Sim(p)


def test_calls_out_of_order():
    d = _codes()
    wl = W.random_small(2, 2, (20, 70), seed=1)
    s = _fresh(wl)
    _expect(d.DDCC_E_STATE, s.init_fields, wl.C0)          # before geometry
    s.init_geometry(wl.psi, wl.cos_theta_iN)
    _expect(d.DDCC_E_STATE, s.step, 1)                      # before fields
    _expect(d.DDCC_E_STATE, s.read_moments)
    _expect(d.DDCC_E_STATE, s.mass)
    _expect(d.DDCC_E_STATE, s.autotune, 2)
    s.init_fields(wl.C0, wl.u0, wl.P0)
    s.step(2)
    assert s.time == 2
    s.close()


def test_invalid_inputs_are_rejected_and_the_context_stays_usable():
    d = _codes()
    wl = W.random_small(2, 2, (20, 70), seed=1)
    s = _fresh(wl)
    bad = np.array(wl.psi)
    bad[3, 5] = 1.5
    _expect(d.DDCC_E_INVAL, s.init_geometry, bad, wl.cos_theta_iN)
    bad[3, 5] = np.nan
    _expect(d.DDCC_E_INVAL, s.init_geometry, bad, wl.cos_theta_iN)
    ct = np.array(wl.cos_theta_iN)
    ct.flat[7] = -1.25
    _expect(d.DDCC_E_INVAL, s.init_geometry, wl.psi, ct)
    s.init_geometry(wl.psi, wl.cos_theta_iN)
    C = np.array(wl.C0)
    C[1, 2, 3] = np.inf
    _expect(d.DDCC_E_INVAL, s.init_fields, C)
    s.init_fields(wl.C0, wl.u0, wl.P0)
    _expect(d.DDCC_E_INVAL, s.step, -1)
    _expect(d.DDCC_E_INVAL, s.set_tile, 0, 3)
    _expect(d.DDCC_E_INVAL, s.set_tile, 32, 0)
    _expect(d.DDCC_E_INVAL, s.autotune, 0)
    e = _expect(d.DDCC_E_INVAL, s.load, np.zeros(16, np.uint8))
    assert "too small" in str(e)
    # the context still steps, and from the same state as a clean one
    s.step(3)
    ref = d.Sim.from_workload(wl, "fp64")
    ref.step(3)
    assert np.array_equal(s.read_moments()[0], ref.read_moments()[0])
    s.close()
    ref.close()


def test_checkpoint_of_another_shape_is_refused():
    d = _codes()
    a = d.Sim.from_workload(W.random_small(2, 2, (20, 70), seed=1), "fp64")
    b = d.Sim.from_workload(W.random_small(2, 2, (20, 72), seed=1), "fp64")
    buf = b.save()
    _expect(d.DDCC_E_INVAL, a.load, buf)
    a.close()
    b.close()


def test_non_finite_population_is_reported_by_the_mass_check():
    """A NaN put into a rest population of a saved state (host side) is
    found by ddcc_mass, which returns DDCC_E_NONFINITE."""
    d = _codes()
    wl = W.random_small(2, 2, (20, 70), seed=1)
    s = d.Sim.from_workload(wl, "fp64")
    buf = s.save()
    n = wl.nodes
    npop = wl.nphase * 8 * n                # moving planes of the phase sets
    off = 56 + npop * 8 + 8 * 123          # rest plane of phase 0, node 123
    nan = np.frombuffer(np.array([np.nan]).tobytes(), np.uint8)
    bad = buf.copy()
    bad[off:off + 8] = nan
    s.load(bad)
    _expect(d.DDCC_E_NONFINITE, s.mass)
    s.load(buf)                            # a good state clears it
    assert np.all(np.isfinite(s.mass()))
    s.close()


def test_periodic_diagnostics_record_the_masses_of_the_checked_levels():
    """Checks every 5 steps inside the step stream: after 23 steps the last
    check is the level 20, and its masses equal ddcc_mass of a context
    stepped to 20 (same kernel, same block order); phase mass is
    conserved between checks."""
    d = _codes()
    wl = W.random_small(2, 3, (37, 100), seed=2)
    s = d.Sim.from_workload(wl, "fp64")
    _expect(d.DDCC_E_STATE, s.diagnostics)             # off by default
    _expect(d.DDCC_E_INVAL, s.set_diagnostics, -1)
    s.set_diagnostics(5)
    m, tc, tn = s.diagnostics()
    assert tc == -1 and tn == -1 and np.all(np.isnan(m))
    s.step(23)
    s.sync()
    m, tc, tn = s.diagnostics()
    assert tc == 20 and tn == -1
    ref = d.Sim.from_workload(wl, "fp64")
    m0 = ref.mass()
    ref.step(20)
    assert np.array_equal(m, ref.mass())
    assert np.abs(m - m0).max() <= 1e-12 * np.abs(m0).max()
    s.set_diagnostics(0)
    _expect(d.DDCC_E_STATE, s.diagnostics)
    s.close()
    ref.close()


def test_periodic_diagnostics_flag_a_non_finite_state():
    """A NaN in the loaded state is seen by the first check; ddcc_sync then
    returns DDCC_E_NONFINITE naming the step, until a good state is
    loaded."""
    d = _codes()
    wl = W.random_small(2, 2, (20, 70), seed=1)
    s = d.Sim.from_workload(wl, "fp32")
    good = s.save()
    npop = wl.nphase * 8 * wl.nodes        # moving planes of the phase sets
    off = 56 + npop * 4 + 8 * 77           # rest plane (float64), node 77
    bad = good.copy()
    bad[off:off + 8] = np.frombuffer(np.array([np.inf]).tobytes(), np.uint8)
    s.set_diagnostics(2)
    s.load(bad)
    s.step(5)
    e = _expect(d.DDCC_E_NONFINITE, s.sync)
    assert "step 2" in str(e)
    _, tc, tn = s.diagnostics()
    assert tc == 4 and tn == 2
    s.load(good)
    s.step(4)
    s.sync()
    assert s.diagnostics()[2] == -1
    s.close()
