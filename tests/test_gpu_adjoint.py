"""Adjoint sweep (ddcc_adjoint) on the GPU.

J = sum w phi C_k / sum phi C_k after n steps (w = node index along x: the
centroid x of phase k); gradients with respect to the per-node angle field
cos theta_iN and psi. Checked against
  * the oracle's reverse-mode derivative (oracle.adjoint, float64 autograd
    of the oracle step) from the same initial state: FP64 within 1e-9 of
    the largest gradient entry; FP32 within 1e-4 (angles and psi, over the
    whole field);
  * central finite differences (Richardson-extrapolated) of the GPU FP64
    forward along random directions: within 1e-6 (the target is 1e-4);
and for properties of the sweep: gradients independent of the checkpoint
interval (bit for bit), zero gradient for a constant weight, the context
left at the final level, and the torch.autograd bridge.
"""
import numpy as np
import pytest

from paper_2311_10314_amd import workloads as W
from tests.helpers import gpu_state_to_oracle

pytestmark = pytest.mark.gpu


def _sim(wl, precision="fp64"):
    from paper_2311_10314_amd.ddcc import Sim
    return Sim.from_workload(wl, precision)


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _wall_layer(psi):
    """Nodes with psi >= 1e-2 whose 5 x 5 neighbourhood has no psi within
    1e-6 of 1 (reported beside the whole-field error). The wetting term is
    weighted by |grad psi|, whose derivative grad psi / |grad psi| is of
    unit size however small grad psi is; a float32 psi would make grad psi
    exactly 0 where psi is within float32 rounding of 1, so float32
    contexts take that derivative from the float64 geometry."""
    near_one = np.zeros(psi.shape, bool)
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            near_one |= np.roll(np.roll(psi, dy, 0), dx, 1) > 1.0 - 1e-6
    return (psi >= 1e-2) & ~near_one


CASES = [
    ("n2_20x70", lambda: W.random_small(2, 2, (20, 70), seed=1), 10, 3),
    ("n3_force_13x66", lambda: W.random_small(
        2, 3, (13, 66), seed=5, force=[2e-5, -1e-5], accel=[0.0, 1e-5]), 8, 5),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_adjoint_matches_oracle(case, precision):
    from oracle import adjoint as A
    import oracle
    name, make, steps, interval = [c for c in CASES if c[0] == case][0]
    wl = make()
    print("case", name, wl.shape, precision, flush=True)
    sim = _sim(wl, precision)
    st0 = gpu_state_to_oracle(wl, sim)
    J, gc, gp = sim.adjoint(steps, interval, phase=0)
    sim.close()
    prm, _, _ = oracle.from_workload(wl)
    Jo, gco, gpo = A.gradient(prm, wl.psi, wl.cos_theta_iN, st0, steps)
    ec, ep = _rel(gc, gco), _rel(gp, gpo)
    m = _wall_layer(np.asarray(wl.psi))
    epm = float(np.abs(gp - gpo)[m].max() / np.abs(gpo[m]).max())
    print("J %.15f oracle %.15f | grad cos %.2e grad psi %.2e (wall layer: "
          "%.2e)" % (J, Jo, ec, ep, epm), flush=True)
    if precision == "fp64":
        assert abs(J - Jo) <= 1e-13 * abs(Jo)
        assert ec < 1e-9 and ep < 1e-9
    else:
        assert abs(J - Jo) <= 1e-6 * abs(Jo)
        assert ec < 1e-4 and ep < 1e-4


def test_adjoint_matches_finite_differences():
    wl = W.random_small(2, 2, (40, 64), seed=7)
    steps, interval = 60, 16
    sim = _sim(wl)
    state = sim.save()
    J, gc, gp = sim.adjoint(steps, interval)
    rng = np.random.default_rng(11)

    def value(psi, cos):
        sim.init_geometry(psi, cos)
        sim.load(state)
        from paper_2311_10314_amd.ddcc import centroid_weight
        return sim.adjoint(steps, 10**6, weight=centroid_weight(wl.shape))[0]

    psi0 = np.asarray(wl.psi)
    cos0 = np.asarray(wl.cos_theta_iN).reshape(gc.shape)
    for which, g in (("cos", gc), ("psi", gp)):
        v = rng.standard_normal(g.shape)
        if which == "psi":
            # keep psi + h v inside [0, 1]: no change where psi is 0 or 1
            v = v * 4.0 * psi0 * (1.0 - psi0)

        def central(h):
            if which == "cos":
                return (value(psi0, cos0 + h * v) -
                        value(psi0, cos0 - h * v)) / (2 * h)
            return (value(psi0 + h * v, cos0) -
                    value(psi0 - h * v, cos0)) / (2 * h)

        h = 2e-4
        fd = (4.0 * central(h / 2) - central(h)) / 3.0
        ad = float((g * v).sum())
        print("%s: adjoint %.12e finite differences %.12e rel %.1e" % (
            which, ad, fd, abs(fd - ad) / abs(ad)), flush=True)
        assert abs(fd - ad) <= 1e-6 * abs(ad)
    sim.close()


def test_interval_does_not_change_the_gradient():
    wl = W.random_small(2, 2, (20, 70), seed=1)
    out = []
    for interval in (1, 4, 100):
        sim = _sim(wl)
        out.append(sim.adjoint(9, interval))
        sim.close()
    for J, gc, gp in out[1:]:
        assert J == out[0][0]
        assert np.array_equal(gc, out[0][1]) and np.array_equal(gp, out[0][2])


def test_constant_weight_gives_zero_gradient():
    wl = W.random_small(2, 3, (13, 66), seed=5)
    sim = _sim(wl)
    J, gc, gp = sim.adjoint(6, 4, phase=1, weight=np.full(wl.shape, 2.0))
    sim.close()
    assert J == pytest.approx(2.0, rel=1e-14)
    assert np.abs(gc).max() < 1e-14 and np.abs(gp).max() < 1e-14


def test_context_left_at_the_final_level():
    wl = W.random_small(2, 2, (20, 70), seed=1)
    a = _sim(wl)
    a.adjoint(7, 3)
    b = _sim(wl)
    b.step(7)
    assert a.time == b.time == 7
    from tests.helpers import unpack_state
    sa, sb = unpack_state(a, a.save()), unpack_state(b, b.save())
    for key in ("f", "g", "hist", "T"):
        assert np.array_equal(sa[key], sb[key])
    a.close()
    b.close()


def test_autograd_bridge():
    import torch

    from paper_2311_10314_amd.autograd import weighted_phase_objective
    wl = W.random_small(2, 2, (20, 70), seed=1)
    sim = _sim(wl)
    state = sim.save()
    cos = torch.tensor(np.asarray(wl.cos_theta_iN).reshape((1,) + wl.shape),
                       requires_grad=True)
    psi = torch.tensor(np.asarray(wl.psi), requires_grad=True)
    J = weighted_phase_objective(cos, psi, sim, state, 6, interval=4)
    (2.0 * J).backward()
    ref = _sim(wl)
    Jr, gc, gp = ref.adjoint(6, 4)
    assert J.item() == Jr
    assert np.array_equal(cos.grad.numpy(), 2.0 * gc)
    assert np.array_equal(psi.grad.numpy(), 2.0 * gp)
    sim.close()
    ref.close()


def test_unsupported_contexts_are_refused():
    from paper_2311_10314_amd.ddcc import DDCC_E_UNSUPPORTED, DDCCError
    wl = W.random_small(2, 2, (20, 70), seed=1)
    s = _sim(wl, "fp16")
    with pytest.raises(DDCCError) as e:
        s.adjoint(2, 1)
    assert e.value.code == DDCC_E_UNSUPPORTED
    s.close()
    two = W.wavy_channel_2d(n=48)
    s = _sim(two)
    with pytest.raises(DDCCError) as e:
        s.adjoint(2, 1)
    assert e.value.code == DDCC_E_UNSUPPORTED
    s.close()


def test_adjoint_channel_full_size():
    """The adjoint workload at its full size: 256 x 256 wavy channel, 2000
    steps, checkpoints every 100. FP64 gradients against Richardson central
    differences of the FP64 forward along smooth random directions (target
    1e-4); FP32 gradients against the FP64 ones."""
    from paper_2311_10314_amd.ddcc import Sim
    wl = W.adjoint_channel_2d(256)
    steps, interval = 2000, 100
    print("adjoint channel 256x256, %d steps" % steps, flush=True)
    sim = Sim.from_workload(wl, "fp64")
    state = sim.save()
    J, gc, gp = sim.adjoint(steps, interval)
    psi0 = np.asarray(wl.psi)
    cos0 = np.asarray(wl.cos_theta_iN).reshape(gc.shape)

    def value(psi, cos):
        sim.init_geometry(psi, cos)
        sim.load(state)
        sim.step(steps)
        return sim.objective()

    assert value(psi0, cos0) == J
    directions = {
        "cos": W.smooth_angle_field(wl.shape, 7, lo=-1.0, hi=1.0)[None],
        "psi": W.smooth_angle_field(wl.shape, 8, lo=-1.0, hi=1.0)
        * 4.0 * psi0 * (1.0 - psi0)}
    for which, g in (("cos", gc), ("psi", gp)):
        v = directions[which]

        def central(h):
            if which == "cos":
                return (value(psi0, cos0 + h * v) -
                        value(psi0, cos0 - h * v)) / (2 * h)
            return (value(psi0 + h * v, cos0) -
                    value(psi0 - h * v, cos0)) / (2 * h)

        h = 2e-3
        fd = (4.0 * central(h / 2) - central(h)) / 3.0
        ad = float((g * v).sum())
        print("%s: adjoint %.10e finite differences %.10e rel %.1e" % (
            which, ad, fd, abs(fd - ad) / abs(ad)), flush=True)
        assert abs(fd - ad) <= 1e-4 * abs(ad)
    sim.close()
    s32 = Sim.from_workload(wl, "fp32")
    J32, gc32, gp32 = s32.adjoint(steps, interval)
    s32.close()
    ec, ep = _rel(gc32, gc), _rel(gp32, gp)
    m = _wall_layer(psi0)
    epm = float(np.abs(gp32 - gp)[m].max() / np.abs(gp[m]).max())
    print("fp32 vs fp64: J %.3e grad cos %.2e grad psi %.2e (wall layer, "
          "%d nodes: %.2e)" % (abs(J32 - J) / abs(J), ec, ep, m.sum(), epm),
          flush=True)
    k = np.unravel_index(np.argmax(np.abs(gp32 - gp)), gp.shape)
    print("largest psi-gradient difference at %s: psi %.17g (float32 %r), "
          "fp64 %.6e fp32 %.6e" % (k, psi0[k], float(np.float32(psi0[k])),
                                   gp[k], gp32[k]), flush=True)
    assert abs(J32 - J) <= 1e-5 * abs(J)
    assert ec < 1e-4 and ep < 1e-4
