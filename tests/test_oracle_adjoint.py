"""Pins of the oracle's reverse-mode derivative (oracle.adjoint).

The gradient comes from torch autograd run through the oracle's own step
on float64 tensors. It is pinned here against things that do not use
autograd:
  * the torch path of the step reproduces the numpy path to rounding (the
    matrix products of the collision sum in another order);
  * central finite differences of the plain numpy oracle, along random
    directions, for the angle field and for psi;
  * the structure of eq. (2.14): the angles enter only multiplied by
    |grad psi|, so dJ/dcos theta vanishes exactly where grad psi = 0;
  * mass conservation: with a constant weight J is constant, so both
    gradients vanish (to rounding).
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint as A
from paper_2311_10314_amd import workloads as W

torch = pytest.importorskip("torch")


def _case(seed=1, shape=(10, 12), N=2, **params):
    wl = W.random_small(2, N, shape, seed=seed, **params)
    prm, geo, st = oracle.from_workload(wl)
    psi = np.asarray(wl.psi)
    cos = np.asarray(wl.cos_theta_iN).reshape((N - 1,) + psi.shape)
    return prm, psi, cos, st


def test_torch_path_is_the_numpy_step():
    prm, psi, cos, st = _case(seed=3, shape=(9, 11), N=3)
    geo_n = oracle.Geometry(prm, psi, cos)
    ref = oracle.run(prm, geo_n, st, 2)
    geo_t = oracle.Geometry(prm, torch.tensor(psi), torch.tensor(cos))
    got = A.to_torch_state(st)
    for _ in range(2):
        got = oracle.step(prm, geo_t, got)
    for a, b in ((got.f, ref.f), (got.g, ref.g), (got.X, ref.X),
                 (got.Y, ref.Y), (got.P, ref.P), (got.T, ref.T)):
        assert np.abs(a.numpy() - b).max() <= 1e-14 * np.abs(b).max()


@pytest.mark.parametrize("seed,N,params", [
    (1, 2, {}),
    (5, 3, {"force": [2e-5, -1e-5], "accel": [0.0, 1e-5]}),
])
def test_gradient_matches_central_differences(seed, N, params):
    steps = 5
    prm, psi, cos, st = _case(seed=seed, N=N, **params)
    J, gc, gp = A.gradient(prm, psi, cos, st, steps)
    assert J == pytest.approx(A.value(prm, psi, cos, st, steps), rel=1e-14)
    rng = np.random.default_rng(seed)

    def central(which, v, h):
        if which == "cos":
            jp = A.value(prm, psi, cos + h * v, st, steps)
            jm = A.value(prm, psi, cos - h * v, st, steps)
        else:
            jp = A.value(prm, psi + h * v, cos, st, steps)
            jm = A.value(prm, psi - h * v, cos, st, steps)
        return (jp - jm) / (2 * h)

    for base, g, which in ((cos, gc, "cos"), (psi, gp, "psi")):
        v = rng.standard_normal(base.shape)
        # Richardson extrapolation of two central differences: the h^2
        # error term cancels, leaving O(h^4) and rounding / h
        h = 2e-4
        fd = (4.0 * central(which, v, h / 2) - central(which, v, h)) / 3.0
        ad = float((g * v).sum())
        print(which, "fd %.12e ad %.12e rel %.1e" % (fd, ad,
                                                     abs(fd - ad) / abs(ad)))
        assert abs(fd - ad) <= 1e-7 * abs(ad)


def test_angle_gradient_vanishes_where_psi_is_flat():
    prm, psi, cos, st = _case(seed=2, shape=(12, 10))
    # a wall only in the lowest rows: psi = 1 exactly from row 5 up
    y = np.arange(12)[:, None] * np.ones((1, 10))
    psi = np.where(y >= 5, 1.0, W.psi_from_distance(y - 2.0))
    geo = oracle.Geometry(prm, psi, cos)
    flat = geo.abs_grad_psi == 0
    assert flat.sum() > 30
    _, gc, _ = A.gradient(prm, psi, cos, st, 3)
    assert np.all(gc[0][flat] == 0.0)
    assert np.abs(gc[0][~flat]).max() > 0


def test_constant_weight_has_no_gradient():
    prm, psi, cos, st = _case(seed=4)
    w = np.full(psi.shape, 3.0)
    J, gc, gp = A.gradient(prm, psi, cos, st, 3, w=w)
    assert J == pytest.approx(3.0, rel=1e-15)
    assert np.abs(gc).max() < 1e-14 and np.abs(gp).max() < 1e-14
