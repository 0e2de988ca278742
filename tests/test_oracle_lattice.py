"""Pins of the oracle's lattice tables, Hermite basis, collision operator and
finite-difference stencils against what the mathematics fixes (no GPU)."""
import itertools

import numpy as np
import pytest

from oracle import lattices as L
from oracle import dd_cclb as D

D0S = (0.3, 1.0 / 3.0, 0.4, 0.45)


def _valid(d0s):
    """(lattice, d0) pairs inside each lattice's positive-weight range: the
    D3Q7 rest weight 1 - 3 d0 needs d0 < 1/3."""
    return [(n, d) for n in L.NAMES for d in d0s
            if not (n == "D3Q7" and d >= 1.0 / 3.0)]


@pytest.mark.parametrize("name,d0", _valid(D0S))
def test_weights_isotropy(name, d0):
    """Section 3 lattice tables: sum w = 1 and sum w c_a c_b = d0 delta_ab;
    all but D3Q7 also give sum w c_x^2 c_y^2 = d0^2 (fourth-order isotropy)
    and odd moments vanish."""
    c = L.velocities(name).astype(float)
    w = L.weights(name, d0)
    d = c.shape[1]
    assert w.min() > 0
    assert abs(w.sum() - 1.0) < 1e-15
    for a, b in itertools.product(range(d), repeat=2):
        assert abs((w * c[:, a] * c[:, b]).sum() - d0 * (a == b)) < 1e-15
        assert abs((w * c[:, a]).sum()) < 1e-16
        for e in range(d):
            assert abs((w * c[:, a] * c[:, b] * c[:, e]).sum()) < 1e-16
    if name != "D3Q7":
        assert abs((w * c[:, 0] ** 2 * c[:, 1] ** 2).sum() - d0 * d0) < 1e-15


@pytest.mark.parametrize("name", ["D2Q9", "D3Q15", "D3Q19"])
def test_weights_are_unique_solution_of_isotropy(name):
    """Shell-constant weights are fixed by the three moment constraints; an
    independent linear solve reproduces the tabulated (or derived) values."""
    d0 = 0.37
    c = L.velocities(name)
    shells = sorted(set((c * c).sum(1)))
    A = []
    for row in ("sum", "cx2", "cx2cy2"):
        line = []
        for s in shells:
            m = (c * c).sum(1) == s
            cs = c[m].astype(float)
            if row == "sum":
                line.append(m.sum())
            elif row == "cx2":
                line.append((cs[:, 0] ** 2).sum())
            else:
                line.append((cs[:, 0] ** 2 * cs[:, 1] ** 2).sum())
        A.append(line)
    wsh = np.linalg.solve(np.array(A, float), [1.0, d0, d0 * d0])
    w = L.weights(name, d0)
    for s, ws in zip(shells, wsh):
        assert np.allclose(w[(c * c).sum(1) == s], ws, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name,d0", _valid((0.3, 0.4, 0.5)))
def test_hermite_basis_invertible(name, d0):
    lat = L.Lattice(name, d0)
    assert np.linalg.matrix_rank(lat.H) == lat.Q
    assert np.abs(lat.H @ lat.Hinv - np.eye(lat.Q)).max() < 1e-13
    # rows are Hermite polynomials: orthogonal to the constant row under w
    # for every row of order >= 1
    for k in range(1, lat.Q):
        assert abs((lat.w * lat.H[k]).sum()) < 1e-15


def test_d2q9_hermite_rows_orthogonal():
    """On D2Q9 the Hermite rows are mutually orthogonal under the weights."""
    lat = L.Lattice("D2Q9", 0.4)
    G = (lat.H * lat.w) @ lat.H.T
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() < 1e-15


@pytest.mark.parametrize("name", L.NAMES)
def test_bgk_special_case(name):
    """All rates equal to s gives Lambda = s I: the collision reduces to the
    textbook BGK update with the (1 - s/2) forcing correction."""
    d0 = 0.3
    lat = L.Lattice(name, d0)
    rng = np.random.default_rng(3)
    shape = (5, 4)
    f = rng.normal(size=(lat.Q,) + shape)
    feq = rng.normal(size=(lat.Q,) + shape)
    F = rng.normal(size=(lat.Q,) + shape)
    s = 1.37
    got = D.collide(lat, f, feq, F, [s] * lat.Q)
    want = f - s * (f - feq) + (1.0 - s / 2.0) * F
    assert np.abs(got - want).max() < 1e-13


@pytest.mark.parametrize("name", ["D2Q9", "D3Q15", "D3Q19"])
def test_collision_relaxes_each_moment_at_its_rate(name):
    """Lambda = H^-1 S H: a perturbation along Hermite row k is relaxed by
    exactly s_k (eq. 3.3)."""
    lat = L.Lattice(name, 0.4)
    rates = {"0": 1.0, "1": 1.1, "21": 1.3, "22": 1.5, "3": 1.7, "4": 1.9}
    rv = lat.rate_vector(rates)
    for k in range(lat.Q):
        mk = np.zeros(lat.Q)
        mk[k] = 1.0
        pert = lat.Hinv @ mk
        out = D.collide(lat, pert[:, None], np.zeros((lat.Q, 1)),
                        np.zeros((lat.Q, 1)), rv)[:, 0]
        assert np.allclose(lat.H @ out, (1.0 - rv[k]) * mk, atol=1e-13)


def test_stencil_symbols_2d():
    """Gradient of sin(kx) is sin(k) cos(kx) (central difference), and the
    psi = 1 divergence form gives the isotropic 9-point Laplacian symbol
    2 (cos k - 1) * (2/3 + 1/3 cos q) for sin(kx) cos(qy)-type modes."""
    n = 16
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    k = 2 * np.pi * 3 / n
    f = np.sin(k * x)
    g = D.grad(f, 2)
    assert np.abs(g[0] - np.sin(k) * np.cos(k * x)).max() < 1e-14
    assert np.abs(g[1]).max() < 1e-14
    lap = D.div_psi_grad(np.ones((n, n)), f, 2)
    assert np.abs(lap - 2.0 * (np.cos(k) - 1.0) * f).max() < 1e-13


def test_stencils_exact_on_polynomials():
    """Away from the periodic seam: gradient exact on quadratics,
    div(psi grad C) exact for psi linear and C quadratic (3D and 2D)."""
    for d in (2, 3):
        n = 12
        grids = np.meshgrid(*[np.arange(n, dtype=float)] * d, indexing="ij")
        xs = list(reversed(grids))            # x, y, (z)
        C = 0.3 * xs[0] ** 2 - 0.2 * xs[1] ** 2 + 0.1 * xs[0] * xs[1] + xs[-1]
        psi = 1.0 + 0.05 * xs[0] - 0.03 * xs[1]
        inner = tuple([slice(2, -2)] * d)
        g = D.grad(C, d)
        want_gx = 0.6 * xs[0] + 0.1 * xs[1] + (1.0 if d == 2 and False else 0)
        assert np.abs((g[0] - (0.6 * xs[0] + 0.1 * xs[1]))[inner]).max() < 1e-12
        L_ = D.div_psi_grad(psi, C, d)
        # div(psi grad C) = grad psi . grad C + psi lap C
        gxC = 0.6 * xs[0] + 0.1 * xs[1]
        gyC = -0.4 * xs[1] + 0.1 * xs[0] + (1.0 if d == 2 else 0.0)
        want = 0.05 * gxC - 0.03 * gyC + psi * (0.6 - 0.4)
        assert np.abs((L_ - want)[inner]).max() < 1e-11
        del want_gx


def test_divergence_form_sums_to_zero():
    """sum_x div(psi grad C) = 0 on a periodic box (conservative form)."""
    rng = np.random.default_rng(5)
    for shape in ((7, 9), (5, 6, 4)):
        psi = rng.uniform(0, 1, size=shape)
        C = rng.normal(size=shape)
        assert abs(D.div_psi_grad(psi, C, len(shape)).sum()) < 1e-12
