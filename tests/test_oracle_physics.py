"""Physics pins of the FP64 oracle: results the paper and the continuum
model fix independently of any implementation (no GPU needed).

Each test names the mistakes it is built to catch. Sizes are small so the
whole file runs in about a minute and a half on one core.
"""
import math
import warnings

import numpy as np
import pytest

from oracle import dd_cclb as O
from paper_2311_10314_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def params_2d(N=2, **kw):
    p = W.default_params(2, N)
    p.update(kw)
    return O.Params(dim=2, lattice_f="D2Q9", lattice_g="D2Q9", **p)


def open_box(prm, shape):
    """psi = 1 everywhere, wetting angles 90 deg (no wall)."""
    psi = np.ones(shape)
    return O.Geometry(prm, psi, np.zeros((prm.N - 1,) + shape))


# ---------------------------------------------------------------------------
# Exact invariants
# ---------------------------------------------------------------------------
def test_mass_of_every_phase_is_conserved():
    """Sum over nodes and populations of f^i is invariant: the equilibrium
    carries phi C_i as its zeroth moment and the source has zero zeroth
    moment (Appendix B), collision keeps the zeroth moment (s0 row), and
    periodic pull streaming only moves populations. Catches a source with a
    non-zero sum, a non-conserving collision row or a lost population."""
    wl = W.random_small(2, 3, (20, 24), seed=5)
    prm = O.Params(dim=2, lattice_f=wl.lattice_f, lattice_g=wl.lattice_g,
                   **wl.params)
    geo = O.Geometry(prm, wl.psi, wl.cos_theta_iN)
    st = O.init_state(prm, geo, wl.C0, wl.u0, wl.P0)
    m0 = O.mass(st)
    st = O.run(prm, geo, st, 300)
    m1 = O.mass(st)
    assert np.all(np.isfinite(m1))
    assert np.max(np.abs(m1 - m0) / np.abs(m0)) < 1e-13


def test_uniform_state_is_invariant():
    """A uniform mixture moving at a uniform velocity in an open box is an
    exact solution: every gradient, source and time derivative vanishes,
    so one hundred steps change nothing beyond rounding (Galilean and
    trivial-state check of eqs. 3.5-3.12)."""
    n = 12
    prm = params_2d(N=3, rho=[1.0, 4.0, 9.0], nu=[0.1, 0.2, 0.05])
    geo = open_box(prm, (n, n))
    C0 = np.array([np.full((n, n), v) for v in (0.2, 0.3, 0.5)])
    u0 = np.array([np.full((n, n), 0.03), np.full((n, n), -0.02)])
    st0 = O.init_state(prm, geo, C0, u0)
    st = O.run(prm, geo, st0, 100)
    assert np.max(np.abs(st.f - st0.f)) < 1e-14
    assert np.max(np.abs(st.g - st0.g)) < 1e-14
    C, u, P = O.moments(prm, geo, st)
    assert np.max(np.abs(u[0] - 0.03)) < 1e-14
    assert np.max(np.abs(u[1] + 0.02)) < 1e-14


def test_reduction_consistency_absent_phase_stays_zero():
    """With the third phase absent at t = 0, the N = 3 model reduces to the
    N = 2 one: mu_3 vanishes identically because g' is odd about 1/2, the
    Laplacians sum to that of a constant and cos(theta_ij) is antisymmetric
    (eqs. 2.9, 2.14), so phi C_3 stays zero and phases 1, 2 follow the N = 2
    run. The N = 3 wall angles theta_13 = 60, theta_23 = 90 give
    cos theta_12 = 1/2 through eq. (2.9). Catches index mistakes in the
    N-phase sums, in the mobility matrix and in eq. (2.9)."""
    n = 40
    x, y = W._grid((n, n))
    psi = W.psi_from_distance(W.periodic_distance((x, y), (n / 2, n / 2),
                                                  (n, n)) - 8.0)
    C1 = W.droplet(W.periodic_distance((x, y), (n / 2, n / 2 + 11), (n, n)),
                   8.0, 5.0)
    p2 = params_2d(N=2, rho=[1.0, 3.0], nu=[0.1, 0.2])
    g2 = O.Geometry(p2, psi, np.full((1, n, n), 0.5))
    s2 = O.init_state(p2, g2, np.array([C1, 1 - C1]))
    p3 = params_2d(N=3, rho=[1.0, 3.0, 7.0], nu=[0.1, 0.2, 0.3])
    g3 = O.Geometry(p3, psi, np.array([np.full((n, n), 0.5),
                                       np.zeros((n, n))]))
    s3 = O.init_state(p3, g3, np.array([C1, 1 - C1, np.zeros((n, n))]))
    s2 = O.run(p2, g2, s2, 200)
    s3 = O.run(p3, g3, s3, 200)
    Ca, ua, Pa = O.moments(p2, g2, s2)
    Cb, ub, Pb = O.moments(p3, g3, s3)
    assert np.abs(s3.f[2].sum(axis=0)).max() < 1e-14
    assert np.abs(Ca[0] - Cb[0]).max() < 1e-12
    assert np.abs(ua - ub).max() < 1e-14
    assert np.abs(ua).max() > 1e-5          # the flow is not trivial


# ---------------------------------------------------------------------------
# Closed forms of the continuum model
# ---------------------------------------------------------------------------
def test_tanh_profile_has_vanishing_chemical_potential():
    """A flat two-phase interface C = (1 + tanh(2 z / eps)) / 2 is the
    equilibrium of the free energy of Section 2.1 only if
    beta = 3 sigma / eps and kappa = 3 eps sigma / 4 (then
    2 beta g'(C) = (3/4) eps sigma C''). The discrete mu of that profile
    must vanish to second order in 1/eps. Catches the printed inverted
    beta, a wrong gradient coefficient and a wrong div(psi grad C)
    stencil."""
    ratios = []
    for eps in (4.0, 8.0, 16.0):
        prm = params_2d(eps=eps)
        nx, ny = 4, 256
        y = np.arange(ny)[:, None] * np.ones((1, nx))
        C1 = 0.25 * (1 + np.tanh(2 * (y - ny / 4) / eps)) * \
            (1 + np.tanh(2 * (3 * ny / 4 - y) / eps))
        geo = open_box(prm, (ny, nx))
        q = O._phase_fields(prm, geo, np.array([C1, 1 - C1]))
        ratios.append(np.abs(q["mu"][0]).max() / (0.01 / eps))
    assert ratios[0] < 0.2
    assert ratios[0] / ratios[1] > 3.5 and ratios[1] / ratios[2] > 3.5


@pytest.mark.parametrize("R", [8.0, 12.0])
def test_laplace_law_static_droplet(R):
    """Pressure jump across a static 2D droplet: P_in - P_out = sigma / R
    (Section 2.1 with the potential-form force of eq. 3.13 and the
    pressure recovery of eq. 19). Started from the jump, averaged over the
    last 200 of 800 steps. Catches wrong eq. (19) constants and a wrong
    force."""
    n, sigma = 48, 0.01
    prm = params_2d()
    geo = open_box(prm, (n, n))
    x, y = W._grid((n, n))
    C1 = W.droplet(W.periodic_distance((x, y), (n / 2, n / 2), (n, n)), R,
                   prm.eps)
    st = O.init_state(prm, geo, np.array([C1, 1 - C1]), None,
                      sigma / R * C1)
    st = O.run(prm, geo, st, 600)
    jumps = []
    for _ in range(20):
        st = O.run(prm, geo, st, 10)
        C, u, P = O.moments(prm, geo, st)
        jumps.append(P[n // 2 - 2:n // 2 + 3, n // 2 - 2:n // 2 + 3].mean()
                     - P[:3, :3].mean())
    assert abs(np.mean(jumps) * R / sigma - 1.0) < 0.04


def _decay_rate(u0, proj, steps=300, n=32, nu=0.1):
    prm = params_2d(nu=[nu, nu])
    geo = open_box(prm, (n, n))
    C0 = np.array([np.ones((n, n)), np.zeros((n, n))])
    st = O.init_state(prm, geo, C0, u0)
    amp = []
    for _ in range(steps):
        st = O.step(prm, geo, st)
        u = O.moments(prm, geo, st)[1]
        amp.append((u[0] * proj).sum() / (proj * proj).sum())
    t = np.arange(1, steps + 1)
    return -np.polyfit(t[50:], np.log(np.array(amp[50:])), 1)[0]


def test_shear_wave_decay_pins_s22():
    """u_x = U sin(k y) decays as exp(-nu k^2 t): only the off-diagonal
    second-order moment carries the shear, so this pins
    nu = (1/s22 - 1/2) c_s^2 (eq. 16)."""
    n = 32
    k = 2 * math.pi / n
    y = np.arange(n)[:, None] * np.ones((1, n))
    u0 = np.zeros((2, n, n))
    u0[0] = 1e-3 * np.sin(k * y)
    rate = _decay_rate(u0, np.sin(k * y))
    assert abs(rate / (0.1 * k * k) - 1) < 0.01


def test_taylor_green_decay_pins_s21():
    """The Taylor-Green vortex decays as exp(-2 nu k^2 t); it strains the
    diagonal second-order moments too, so it pins
    nu = (1/s21 - 1/2)(c^2 - c_s^2)/2 (eq. 16): with s21 taken from the
    s22 relation the rate is off by about a quarter."""
    n = 32
    k = 2 * math.pi / n
    x = np.arange(n)[None, :] * np.ones((n, 1))
    y = np.arange(n)[:, None] * np.ones((1, n))
    u0 = np.zeros((2, n, n))
    u0[0] = 1e-3 * np.sin(k * x) * np.cos(k * y)
    u0[1] = -1e-3 * np.cos(k * x) * np.sin(k * y)
    rate = _decay_rate(u0, np.sin(k * x) * np.cos(k * y))
    assert abs(rate / (0.2 * k * k) - 1) < 0.01


def _channel(h, ny, nx, rho, nu, G, C1, steps, lam=0.5):
    prm = params_2d(rho=list(rho), nu=list(nu), force=[G, 0.0], lam=lam)
    y = np.arange(ny)[:, None] * np.ones((1, nx)) + 0.0
    psi = W.psi_from_distance(h - np.abs(y - ny / 2))
    geo = O.Geometry(prm, psi, np.zeros((1, ny, nx)))
    st = O.init_state(prm, geo, np.array([C1, 1 - C1]))
    st = O.run(prm, geo, st, steps)
    C, u, P = O.moments(prm, geo, st)
    return prm, psi, u


def test_channel_flow_viscosity_and_force_balance():
    """Body-force driven flow in a psi-embedded channel (eq. 2.13c with the
    penalty of eq. 3.13). Away from the diffuse walls the profile is a
    parabola with u'' = -G / (rho nu); at steady state the total body force
    equals the total penalty force exactly (viscous and pressure forces sum
    to zero on a periodic box). Catches a wrong force density, a wrong
    penalty and a wrong viscosity relation."""
    ny, nx, h, nu, G = 40, 4, 12, 0.5, 1e-5
    prm, psi, u = _channel(h, ny, nx, (1.0, 1.0), (nu, nu), G,
                           np.ones((ny, nx)), 1500)
    yy = np.arange(ny) - ny / 2
    core = np.abs(yy) <= 4
    a = np.polyfit(yy[core], u[0][core, 0], 2)[0]
    assert abs(a / (-G / (2 * nu)) - 1) < 0.01
    balance = (psi * G).sum() / ((1 - psi) * prm.lam * u[0]).sum()
    assert abs(balance - 1) < 1e-4


def test_layered_channel_per_phase_viscosity():
    """Two layers (phase 1 above the mid-plane, phase 2 below) with dynamic
    viscosities mu_k = rho_k nu_k differing by 3x: each bulk layer is a
    parabola with u'' = -G / mu_k (the linear mixing of rho and nu,
    Section 2.2, and the local rates of eq. 16)."""
    ny, nx, h, G = 52, 4, 18, 1e-5
    rho, nu = (1.0, 2.0), (0.3, 0.45)
    yy = np.arange(ny)[:, None] * np.ones((1, nx)) - ny / 2
    C1 = 0.5 * (1 + np.tanh(2 * yy / 5.0))
    prm, psi, u = _channel(h, ny, nx, rho, nu, G, C1, 3000)
    y1 = np.arange(ny) - ny / 2
    for k, sel in ((0, (y1 >= 5) & (y1 <= 10)), (1, (y1 >= -10) & (y1 <= -5))):
        a = np.polyfit(y1[sel], u[0][sel, 0], 2)[0]
        assert abs(a / (-G / (2 * rho[k] * nu[k])) - 1) < 0.03, k


# ---------------------------------------------------------------------------
# Wetting (eqs. 2.9, 2.14)
# ---------------------------------------------------------------------------
def _contour(C, ymin):
    pts = []
    ny, nx = C.shape
    for j in range(ny - 1):
        for i in range(nx - 1):
            for dj, di in ((0, 1), (1, 0)):
                a, b = C[j, i] - 0.5, C[j + dj, i + di] - 0.5
                if a * b <= 0 and a != b and j > ymin:
                    t = a / (a - b)
                    pts.append((i + t * di, j + t * dj))
    return np.array(pts)


def _cap_angle(theta_init, theta_wall, steps=1000, nx=64, ny=40, yw=6.0,
               R=14.0):
    """Droplet cap on the flat wall y = yw of a psi-embedded slab; returns
    the contact angle (inside the droplet) of the circle fitted to the
    C_1 = 1/2 contour after `steps` steps."""
    prm = params_2d()
    x, y = W._grid((ny, nx))
    psi = W.psi_from_distance(np.minimum(y - yw, (ny - yw) - y))
    geo = O.Geometry(prm, psi, np.full((1, ny, nx),
                                       math.cos(math.radians(theta_wall))))
    yc = yw - R * math.cos(math.radians(theta_init))
    C1 = W.droplet(np.sqrt((x - nx / 2) ** 2 + (y - yc) ** 2), R, prm.eps)
    st = O.init_state(prm, geo, np.array([C1, 1 - C1]))
    st = O.run(prm, geo, st, steps)
    C = O.moments(prm, geo, st)[0][0]
    p = _contour(C, yw + 3)
    A = np.c_[2 * p[:, 0], 2 * p[:, 1], np.ones(len(p))]
    (xc, ycf, c), *_ = np.linalg.lstsq(A, (p ** 2).sum(axis=1), rcond=None)
    Rf = math.sqrt(c + xc * xc + ycf * ycf)
    return math.degrees(math.acos(max(-1.0, min(1.0, (yw - ycf) / Rf))))


def test_contact_angle_flat_wall():
    """A cap started at the wall angle keeps it; caps started at 90 deg move
    toward 60 or 120 deg. With the wetting term doubled, halved or of the
    wrong sign the 60-deg cap leaves the 2-deg band or the 90-deg caps move
    the wrong way (checked by planting those mistakes)."""
    assert abs(_cap_angle(60, 60) - 60) < 2.0
    assert _cap_angle(90, 60) < 90 - 1.5
    assert _cap_angle(90, 120) > 90 + 1.5


# ---------------------------------------------------------------------------
# Several walls (Section 4.5): psi = prod_k psi_k, wetting per wall
# ---------------------------------------------------------------------------
def _band_walls(ny, nx, y_bottom, y_top, thick=16.0):
    """Two solid bands 'thick' cells thick: band 1 ends at y_bottom (its top
    face is the channel's bottom wall), band 2 starts at y_top. Each band's
    psi_k is smooth and periodic on its own (fluid on both sides of both
    bands), as a wall's characteristic function must be."""
    x, y = W._grid((ny, nx))
    shape = (ny, nx)
    c1 = (0.0, y_bottom - thick / 2)
    c2 = (0.0, y_top + thick / 2)
    d1 = np.abs(W._periodic_delta(y, c1[1], ny)) - thick / 2
    d2 = np.abs(W._periodic_delta(y, c2[1], ny)) - thick / 2
    return x, y, W.psi_from_distance(d1), W.psi_from_distance(d2)


def test_two_separated_walls_with_one_angle_match_one_wall():
    """Two solid bands 16 cells thick, 36 and 28 cells apart, with the same
    angle: the per-wall sum cos theta |grad psi_1| + cos theta |grad psi_2|
    equals cos theta |grad(psi_1 psi_2)| wherever the walls' tails do not
    overlap, so the two descriptions evolve alike (to the exp(-24)-small
    overlap); the droplet stays within one band and the channel."""
    ny, nx, yw = 96, 48, 26.0
    x, y, pb, pt = _band_walls(ny, nx, yw, 62.0)
    prm = params_2d()
    ct = np.full((1, ny, nx), math.cos(math.radians(60.0)))
    C1 = W.droplet(np.sqrt((x - nx / 2) ** 2 + (y - yw) ** 2), 12.0, prm.eps)
    C0 = np.array([C1, 1 - C1])
    g1 = O.Geometry(prm, pb * pt, ct)
    g2 = O.Geometry(prm, None, None, walls=[(pb, ct), (pt, ct)])
    assert np.array_equal(g1.psi, g2.psi)
    s1 = O.run(prm, g1, O.init_state(prm, g1, C0), 100)
    s2 = O.run(prm, g2, O.init_state(prm, g2, C0), 100)
    Ca, ua, _ = O.moments(prm, g1, s1)
    Cb, ub, _ = O.moments(prm, g2, s2)
    assert np.abs(Ca - Cb).max() < 1e-9
    # the walls' tails meet in the 28-cell channel across the periodic
    # boundary (weights differ by ~4e-6 there), which shows up in u at the
    # 1e-8 level
    assert np.abs(ua - ub).max() < 1e-7 * np.abs(ua).max()


def test_each_wall_wets_with_its_own_angle():
    """A 90-deg cap on the bottom wall of a channel whose bottom wall has
    60 deg and top wall 120 deg spreads (its angle falls); with the two
    walls' angles swapped it contracts. Taking the other wall's angle, or
    one angle for both, breaks one of the two."""
    ny, nx, yw, R = 80, 64, 22.0, 12.0
    x, y, pb, pt = _band_walls(ny, nx, yw, 52.0)
    prm = params_2d()
    C1 = W.droplet(np.sqrt((x - nx / 2) ** 2 + (y - yw) ** 2), R, prm.eps)
    C0 = np.array([C1, 1 - C1])
    angles = []
    for th_b, th_t in ((60.0, 120.0), (120.0, 60.0)):
        cb = np.full((1, ny, nx), math.cos(math.radians(th_b)))
        ctp = np.full((1, ny, nx), math.cos(math.radians(th_t)))
        geo = O.Geometry(prm, None, None, walls=[(pb, cb), (pt, ctp)])
        st = O.run(prm, geo, O.init_state(prm, geo, C0), 1000)
        C = O.moments(prm, geo, st)[0][0]
        p = _contour(C, yw + 3)
        A = np.c_[2 * p[:, 0], 2 * p[:, 1], np.ones(len(p))]
        (xc, ycf, c), *_ = np.linalg.lstsq(A, (p ** 2).sum(axis=1),
                                           rcond=None)
        Rf = math.sqrt(c + xc * xc + ycf * ycf)
        angles.append(math.degrees(math.acos(max(-1.0, min(1.0,
                                                           (yw - ycf) / Rf)))))
    assert angles[0] < 90 - 1.5 and angles[1] > 90 + 1.5, angles


def test_d3q7_and_d3q15_phase_sets_agree():
    """The paper's 3D phase lattice D3Q7 and D3Q15 solve the same
    phase-field equation (the moment identities of Appendix B hold for
    both), so a droplet advected at u = 0.01 for 60 steps ends up alike:
    the difference is a small part of the change of C (truncation-level),
    which a wrong D3Q7 weight, velocity or relaxation row would not give."""
    n = 20
    shape = (n, n, n)
    x, y, z = W._grid(shape)
    C1 = W.droplet(W.periodic_distance((x, y, z), (n / 2, n / 2, n / 2),
                                       shape), 6.0, 5.0)
    res = {}
    for lf in ("D3Q7", "D3Q15"):
        p = W.default_params(3, 2, d0=0.3, rho=[1.0, 2.0])
        prm = O.Params(dim=3, lattice_f=lf, lattice_g="D3Q19", **p)
        geo = O.Geometry(prm, np.ones(shape), np.zeros((1,) + shape))
        u0 = np.zeros((3,) + shape)
        u0[0] = 0.01
        st = O.init_state(prm, geo, np.array([C1, 1 - C1]), u0)
        res[lf] = O.moments(prm, geo, O.run(prm, geo, st, 60))
    change = np.abs(res["D3Q15"][0][0] - C1).max()
    assert change > 0.05
    assert np.abs(res["D3Q7"][0] - res["D3Q15"][0]).max() < 0.1 * change
    assert np.abs(res["D3Q7"][1] - res["D3Q15"][1]).max() < \
        0.05 * np.abs(res["D3Q15"][1]).max()


def _curved_cap_angle(theta, steps=1500, n=96, Rs=20.0, Rl=16.0):
    """Droplet on a psi-embedded disk (the geometry of the 128^2 disk case,
    scaled down): the droplet of radius Rl starts as the circle that meets
    the disk of radius Rs at the angle theta, the wall has angle theta, and
    after `steps` steps a circle is fitted to the C_1 = 1/2 contour away
    from the wall. The contact angle follows from the triangle of the two
    centres and a contact point (law of cosines):
    cos theta = (Rs^2 + R^2 - d^2) / (2 Rs R), d the centre distance."""
    prm = params_2d()
    x, y = W._grid((n, n))
    c = (n / 2, n / 2 - 10)
    ds = W.periodic_distance((x, y), c, (n, n))
    psi = W.psi_from_distance(ds - Rs)
    geo = O.Geometry(prm, psi, np.full((1, n, n),
                                       math.cos(math.radians(theta))))
    d0 = math.sqrt(Rs * Rs + Rl * Rl
                   - 2 * Rs * Rl * math.cos(math.radians(theta)))
    C1 = W.droplet(W.periodic_distance((x, y), (c[0], c[1] + d0), (n, n)),
                   Rl, prm.eps)
    st = O.run(prm, geo, O.init_state(prm, geo, np.array([C1, 1 - C1])),
               steps)
    C = O.moments(prm, geo, st)[0][0]
    far = ds > Rs + 4
    pts = []
    for j in range(n - 1):
        for i in range(n - 1):
            for dj, di in ((0, 1), (1, 0)):
                if not (far[j, i] and far[j + dj, i + di]):
                    continue
                a, b = C[j, i] - 0.5, C[j + dj, i + di] - 0.5
                if a * b <= 0 and a != b:
                    t = a / (a - b)
                    pts.append((i + t * di, j + t * dj))
    p = np.array(pts)
    A = np.c_[2 * p[:, 0], 2 * p[:, 1], np.ones(len(p))]
    (xc, yc, cc), *_ = np.linalg.lstsq(A, (p ** 2).sum(axis=1), rcond=None)
    R = math.sqrt(cc + xc * xc + yc * yc)
    d = math.hypot(xc - c[0], yc - c[1])
    cos = (Rs * Rs + R * R - d * d) / (2 * Rs * R)
    return math.degrees(math.acos(max(-1.0, min(1.0, cos))))


@pytest.mark.parametrize("theta", [60.0, 120.0])
def test_contact_angle_curved_wall(theta):
    """Young's angle on a curved psi-embedded wall (eqs. 2.9, 2.14 on a disk,
    as in Section 4.4 for a sphere): a cap started at the wall angle keeps
    it within 2 degrees after 1500 steps (measured 60.4 and 121.2; started
    at 90 degrees on these walls the caps move to 87.5 and 93.9 in the same
    time, so the wetting term, not the initial shape, holds the angle)."""
    assert abs(_curved_cap_angle(theta) - theta) < 2.0


def test_laplace_law_static_droplet_3d():
    """3D pressure jump across a static droplet: P_in - P_out = 2 sigma / R
    (Section 2.1 with the force of eq. 3.13 and the pressure of eq. 19 on
    the D3Q19 flow set, K = w_0 / (1 - d0)), with D3Q15 phase sets at the
    production rates. 24^3 box, R = 7, eps = 4, started from the jump and
    averaged over steps 100-300 (acoustic oscillations of a few percent
    remain; measured 0.974 of 2 sigma / R). Catches a wrong 3D pressure
    prefactor c_s^2 / (1 - w_0), a 2D curvature factor and a wrong 3D
    force."""
    n, R, sigma = 24, 7.0, 0.01
    shape = (n, n, n)
    p = W.default_params(3, 2)
    p.update(eps=4.0)
    prm = O.Params(dim=3, lattice_f="D3Q15", lattice_g="D3Q19", **p)
    geo = O.Geometry(prm, np.ones(shape), np.zeros((1,) + shape))
    x, y, z = W._grid(shape)
    C1 = W.droplet(W.periodic_distance((x, y, z), (n / 2, n / 2, n / 2),
                                       shape), R, prm.eps)
    st = O.init_state(prm, geo, np.array([C1, 1 - C1]), None,
                      2 * sigma / R * C1)
    st = O.run(prm, geo, st, 100)
    c = n // 2
    jumps = []
    for _ in range(20):
        st = O.run(prm, geo, st, 10)
        P = O.moments(prm, geo, st)[2]
        jumps.append(P[c - 1:c + 2, c - 1:c + 2, c - 1:c + 2].mean()
                     - P[:2, :2, :2].mean())
    assert abs(np.mean(jumps) * R / (2 * sigma) - 1.0) < 0.06


def _heavy_drop_on_wall(steps, monkeypatch=None, printed=False):
    """A droplet of density 1 in an ambient of density 0.01 (the density
    ratio of Section 4.1) half-way into a psi-embedded flat wall (90 deg),
    sigma = 0.01, m0 = 0.01, 64 x 48 box. Returns max |u| after `steps`
    steps and after half of them. printed: the volume fractions divided by
    psi (floored at 1e-6) as printed, instead of by sum_j phi C_j."""
    nx, ny, R, yw = 64, 48, 12.0, 8.0
    p = W.default_params(2, 2)
    p.update(rho=[1.0, 0.01], sigma=[[0.0, 0.01], [0.01, 0.0]], m0=0.01)
    if printed:
        p.update(psi_min=1e-6)
        monkeypatch.setattr(O, "volume_fractions",
                            lambda prm, geo, psiC: psiC / geo.psi_hat)
    prm = O.Params(dim=2, lattice_f="D2Q9", lattice_g="D2Q9", **p)
    x, y = W._grid((ny, nx))
    psi = W.psi_from_distance(np.abs(W._periodic_delta(y, yw - 8.0, ny)) - 8.0)
    geo = O.Geometry(prm, psi, np.zeros((1, ny, nx)))
    C1 = W.droplet(np.sqrt((x - nx / 2) ** 2 + (y - yw) ** 2), R, prm.eps)
    st = O.init_state(prm, geo, np.array([C1, 1 - C1]))
    m0 = O.mass(st)
    st = O.run(prm, geo, st, steps // 2)
    u_half = np.abs(O.moments(prm, geo, st)[1]).max()
    st = O.run(prm, geo, st, steps - steps // 2)
    u_end = np.abs(O.moments(prm, geo, st)[1]).max()
    return u_half, u_end, np.abs(O.mass(st) - m0) / np.abs(m0)


def test_density_ratio_100_droplet_stays_bounded():
    """Bounded state at the paper's density ratio 1 : 0.01 (Section 4.1):
    the spurious currents of a heavy droplet on a wall decay (measured
    max |u| 3.9e-5 at step 1250, 3.3e-5 at 3000) and each phase's mass is
    conserved."""
    u_half, u_end, drift = _heavy_drop_on_wall(1500)
    assert np.isfinite(u_end) and u_end < 1e-4 and u_end <= u_half
    assert drift.max() < 1e-12


def test_printed_volume_fraction_divisor_diverges(monkeypatch):
    """The same run with the printed divisor C_i = phi C_i / phi (psi_min =
    1e-6) instead of sum_j phi C_j: the currents grow (6e-4 at step 1000,
    1e-3 at 1250) and the run is non-finite by step 1750. This decides the
    reading of the volume fractions for the oracle and the library."""
    u_half, u_end, _ = _heavy_drop_on_wall(1500, monkeypatch, printed=True)
    assert not (u_end < 1e-3)
