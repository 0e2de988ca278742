"""Seeded synthetic workloads: geometry (psi), wetting angles and initial
phase fields for the DD-CCLB step.

This module only draws and shapes inputs; it holds none of the scheme's
arithmetic. Both the library's tests/bench and the reference checks take
their inputs from here. Geometry follows the paper's own constructions:
psi = (1 + tanh(2 d / eps0)) / 2 of the signed distance d (> 0 in the fluid),
products of such functions for several walls (Section 4.5), droplets with a
tanh profile of width eps (Section 2.1).

Arrays are (ny, nx) in 2D and (nz, ny, nx) in 3D (x fastest).
"""
import math

import numpy as np

PSI_WIDTH = 1.5   # psi = (1 + tanh(d / (sqrt(2) * 1.5))) / 2, i.e. eps0 = 2 sqrt(2) * 1.5


class Workload:
    """Inputs of one run. `params` holds plain numbers in lattice units."""

    def __init__(self, name, dim, shape, lattice_f, lattice_g, params, psi,
                 cos_theta_iN, C0, u0, P0, steps):
        self.name = name
        self.dim = dim
        self.shape = tuple(shape)
        self.lattice_f = lattice_f
        self.lattice_g = lattice_g
        self.params = params
        self.psi = psi
        self.cos_theta_iN = cos_theta_iN
        self.C0 = C0
        self.u0 = u0
        self.P0 = P0
        self.steps = steps
        self.walls = None    # several walls: [(psi_k, cos theta^k_iN)]

    @property
    def nphase(self):
        return self.C0.shape[0]

    @property
    def nodes(self):
        return int(np.prod(self.shape))


def _grid(shape):
    """Coordinate arrays (x, y[, z]) of a grid of the given array shape."""
    axes = [np.arange(n, dtype=np.float64) for n in shape]
    mesh = np.meshgrid(*axes, indexing="ij")
    return tuple(reversed(mesh))   # x, y, (z)


def _periodic_delta(a, b, n):
    d = a - b
    return d - n * np.round(d / n)


def periodic_distance(coords, centre, shape):
    """Minimum-image Euclidean distance from `centre` (x, y[, z])."""
    sizes = tuple(reversed(shape))
    acc = 0.0
    for xa, ca, n in zip(coords, centre, sizes):
        acc = acc + _periodic_delta(xa, ca, n) ** 2
    return np.sqrt(acc)


def psi_from_distance(d, width=PSI_WIDTH):
    """Smooth characteristic function of the fluid region,
    (1 + tanh(x)) / 2 with x = d / (sqrt(2) width), evaluated as the equal
    logistic 1 / (1 + exp(-2 x)) so that it does not cancel to exactly 0
    a few cells inside the solid."""
    x = np.asarray(d, dtype=np.float64) / (math.sqrt(2.0) * width)
    return 1.0 / (1.0 + np.exp(np.minimum(-2.0 * x, 700.0)))


def droplet(r, radius, eps):
    """Volume fraction of a droplet: (1 + tanh(2 (R - r) / eps)) / 2."""
    return 0.5 * (1.0 + np.tanh(2.0 * (radius - r) / eps))


def default_params(dim, N, **kw):
    """Parameters shared by the workloads. The penalty coefficient of
    (1 - psi) u is 0.5 per step: the printed 1 / eps0^3 taken in lattice
    units (0.013 for eps0 = 4.2) lets an interface that touches a flat wall
    grow an instability inside the wall layer within a few hundred steps."""
    p = dict(d0=0.4, eps=5.0, eps0=2.0 * math.sqrt(2.0) * PSI_WIDTH, m0=0.05,
             rho0=1.0, psi_min=1e-30, lam=0.5,
             sigma=[[0.0 if i == j else 0.01 for j in range(N)]
                    for i in range(N)],
             rho=[1.0] * N, nu=[0.1] * N,
             s_f={"0": 1.0, "1": 10.0 / 19.0, "21": 1.2, "22": 1.2, "3": 1.2,
                  "4": 1.2},
             s_g={"0": 1.0, "1": 1.2, "3": 1.2, "4": 1.2},
             accel=[0.0] * dim, force=[0.0] * dim)
    p.update(kw)
    return p


def disk_on_droplet_2d(n=128, steps=1000, theta_deg=60.0, r_solid=30.0,
                       r_drop=20.0):
    """2D, N = 2: a solid disk at the box centre and a droplet sitting on it
    (the 128 x 128 case: R_s = 30, droplet R = 20 centred on the disk top)."""
    shape = (n, n)
    x, y = _grid(shape)
    cx = cy = n / 2.0
    s = n / 128.0
    rs = r_solid * s
    rd = r_drop * s
    d_solid = periodic_distance((x, y), (cx, cy), shape) - rs
    psi = psi_from_distance(d_solid)
    r = periodic_distance((x, y), (cx, cy + rs), shape)
    C1 = droplet(r, rd, 5.0)
    C0 = np.stack([C1, 1.0 - C1])
    ct = np.full((1,) + shape, math.cos(math.radians(theta_deg)))
    return Workload("disk_droplet_2d", 2, shape, "D2Q9", "D2Q9",
                    default_params(2, 2), psi, ct, C0, np.zeros((2,) + shape),
                    np.zeros(shape), steps)


POROUS_PSI_WIDTH = 3.0   # eps0 = 2 sqrt(2) * 3 = 8.5 cells


def porous_bands_2d(n=512, n_disks=40, steps=20000, seed=2311,
                    psi_width=POROUS_PSI_WIDTH, lam=None):
    """2D, N = 3: a periodic porous medium of non-overlapping disks (seeded
    uniform centres, radii U[10, 30] scaled with n/512), three vertical phase
    bands, per-obstacle angles theta_13, theta_23 ~ U[45, 135] deg, density
    ratios 1:10:100 and a body force density 1e-6 along x.

    The wall layer is wider than in the single-disk case (eps0 = 8.5 cells,
    within the 4-8 cell layers of the paper's runs): with a density ratio of
    100 at the walls the 4.2-cell layer is unstable. Penalty lam defaults to
    0.5 per step (the strong end of the paper's runs)."""
    rng = np.random.default_rng(seed)
    shape = (n, n)
    x, y = _grid(shape)
    s = n / 512.0
    eps0 = 2.0 * math.sqrt(2.0) * psi_width
    centres = []
    radii = []
    tries = 0
    while len(centres) < n_disks:
        tries += 1
        if tries > 200000:
            raise RuntimeError("disk packing failed")
        c = rng.uniform(0.0, n, size=2)
        r = rng.uniform(10.0, 30.0) * s
        ok = True
        for c2, r2 in zip(centres, radii):
            dx = _periodic_delta(c[0], c2[0], n)
            dy = _periodic_delta(c[1], c2[1], n)
            if math.hypot(dx, dy) < r + r2 + 2.0 * eps0:
                ok = False
                break
        if ok:
            centres.append(c)
            radii.append(r)
    theta = rng.uniform(45.0, 135.0, size=(n_disks, 2))
    psi = np.ones(shape)
    nearest = np.full(shape, -1, dtype=np.int64)
    best = np.full(shape, np.inf)
    for k, (c, r) in enumerate(zip(centres, radii)):
        dist = periodic_distance((x, y), (c[0], c[1]), shape) - r
        psi = psi * psi_from_distance(dist, psi_width)
        closer = dist < best
        best = np.where(closer, dist, best)
        nearest = np.where(closer, k, nearest)
    ct = np.stack([np.cos(np.radians(theta[nearest, 0])),
                   np.cos(np.radians(theta[nearest, 1]))])
    # three vertical bands with tanh edges at x = 0, n/3, 2n/3 (periodic)
    eps = 5.0
    edges = [0.0, n / 3.0, 2.0 * n / 3.0]
    raw = []
    for b in range(3):
        lo, hi = edges[b], edges[(b + 1) % 3] if b < 2 else float(n)
        mid = 0.5 * (lo + hi)
        half = 0.5 * (hi - lo)
        dx = np.abs(_periodic_delta(x, mid, n))
        raw.append(0.5 * (1.0 + np.tanh(2.0 * (half - dx) / eps)))
    raw = np.stack(raw)
    C0 = raw / raw.sum(axis=0, keepdims=True)
    prm = default_params(2, 3, rho=[1.0, 10.0, 100.0],
                         force=[1e-6, 0.0], eps0=eps0,
                         lam=0.5 if lam is None else lam)
    return Workload("porous_bands_2d", 2, shape, "D2Q9", "D2Q9", prm, psi,
                    ct, C0, np.zeros((2,) + shape), np.zeros(shape), steps)


def droplet_impact_sphere_3d(n=256, steps=5000):
    """3D, N = 2: a solid sphere (R = 60 at (128, 128, 100) for n = 256) and a
    droplet (R = 40 at (128, 128, 206)) moving towards it at 0.02; density
    ratio 10, theta = 90 deg; D3Q15 phase sets and a D3Q19 flow set.
    Sizes scale with n/256."""
    shape = (n, n, n)
    x, y, z = _grid(shape)
    s = n / 256.0
    sc = (128.0 * s, 128.0 * s, 100.0 * s)
    dc = (128.0 * s, 128.0 * s, 206.0 * s)
    d_solid = periodic_distance((x, y, z), sc, shape) - 60.0 * s
    psi = psi_from_distance(d_solid)
    r = periodic_distance((x, y, z), dc, shape)
    eps = 5.0
    C1 = droplet(r, 40.0 * s, eps)
    C0 = np.stack([C1, 1.0 - C1])
    u0 = np.zeros((3,) + shape)
    u0[2] = -0.02 * C1
    ct = np.zeros((1,) + shape)    # cos 90 deg
    prm = default_params(3, 2, rho=[10.0, 1.0])
    return Workload("droplet_sphere_3d", 3, shape, "D3Q15", "D3Q19", prm,
                    psi, ct, C0, u0, np.zeros(shape), steps)


def wavy_channel_2d(n=256, theta_bottom=(120.0, 60.0), theta_top=(120.0, 60.0),
                    amplitude=None, thick=None, steps=2000):
    """2D, N = 3, two walls with their own wetting angles (Section 4.5): the
    bottom wall y = n/4 + B(x) and the top wall y = 3n/4 - B(x) of a
    periodic wavy channel, B(x) = 0.05 n sin(4 pi x / n) (the paper's
    sqrt-modulated profile is not periodic). Each wall is a solid band
    `thick` cells thick (default n/6) behind its face, with its own smooth
    characteristic function psi_k and angles (theta^k_13, theta^k_23); the
    bands leave fluid on both sides (a second channel across the periodic
    boundary), so that every psi_k is smooth on the periodic box by itself.
    A compound droplet (inner phase 1 of radius n/10, outer phase 2 of radius
    n/6, phase 3 around) sits at the channel centre, pushed along x by a body
    force density. The walls are in `walls` as (psi_k, cos theta^k_iN)."""
    shape = (n, n)
    x, y = _grid(shape)
    A = 0.05 * n if amplitude is None else amplitude
    w = n / 6.0 if thick is None else thick
    B = A * np.sin(4.0 * math.pi * x / n)
    c1 = n / 4.0 + B - w / 2.0           # band 1 ends at the bottom wall
    c2 = 3.0 * n / 4.0 - B + w / 2.0     # band 2 starts at the top wall
    psi1 = psi_from_distance(np.abs(_periodic_delta(y, c1, n)) - w / 2.0)
    psi2 = psi_from_distance(np.abs(_periodic_delta(y, c2, n)) - w / 2.0)
    walls = []
    for psi_k, th in ((psi1, theta_bottom), (psi2, theta_top)):
        ct = np.stack([np.full(shape, math.cos(math.radians(t))) for t in th])
        walls.append((psi_k, ct))
    r = periodic_distance((x, y), (n / 2.0, n / 2.0), shape)
    eps = 5.0
    inner = droplet(r, n / 10.0, eps)
    outer = droplet(r, n / 6.0, eps)
    C1 = inner
    C2 = np.clip(outer - inner, 0.0, 1.0)
    C3 = 1.0 - C1 - C2
    prm = default_params(2, 3, rho=[1.0, 1.0, 0.1], force=[1e-6, 0.0])
    wl = Workload("wavy_channel_2d", 2, shape, "D2Q9", "D2Q9", prm,
                  psi1 * psi2, walls[0][1], np.stack([C1, C2, C3]),
                  np.zeros((2,) + shape), np.zeros(shape), steps)
    wl.walls = walls
    return wl


def _distance_to_curve(x, y, xc, yc, n):
    """Minimum-image distance from the nodes (x, y) to the polyline of
    samples (xc, yc) on the periodic n x n box."""
    best = np.full(x.shape, np.inf)
    for xs, ys in zip(xc, yc):
        dx = _periodic_delta(x, xs, n)
        dy = _periodic_delta(y, ys, n)
        np.minimum(best, dx * dx + dy * dy, out=best)
    return np.sqrt(best)


def smooth_angle_field(shape, seed, kmax=4, lo=60.0, hi=120.0):
    """Angles in degrees: a sum of Fourier modes with |k| <= kmax (k != 0)
    and N(0, 1) cosine and sine coefficients, mapped affinely onto
    [lo, hi]."""
    rng = np.random.default_rng(seed)
    ny, nx = shape
    x, y = _grid(shape)
    F = np.zeros(shape)
    for kx in range(-kmax, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            if (kx, ky) == (0, 0) or kx * kx + ky * ky > kmax * kmax:
                continue
            ph = 2.0 * math.pi * (kx * x / nx + ky * y / ny)
            a, b = rng.standard_normal(2)
            F += a * np.cos(ph) + b * np.sin(ph)
    return lo + (hi - lo) * (F - F.min()) / (F.max() - F.min())


def adjoint_channel_2d(n=256, steps=2000, seed=2312, force=1e-6):
    """2D, N = 2, the wavy channel of the adjoint workload: bottom wall
    y = 40 + 20 sin(2 pi x / 64) and top wall y = 216 - 20 sin(2 pi x / 64)
    (sizes scale with n / 256), one psi from the signed distance to the
    nearer wall (fluid between them, solid band across the periodic
    boundary). The wetting angle theta_12 varies per node: a smooth random
    field (Fourier modes |k| <= 4, seed 2312) mapped onto [60, 120] degrees.
    A droplet of radius 30 rests on the bottom wall with its centre 20 cells
    above the wall at x = n/2 (at the channel centre it would touch no wall
    and the objective would not depend on the angles), density ratio 1, a
    body force density `force` along x."""
    shape = (n, n)
    x, y = _grid(shape)
    s = n / 256.0
    amp, period = 20.0 * s, 64.0 * s
    xs = np.arange(0.0, n, 0.125)
    yb = 40.0 * s + amp * np.sin(2.0 * math.pi * xs / period)
    yt = 216.0 * s - amp * np.sin(2.0 * math.pi * xs / period)
    d = np.minimum(_distance_to_curve(x, y, xs, yb, n),
                   _distance_to_curve(x, y, xs, yt, n))
    ybx = 40.0 * s + amp * np.sin(2.0 * math.pi * x / period)
    ytx = 216.0 * s - amp * np.sin(2.0 * math.pi * x / period)
    inside = (y > ybx) & (y < ytx)
    psi = psi_from_distance(np.where(inside, d, -d))
    theta = smooth_angle_field(shape, seed)
    ct = np.cos(np.radians(theta))[None]
    cx = n / 2.0
    wall = 40.0 * s + amp * math.sin(2.0 * math.pi * cx / period)
    r = periodic_distance((x, y), (cx, wall + 20.0 * s), shape)
    C1 = droplet(r, 30.0 * s, 5.0)
    prm = default_params(2, 2, force=[force, 0.0])
    return Workload("adjoint_channel_2d", 2, shape, "D2Q9", "D2Q9", prm, psi,
                    ct, np.stack([C1, 1.0 - C1]), np.zeros((2,) + shape),
                    np.zeros(shape), steps)


BATCH_SIDES = (64, 96, 128, 192, 256)


def batched_instance(k, seed=2313, steps=2000):
    """Instance k of the batched workload: 2D, N = 2, grid sides drawn
    independently from BATCH_SIDES, 1-8 non-overlapping solid disks with
    radii U[0.05, 0.12] min(nx, ny), one droplet of radius U[8, 24] clear of
    the disks, wetting angle U[30, 150] deg, interface width eps = 4. Seeded
    by (seed, k), so any subset of the batch can be rebuilt alone."""
    rng = np.random.default_rng([seed, k])
    nx = int(rng.choice(BATCH_SIDES))
    ny = int(rng.choice(BATCH_SIDES))
    shape = (ny, nx)
    x, y = _grid(shape)
    m = min(nx, ny)
    eps0 = 2.0 * math.sqrt(2.0) * PSI_WIDTH
    n_disks = int(rng.integers(1, 9))
    centres, radii = [], []
    tries = 0
    while len(centres) < n_disks and tries < 20000:
        tries += 1
        c = (rng.uniform(0, nx), rng.uniform(0, ny))
        r = rng.uniform(0.05, 0.12) * m
        if all(math.hypot(_periodic_delta(c[0], c2[0], nx),
                          _periodic_delta(c[1], c2[1], ny)) >= r + r2 + 2 * eps0
               for c2, r2 in zip(centres, radii)):
            centres.append(c)
            radii.append(r)
    psi = np.ones(shape)
    for c, r in zip(centres, radii):
        psi = psi * psi_from_distance(periodic_distance((x, y), c, shape) - r)
    eps = 4.0
    R = rng.uniform(8.0, 24.0)
    R = min(R, 0.3 * m)
    best, best_c = -np.inf, (nx / 2.0, ny / 2.0)
    for _ in range(200):          # the candidate centre farthest from walls
        c = (rng.uniform(0, nx), rng.uniform(0, ny))
        gap = min([math.hypot(_periodic_delta(c[0], c2[0], nx),
                              _periodic_delta(c[1], c2[1], ny)) - r2 - R
                   for c2, r2 in zip(centres, radii)] + [np.inf])
        if gap > best:
            best, best_c = gap, c
        if gap > eps0 + eps:
            break
    C1 = droplet(periodic_distance((x, y), best_c, shape), R, eps)
    theta = rng.uniform(30.0, 150.0)
    ct = np.full((1,) + shape, math.cos(math.radians(theta)))
    prm = default_params(2, 2, eps=eps)
    return Workload("batch_%d" % k, 2, shape, "D2Q9", "D2Q9", prm, psi, ct,
                    np.stack([C1, 1.0 - C1]), np.zeros((2,) + shape),
                    np.zeros(shape), steps)


def batched_instances(count=256, seed=2313, steps=2000):
    """The batched workload: `count` independent instances (see
    batched_instance) that share N and the method parameters."""
    return [batched_instance(k, seed, steps) for k in range(count)]


def random_small(dim, N, shape, seed, lattice_f=None, lattice_g=None,
                 **params):
    """Smooth random fields on a small periodic box (used for parity of
    ragged / odd shapes): a few random solid blobs, random smooth phases
    normalised to sum 1, random angles, small random velocity."""
    rng = np.random.default_rng(seed)
    coords = _grid(shape)
    psi = np.ones(shape)
    for _ in range(2):
        c = [rng.uniform(0, n) for n in reversed(shape)]
        r = rng.uniform(2.0, max(2.5, 0.25 * min(shape)))
        psi = psi * psi_from_distance(periodic_distance(coords, c, shape) - r)
    raw = []
    for _ in range(N):
        acc = np.full(shape, 0.2)
        for _ in range(3):
            c = [rng.uniform(0, n) for n in reversed(shape)]
            r = rng.uniform(2.0, max(2.5, 0.3 * min(shape)))
            acc = acc + droplet(periodic_distance(coords, c, shape), r, 4.0)
        raw.append(acc)
    raw = np.stack(raw)
    C0 = raw / raw.sum(axis=0, keepdims=True)
    ct = rng.uniform(-0.7, 0.7, size=(N - 1,) + shape)
    u0 = rng.uniform(-0.01, 0.01, size=(dim,) + shape)
    P0 = rng.uniform(-1e-4, 1e-4, size=shape)
    if lattice_f is None:
        lattice_f = "D2Q9" if dim == 2 else "D3Q15"
    if lattice_g is None:
        lattice_g = "D2Q9" if dim == 2 else "D3Q19"
    sig = [[0.0 if i == j else 0.01 + 0.002 * (i + j) for j in range(N)]
           for i in range(N)]
    prm = default_params(dim, N, sigma=sig,
                         rho=[1.0 + 2.0 * i for i in range(N)],
                         nu=[0.1 - 0.02 * i for i in range(N)])
    prm.update(params)
    return Workload("random_%dd_n%d" % (dim, N), dim, shape, lattice_f,
                    lattice_g, prm, psi, ct, C0, u0, P0, 0)
