"""Discrete-velocity sets, weights and Hermite moment bases for the oracle.

TEST INFRASTRUCTURE. This module belongs to the FP64 reference oracle; only
tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may use it.
It shares no code with the HIP path.

Source: Liu, Zhan, Chen, Chai, Shi, arXiv 2311.10314, Section 3 (lattice
tables for D2Q9, D3Q7, D3Q15 with d0-dependent weights, d0 = c_s^2/c^2).
Lattice units throughout: dx = dt = c = 1, so c_s^2 = d0.

D3Q19 is not tabulated in the paper. Its weights here are the unique solution
of the same moment constraints the paper's tables satisfy (sum w = 1,
sum w c_x^2 = d0, sum w c_x^2 c_y^2 = d0^2, with one weight per shell).

The Hermite basis H is not written out in the paper (Section 3, eq. 3.4 only
names it). The rows used are Hermite polynomials in c with the lattice c_s^2,
ordered to match the printed relaxation matrices S:
  H_a = c_a, H_aa = c_a^2 - c_s^2, H_ab = c_a c_b.
Relaxation groups: '0' conserved-zeroth, '1' first order, '21' diagonal
second order, '22' off-diagonal second order, '3' third, '4' fourth.
"""
import numpy as np

# Velocity order is part of the population layout shared with the library's
# save/load format; only the order within each shell is a convention.
_D2Q9 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
         (1, 1), (-1, 1), (-1, -1), (1, -1)]
_FACES3 = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
_D3Q7 = [(0, 0, 0)] + _FACES3
_D3Q15 = [(0, 0, 0)] + _FACES3 + [(a, b, c) for a in (1, -1) for b in (1, -1)
                                  for c in (1, -1)]
_EDGES3 = []
for _i, _j in ((0, 1), (0, 2), (1, 2)):
    for _a in (1, -1):
        for _b in (1, -1):
            _v = [0, 0, 0]
            _v[_i] = _a
            _v[_j] = _b
            _EDGES3.append(tuple(_v))
_D3Q19 = [(0, 0, 0)] + _FACES3 + _EDGES3

NAMES = ("D2Q9", "D3Q7", "D3Q15", "D3Q19")


def velocities(name):
    """Integer velocity vectors c_p (Q x d), in units of c."""
    table = {"D2Q9": _D2Q9, "D3Q7": _D3Q7, "D3Q15": _D3Q15, "D3Q19": _D3Q19}
    return np.array(table[name], dtype=np.int64)


def weights(name, d0):
    """Weights w_p(d0), Section 3 lattice tables (D3Q19: see module doc)."""
    c = velocities(name)
    shell = (c * c).sum(axis=1)
    if name == "D2Q9":
        table = {0: (1.0 - d0) ** 2, 1: (d0 - d0 * d0) / 2.0, 2: d0 * d0 / 4.0}
    elif name == "D3Q7":
        table = {0: 1.0 - 3.0 * d0, 1: d0 / 2.0}
    elif name == "D3Q15":
        table = {0: 1.0 - 3.0 * d0 + 2.0 * d0 * d0, 1: (d0 - d0 * d0) / 2.0,
                 3: d0 * d0 / 8.0}
    elif name == "D3Q19":
        table = {0: 1.0 - 3.0 * d0 + 3.0 * d0 * d0,
                 1: (d0 - 2.0 * d0 * d0) / 2.0, 2: d0 * d0 / 4.0}
    else:
        raise ValueError(name)
    return np.array([table[int(s)] for s in shell], dtype=np.float64)


def hermite_basis(name, cs2):
    """Return (H, groups): H is the Q x Q Hermite transformation matrix whose
    rows are listed in the order of the relaxation matrix S of Section 3;
    groups[k] names the relaxation rate of row k."""
    c = velocities(name).astype(np.float64)
    x = c[:, 0]
    y = c[:, 1]
    one = np.ones_like(x)

    def h2(a):
        return a * a - cs2

    if name == "D2Q9":
        rows = [one, x, y, h2(x), h2(y), x * y, h2(x) * y, h2(y) * x,
                h2(x) * h2(y)]
        groups = ["0", "1", "1", "21", "21", "22", "3", "3", "4"]
    else:
        z = c[:, 2]
        if name == "D3Q7":
            rows = [one, x, y, z, h2(x), h2(y), h2(z)]
            groups = ["0", "1", "1", "1", "21", "21", "21"]
        elif name == "D3Q15":
            rows = [one, x, y, z, h2(x), h2(y), h2(z), x * y, x * z, y * z,
                    x * (h2(y) + h2(z)), y * (h2(x) + h2(z)),
                    z * (h2(x) + h2(y)), x * y * z,
                    h2(x) * h2(y) + h2(x) * h2(z) + h2(y) * h2(z)]
            groups = ["0", "1", "1", "1", "21", "21", "21", "22", "22", "22",
                      "3", "3", "3", "3", "4"]
        elif name == "D3Q19":
            rows = [one, x, y, z, h2(x), h2(y), h2(z), x * y, x * z, y * z,
                    h2(x) * y, h2(x) * z, h2(y) * x, h2(y) * z, h2(z) * x,
                    h2(z) * y, h2(x) * h2(y), h2(x) * h2(z), h2(y) * h2(z)]
            groups = (["0", "1", "1", "1", "21", "21", "21", "22", "22", "22"]
                      + ["3"] * 6 + ["4"] * 3)
        else:
            raise ValueError(name)
    return np.array(rows, dtype=np.float64), groups


class Lattice:
    """One velocity set at a given d0: c (Q x d), w (Q), H, H^-1, groups."""

    def __init__(self, name, d0):
        self.name = name
        self.d0 = float(d0)
        self.cs2 = float(d0)          # c_s^2 = d0 c^2 with c = 1
        self.c = velocities(name)
        self.d = self.c.shape[1]
        self.Q = self.c.shape[0]
        self.w = weights(name, d0)
        self.H, self.groups = hermite_basis(name, self.cs2)
        self.Hinv = np.linalg.inv(self.H)

    def rate_vector(self, rates):
        """Diagonal of S from a dict {'0': s0, '1': s1, '21': ..., '4': s4};
        values may be scalars or per-node arrays."""
        return [rates[g] for g in self.groups]


def stencil_lattice(d):
    """Fixed isotropic finite-difference stencil (independent of the LB d0):
    D2Q9 weights at d0 = 1/3 in 2D, D3Q19 weights at d0 = 1/3 in 3D."""
    name = "D2Q9" if d == 2 else "D3Q19"
    return velocities(name), weights(name, 1.0 / 3.0), 1.0 / 3.0
