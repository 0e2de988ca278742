"""FP64 reference oracle for the DD-CCLB step (arXiv 2311.10314).

TEST INFRASTRUCTURE ONLY: tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py are the only users. The product path (the HIP
library in paper_2311_10314_amd/ and its binding) never imports, links or
runs anything here, and this package imports nothing from it.

Every function here is pinned by a -m "not gpu" test in
tests/test_oracle_*.py against what the paper and the mathematics fix
(isotropy of the weights, the BGK special case, Appendix C's pressure
constants, mass conservation, reduction consistency, the tanh profile,
Laplace's law, Young's angle, shear-wave, Taylor-Green and layered-channel
solutions); oracle.adjoint against Richardson central differences.
"""
from . import lattices, dd_cclb  # noqa: F401
from .dd_cclb import (Params, Geometry, State, init_state, step, run,  # noqa: F401
                      macroscopic, moments, mass)


def from_workload(wl):
    """Oracle Params/Geometry/State for a workloads.Workload."""
    p = dict(wl.params)
    prm = Params(dim=wl.dim, lattice_f=wl.lattice_f, lattice_g=wl.lattice_g,
                 **p)
    geo = Geometry(prm, wl.psi, wl.cos_theta_iN, walls=wl.walls)
    st = init_state(prm, geo, wl.C0, wl.u0, wl.P0)
    return prm, geo, st
