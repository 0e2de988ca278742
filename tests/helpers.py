"""Shared helpers of the test suite (no method arithmetic here)."""
import numpy as np

import oracle
from paper_2311_10314_amd import workloads as W


def rel_linf(a, b):
    """max |a - b| / max |b| (per field)."""
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


def oracle_run(wl, steps):
    prm, geo, st = oracle.from_workload(wl)
    m0 = oracle.mass(st)
    st = oracle.run(prm, geo, st, steps)
    C, u, P = oracle.moments(prm, geo, st)
    return dict(C=C, u=u, P=P, mass0=m0, mass=oracle.mass(st), state=st,
                prm=prm, geo=geo)


def small_cases():
    """Ragged shapes spanning several 64 x 8 tiles and partial tiles."""
    return [
        W.random_small(2, 2, (20, 70), seed=1),
        W.random_small(2, 3, (37, 100), seed=2),
        W.random_small(2, 4, (11, 130), seed=3),
        W.random_small(2, 2, (9, 13), seed=4),
    ]
