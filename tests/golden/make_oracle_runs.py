"""Writes the oracle's 1000-step results on the full-size 2D porous box and
the reduced 3D sphere box, which the GPU parity tests compare with (the
oracle takes minutes for these, too long to run inside a test).

Calls only oracle/ and the seeded input generators of workloads.py; the
oracle runs on float64 CPU tensors (torch), the same arithmetic as on
numpy arrays.

    python tests/golden/make_oracle_runs.py [--threads 8] [name ...]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

# name -> (workload factory, steps)
RUNS = {
    "porous512_n3_1000": (lambda W: W.porous_bands_2d(512), 1000),
    "sphere64_n2_1000": (lambda W: W.droplet_impact_sphere_3d(64), 1000),
}


def path_of(name):
    return os.path.join(HERE, name + ".npz")


def make(name, threads):
    import torch

    import oracle
    from oracle import dd_cclb as O
    from paper_2311_10314_amd import workloads as W

    torch.set_num_threads(threads)
    factory, steps = RUNS[name]
    wl = factory(W)
    prm, geo, st = oracle.from_workload(wl)
    m0 = oracle.mass(st)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    geo_t = O.Geometry(prm, t(wl.psi), t(wl.cos_theta_iN))
    st = O.State(t(st.f), t(st.g), t(st.X), t(st.Y), t(st.P), t(st.T))
    t0 = time.time()
    for k in range(steps):
        st = O.step(prm, geo_t, st)
        if (k + 1) % 100 == 0:
            print("%s: %d/%d steps, %.0f s" % (name, k + 1, steps,
                                              time.time() - t0), flush=True)
    C, u, P = O.moments(prm, geo_t, st)
    m1 = np.array([float(st.f[i].sum()) for i in range(prm.N)])
    np.savez_compressed(path_of(name), C=C.numpy(), u=u.numpy(), P=P.numpy(),
                        mass0=m0, mass=m1, steps=steps)
    print("wrote", path_of(name), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("names", nargs="*", default=sorted(RUNS))
    a = ap.parse_args(argv)
    for name in a.names:
        make(name, a.threads)


if __name__ == "__main__":
    main()
