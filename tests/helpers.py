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


def gpu_state_to_oracle(wl, sim):
    """Oracle State built from a library checkpoint (populations after
    streaming, g_0 with rho0 added back, history unpacked)."""
    from oracle.dd_cclb import State
    from paper_2311_10314_amd.ddcc import streamed, unpack_state
    s = unpack_state(sim, sim.save())
    N, d = s["N"], s["dim"]
    f = np.stack([streamed(np.asarray(s["f"][i], np.float64), s["lf"])
                  for i in range(N)])
    g = streamed(np.asarray(s["g"], np.float64), s["lg"])
    g[0] += wl.params["rho0"]
    h = np.asarray(s["hist"], np.float64)
    shape = wl.shape
    X = h[:N * d].reshape((N, d) + shape)
    Y = np.zeros((d, d) + shape)
    T = np.zeros((d, d) + shape)
    o = N * d
    pairs = [(a, b) for a in range(d) for b in range(a, d)]
    for k, (a, b) in enumerate(pairs):
        Y[a, b] = h[o + k]
        Y[b, a] = h[o + k]
    P = h[o + len(pairs)].copy()
    tpairs = [(a, b) for a in range(d) for b in range(a + 1, d)]
    Tg = np.asarray(s["T"], np.float64)
    for k, (a, b) in enumerate(tpairs):
        T[a, b] = Tg[k]
        T[b, a] = -Tg[k]
    return State(f, g, X, Y, P, T)


def window_state(wl, s, center, hw):
    """Oracle State on the (2 hw + 1)^d window of nodes around `center`
    (array indices, periodic), built from an unpack_state dict s of a
    library checkpoint. The window's own periodic wrap is wrong only near
    its edge: a node's next state depends on the state within 4 nodes, so
    outputs within hw - 4 of the centre are those of the full box."""
    from oracle.dd_cclb import State
    from paper_2311_10314_amd.ddcc import streamed
    N, d = s["N"], s["dim"]
    shape = wl.shape
    pad = [(np.arange(-hw - 1, hw + 2) + c) % n for c, n in zip(center, shape)]
    sub = lambda a: a[(Ellipsis,) + np.ix_(*pad)]
    crop = (Ellipsis,) + (slice(1, -1),) * d
    f = np.stack([streamed(np.asarray(sub(s["f"][i]), np.float64), s["lf"])
                  for i in range(N)])[crop]
    g = streamed(np.asarray(sub(s["g"]), np.float64), s["lg"])[crop]
    g[0] += wl.params["rho0"]
    h = np.asarray(sub(s["hist"]), np.float64)[crop]
    wshape = h.shape[1:]
    X = h[:N * d].reshape((N, d) + wshape)
    Y = np.zeros((d, d) + wshape)
    T = np.zeros((d, d) + wshape)
    o = N * d
    pairs = [(a, b) for a in range(d) for b in range(a, d)]
    for k, (a, b) in enumerate(pairs):
        Y[a, b] = h[o + k]
        Y[b, a] = h[o + k]
    P = h[o + len(pairs)].copy()
    tpairs = [(a, b) for a in range(d) for b in range(a + 1, d)]
    Tg = np.asarray(sub(s["T"]), np.float64)[crop]
    for k, (a, b) in enumerate(tpairs):
        T[a, b] = Tg[k]
        T[b, a] = -Tg[k]
    return State(f, g, X, Y, P, T)


def window(a, center, hw):
    """The (2 hw + 1)^d periodic window of a grid array (last axes)."""
    d = len(center)
    shape = a.shape[-d:]
    idx = [(np.arange(-hw, hw + 1) + c) % n for c, n in zip(center, shape)]
    return a[(Ellipsis,) + np.ix_(*idx)]
