"""Reverse-mode derivative of the oracle time step (arXiv 2311.10314).

TEST INFRASTRUCTURE. Only tests/ may import or run this module. The product
path (the HIP library and its binding) never calls it and shares no code
with it.

What it computes. For a phase-weighted objective of the state after
`nsteps` steps,

    J = sum_x w(x) phi C_k(x) / sum_x phi C_k(x),   phi C_k = sum_p f^k_p,

(w(x) = x, the node index along x, makes J the centroid x of phase k; an
indicator w makes J the fraction of phase k inside a region), it returns

    dJ / d cos theta_iN(x)   for the per-node wetting angles of eq. (2.9),
    dJ / d psi(x)            for the smooth characteristic function,

with the initial populations and history held fixed. The derivative is taken
by reverse-mode automatic differentiation (torch autograd, float64, CPU) of
the oracle's own step: oracle.dd_cclb runs the same code on torch tensors,
so the result is the exact derivative of the oracle's discrete map up to
rounding. psi enters through psi itself, psi_hat = max(psi, psi_min),
grad psi and |grad psi| (whose derivative at grad psi = 0 is taken as 0).
One wall (a single psi with its angle field).
"""
import numpy as np

from . import dd_cclb as dd


def _torch():
    import torch
    return torch


def to_torch_state(st):
    torch = _torch()
    t = lambda a: torch.tensor(np.array(a, dtype=np.float64))
    return dd.State(t(st.f), t(st.g), t(st.X), t(st.Y), t(st.P), t(st.T))


def objective(st, phase, w):
    """J of the module docstring for a numpy or torch state."""
    psiC = st.f[phase].sum(axis=0)
    return (w * psiC).sum() / psiC.sum()


def centroid_weight(shape):
    """w(x) = x: the node index along x (array axis -1)."""
    return np.broadcast_to(np.arange(shape[-1], dtype=np.float64),
                           shape).copy()


def gradient(prm, psi, cos_theta_iN, st0, nsteps, phase=0, w=None):
    """J and its gradients with respect to cos theta_iN (shape (N - 1,) +
    grid) and psi (grid), by reverse-mode differentiation of `nsteps` oracle
    steps from the numpy state st0. w defaults to the centroid weight."""
    torch = _torch()
    psi = np.asarray(psi, dtype=np.float64)
    shape = psi.shape
    cos = np.asarray(cos_theta_iN, dtype=np.float64).reshape(
        (prm.N - 1,) + shape)
    w = centroid_weight(shape) if w is None else np.asarray(w, np.float64)
    psi_t = torch.tensor(psi, requires_grad=True)
    cos_t = torch.tensor(cos, requires_grad=True)
    geo = dd.Geometry(prm, psi_t, cos_t)
    st = to_torch_state(st0)
    for _ in range(int(nsteps)):
        st = dd.step(prm, geo, st)
    J = objective(st, phase, torch.as_tensor(w))
    J.backward()
    return (float(J.detach()), cos_t.grad.numpy().copy(),
            psi_t.grad.numpy().copy())


def value(prm, psi, cos_theta_iN, st0, nsteps, phase=0, w=None):
    """J alone from the plain numpy oracle (for finite differences)."""
    psi = np.asarray(psi, dtype=np.float64)
    w = centroid_weight(psi.shape) if w is None else np.asarray(w, np.float64)
    geo = dd.Geometry(prm, psi, cos_theta_iN)
    st = dd.run(prm, geo, st0, nsteps)
    return float(objective(st, phase, w))
