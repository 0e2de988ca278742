"""torch.autograd bridge to the adjoint sweep of the library (ddcc_adjoint).

`weighted_phase_objective(cos_theta, psi, sim, state, nsteps, ...)` returns
J = sum_x w(x) phi C_k(x) / sum_x phi C_k(x) after `nsteps` steps from the
checkpoint `state` (a buffer of Sim.save) as a 0-d tensor that carries
dJ/dcos_theta and dJ/dpsi back to its inputs. The forward call runs the
forward and the reverse sweep on the GPU (the gradient is computed once,
with the value); backward only scales the stored gradients by the incoming
one. Geometry and state are set on `sim` for every call, so repeated calls
with new angle fields or geometry are independent.
"""
import numpy as np
import torch

from .ddcc import centroid_weight


class _WeightedPhaseObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cos_theta, psi, sim, state, nsteps, interval, phase,
                weight):
        ct = cos_theta.detach().to("cpu", torch.float64).numpy()
        ps = psi.detach().to("cpu", torch.float64).numpy()
        sim.init_geometry(ps, ct)
        sim.load(state)
        J, gc, gp = sim.adjoint(nsteps, interval, phase, weight)
        ctx.save_for_backward(
            torch.as_tensor(gc).to(cos_theta.device, cos_theta.dtype),
            torch.as_tensor(gp).to(psi.device, psi.dtype))
        return torch.tensor(J, dtype=torch.float64, device=cos_theta.device)

    @staticmethod
    def backward(ctx, gJ):
        gc, gp = ctx.saved_tensors
        return (gJ * gc, gJ * gp, None, None, None, None, None, None)


def weighted_phase_objective(cos_theta, psi, sim, state, nsteps,
                             interval=100, phase=0, weight=None):
    """cos_theta: tensor (nphase - 1,) + shape; psi: tensor `shape`; sim: a
    2D FP64 or FP32 Sim; state: Sim.save() buffer of the initial state;
    weight: numpy array of `shape` (default: node index along x, so J is
    the centroid x of `phase`)."""
    if weight is None:
        weight = centroid_weight(tuple(psi.shape))
    return _WeightedPhaseObjective.apply(cos_theta, psi, sim, state,
                                         int(nsteps), int(interval),
                                         int(phase), np.asarray(weight))
