"""torch.autograd.Function mapping the design field gamma to the window
objective J (Algorithm "Optimization iteration": forward solve to the
representative window, then the adjoint over that window).

forward: sets gamma (reset to t = 0), runs the window loop until the
consecutive-window test passes or the maximum number of windows is reached,
and returns J of that window (0-dim FP64). The window checkpoints stay in
HBM. backward: the discrete adjoint over that window, grad_out * dJ/dgamma.

The derivative is that of the window-restricted subproblem: the state
entering the representative window and the choice of the window are held
fixed (Sec. 3.2). Finite differences of Solver.replay are its check.
"""

import torch


class WindowedJ(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma, solver, max_steps):
        solver.set_gamma(gamma)
        rep = solver.forward(max_steps, stop_on_converge=True)
        if rep["windows_done"] == 0:
            raise RuntimeError("no window completed within max_steps")
        ctx.solver = solver
        ctx.window = rep["w_eff"]
        ctx.gshape = gamma.shape
        return torch.tensor(rep["J_eff"], dtype=torch.float64, device=gamma.device)

    @staticmethod
    def backward(ctx, grad_out):
        g, _ = ctx.solver.adjoint(ctx.window)
        g = g.to(grad_out.device).reshape(ctx.gshape)
        return grad_out * g, None, None


def windowed_objective(gamma, solver, max_steps):
    """J(gamma) with autograd support through the discrete adjoint."""
    return WindowedJ.apply(gamma, solver, max_steps)
