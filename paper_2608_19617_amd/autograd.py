"""torch.autograd.Function mapping the design field gamma to the window
objective J (Algorithm "Optimization iteration": forward solve to the
representative window, then the adjoint over that window, then Eq.
sensitivity).

Two ways to run the forward, one derivative:

* from rest (``start=None``): set gamma (reset to t = 0), run the window loop
  until the consecutive-window test passes or the maximum number of windows
  is reached (Algorithm "LES solver"), and return J of that window;
* from a fixed window-start state (``start=(f, step)`` as returned by
  Solver.get_state): run exactly one window from that state with gamma and
  return its J. This is the window-restricted subproblem itself, so central
  finite differences through this form check the backward (the protocol of
  Sec. 4.2.1: same representative window, same sampling instants).

backward: the discrete adjoint over the window that forward returned
(checkpoints left in HBM by the forward), grad_out * dJ/dgamma. The state
entering the window and the choice of the window are held fixed (Sec. 3.2).
The gradient has gamma's layout: [x, y(, z)] when gamma has the grid's
shape, otherwise the library's flat node order (x fastest), reshaped to
gamma's shape, which is how Solver reads such a gamma.
"""

import torch


class WindowedJ(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma, solver, max_steps, start=None):
        solver.set_gamma(gamma)
        if start is None:
            rep = solver.forward(max_steps, stop_on_converge=True)
        else:
            f, step = start
            solver.set_state(f, step)
            rep = solver.forward(solver.w.window_len)
        if rep["windows_done"] == 0:
            raise RuntimeError("no window completed within max_steps")
        ctx.solver = solver
        ctx.window = rep["w_eff"]
        ctx.generation = solver.generation
        ctx.gshape = tuple(gamma.shape)
        ctx.grid = ctx.gshape == tuple(solver.shape)
        ctx.gdtype = gamma.dtype
        return torch.tensor(rep["J_eff"], dtype=torch.float64, device=gamma.device)

    @staticmethod
    def backward(ctx, grad_out):
        sv = ctx.solver
        if sv.generation != ctx.generation:
            raise RuntimeError("WindowedJ.backward: the solver ran again (set_gamma, reset, forward or "
                               "set_state) after this J was computed; its checkpoints belong to another "
                               "run, so the gradient of this J is no longer available")
        g, _ = sv.adjoint(ctx.window)                  # [x, y(, z)] view
        if not ctx.grid:
            g = g.permute(*range(g.ndim - 1, -1, -1)).reshape(-1)   # flat node order, x fastest
        g = g.reshape(ctx.gshape).to(device=grad_out.device, dtype=ctx.gdtype)
        return grad_out.to(ctx.gdtype) * g, None, None, None


def windowed_objective(gamma, solver, max_steps, start=None):
    """J(gamma) with autograd support through the discrete adjoint: from rest
    with the window criterion (start=None), or one window from a fixed
    window-start state start = (f, step)."""
    return WindowedJ.apply(gamma, solver, max_steps, start)
