"""The optimisation loop (Algorithm "Optimization iteration"): each iteration
maps the design variables to gamma (density filter and Heaviside
projection), runs the forward windows with the consecutive-window test
(Algorithm "LES solver"), takes the adjoint over the representative window,
carries dJ/dgamma back to the design variables (chain rule) and takes the
projected-gradient step under the volume constraint that stands in for MMA.
The projection parameter starts at beta and doubles every beta_every
iterations up to beta_max (Sec. "Topology optimization procedure"); the loop
stops after n_max iterations or when the relative change of J_eff falls to
eps_o. Every step runs in the HIP library; this module only sequences the
calls."""

import torch

from .design import Design
from .solver import Solver


def optimize(w, mask, x0, prec="f32", radius=4.0, eta=0.5, beta=2.0, beta_max=16.0, beta_every=10,
             move=0.2, vmax=0.5, n_max=50, eps_o=1e-3, base=None, callback=None, vmin=0.0, steps=None,
             u_ref=None):
    """Returns (x, history): the design variables ([x, y(, z)] FP64 torch
    tensor on the GPU) and one record per iteration (J_eff, volume fraction,
    beta, representative window, multiplier). `base` is gamma off the design
    domain (default: the workload's gamma). steps = None: each iteration runs
    the windows until the consecutive-window test passes (the representative
    window); otherwise a prescribed window: `steps` steps from t = 0 and the
    last of its windows (steps a multiple of the window length). u_ref: the
    reference mean velocity of the wake objective on its measurement box."""
    dz = Design(w.shape, mask, w.gamma if base is None else base, radius)
    sv = Solver(w, prec)
    if u_ref is not None:
        sv.set_wake_reference(u_ref)
    x = torch.as_tensor(x0, dtype=torch.float64).to(sv.device)
    hist, J_prev = [], None
    try:
        for m in range(n_max):
            gamma, V = dz.map(x, beta, eta)
            sv.set_gamma(gamma)
            if steps is None:
                rep = sv.forward(w.max_windows * w.window_len, stop_on_converge=True)
            else:
                rep = sv.forward(steps)
            g, J = sv.adjoint()
            gJ, gV = dz.chain(x, beta, eta, g)
            x_new, _, lam = dz.update(x, gJ, gV, beta, eta, move, vmax, vmin)
            rec = {"iter": m, "J": J, "V": V, "beta": beta, "w_eff": int(rep["w_eff"]), "lam": lam}
            hist.append(rec)
            if callback is not None:
                callback(rec)
            stop = J_prev is not None and abs(J - J_prev) <= eps_o * abs(J)
            J_prev = J
            if stop:
                break
            x = x_new.contiguous()
            if (m + 1) % beta_every == 0:
                beta = min(2.0 * beta, beta_max)
    finally:
        sv.close()
        dz.close()
    return x, hist
