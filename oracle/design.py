"""Design update of the optimisation loop (Sec. "Topology optimization
procedure" and Algorithm "Optimization iteration"): the density filter of
radius r, the Heaviside projection, the volume fraction, their chain-rule
transposes applied to the sensitivities, and a projected-gradient update of
the design variables that stands in for MMA.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke entry point and the
CPU-baseline leg of the benchmark, never by the product path.

Conventions (readings of the paper, listed in the design notes):
* Fields are arrays indexed [x, y] or [x, y, z]. gamma = 1 is solid (the
  paper's 1 - phi); the design variables x live on the design-domain nodes D
  (a boolean mask); every other node keeps a fixed gamma (`base`).
* Density filter (cone weights, as in the filter the paper cites): for i in D,
  x~_i = sum_{j in D} w_ij x_j / sum_{j in D} w_ij with w_ij = r - |x_i - x_j|
  for |x_i - x_j| < r, 0 otherwise; no periodic wrap.
* Heaviside projection (the tanh form of the projection the paper cites):
  H(x~) = [tanh(beta eta) + tanh(beta (x~ - eta))] / [tanh(beta eta) +
  tanh(beta (1 - eta))]; gamma_i = H(x~_i) on D.
* Volume fraction: V = (1 / n_D) sum_{i in D} gamma_i (the paper's mean of
  1 - phi over the design domain).
* Chain rule: dJ/dx_j = sum_{i in D} (dx~_i/dx_j) H'(x~_i) dJ/dgamma_i with
  dx~_i/dx_j = w_ij / W_i, W_i = sum_{k in D} w_ik (j in D).
* Update (the MMA stand-in): with the gradients scaled by their largest
  magnitude on D, x(lam) = clip(x - m (g_J + lam g_V), max(0, x - m),
  min(1, x + m)) on D; lam = 0 if V_min <= V(gamma(x(0))) <= V_max,
  otherwise the lam of smallest magnitude (to bisection accuracy) that
  brings V(gamma(x(lam))) back inside: lam > 0 above V_max, lam < 0 below
  V_min (the paper's constraints are two-sided).

parity: filter, projection and volume are pinned by closed forms and
invariants, the transposes by the dot-product identity and by complex-step
derivatives of the composed map, the update by its constraint and bound
properties (tests/test_oracle_design.py).
"""

import numpy as np


def filter_offsets(radius, dim):
    """Integer offsets o with |o| < radius and their weights radius - |o|."""
    h = int(np.ceil(radius)) - 1
    rng = range(-h, h + 1)
    offs, wts = [], []
    if dim == 2:
        grid = [(a, b) for a in rng for b in rng]
    else:
        grid = [(a, b, c) for a in rng for b in rng for c in rng]
    for o in grid:
        d = float(np.sqrt(sum(k * k for k in o)))
        if d < radius:
            offs.append(o)
            wts.append(radius - d)
    return offs, np.array(wts)


def _shifted(a, o):
    """b[i] = a[i + o] where i + o lies in the grid, else 0."""
    b = np.zeros_like(a)
    src, dst = [], []
    for k, n in zip(o, a.shape):
        if k >= 0:
            src.append(slice(k, n))
            dst.append(slice(0, n - k))
        else:
            src.append(slice(0, n + k))
            dst.append(slice(-k, n))
    b[tuple(dst)] = a[tuple(src)]
    return b


def filter_weight_sums(mask, radius):
    """W_i = sum_{j in D} w_ij for every node i."""
    m = mask.astype(float)
    offs, wts = filter_offsets(radius, mask.ndim)
    W = np.zeros(mask.shape)
    for o, w in zip(offs, wts):
        W += w * _shifted(m, o)
    return W


def density_filter(x, mask, radius):
    """x~ on D; x itself elsewhere."""
    m = mask.astype(float)
    offs, wts = filter_offsets(radius, mask.ndim)
    acc = np.zeros(x.shape, dtype=np.result_type(x, float))
    for o, w in zip(offs, wts):
        acc = acc + w * _shifted(m * x, o)
    W = filter_weight_sums(mask, radius)
    return np.where(mask, acc / np.where(mask, W, 1.0), x)


def density_filter_transpose(t, mask, radius):
    """g_j = sum_{i in D} (w_ij / W_i) t_i for j in D, 0 elsewhere."""
    m = mask.astype(float)
    W = filter_weight_sums(mask, radius)
    s = np.where(mask, t / np.where(mask, W, 1.0), 0.0)
    offs, wts = filter_offsets(radius, mask.ndim)
    g = np.zeros(t.shape, dtype=np.result_type(t, float))
    for o, w in zip(offs, wts):
        g = g + w * _shifted(s, o)       # w is even in o: w_ij = w_ji
    return m * g


def heaviside(xt, beta, eta):
    num = np.tanh(beta * eta) + np.tanh(beta * (xt - eta))
    return num / (np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta)))


def heaviside_derivative(xt, beta, eta):
    th = np.tanh(beta * (xt - eta))
    return beta * (1.0 - th * th) / (np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta)))


def physical_field(x, mask, base, radius, beta, eta):
    """gamma: the projected filtered design on D, base elsewhere."""
    return np.where(mask, heaviside(density_filter(x, mask, radius), beta, eta), base)


def volume_fraction(gamma, mask):
    return float(np.sum(np.where(mask, gamma, 0.0)) / np.count_nonzero(mask))


def chain(x, mask, radius, beta, eta, dJdgamma):
    """(dJ/dx, dV/dx) on D (0 elsewhere) for a sensitivity dJ/dgamma."""
    xt = density_filter(x, mask, radius)
    dH = heaviside_derivative(xt, beta, eta)
    gJ = density_filter_transpose(np.where(mask, dH * dJdgamma, 0.0), mask, radius)
    gV = density_filter_transpose(np.where(mask, dH / np.count_nonzero(mask), 0.0), mask, radius)
    return gJ, gV


def _scaled(g, mask):
    top = np.max(np.abs(np.where(mask, g, 0.0)))
    return g / top if top > 0 else np.zeros_like(g)


def update(x, dJdx, dVdx, mask, base, radius, beta, eta, move, vmax, vmin=0.0, iters=60):
    """One projected-gradient step under vmin <= V <= vmax: returns
    (x_new, V(x_new), lam). V(x(lam)) does not increase with lam (dV/dx >= 0),
    so lam = 0 when V(x(0)) lies in the bounds, lam > 0 when it exceeds vmax
    and lam < 0 when it is below vmin. Bracketing doubles |lam| from 1;
    bisection then halves the bracket `iters` times and keeps its feasible
    end."""
    sJ, sV = _scaled(dJdx, mask), _scaled(dVdx, mask)
    lo = np.maximum(0.0, x - move)
    hi = np.minimum(1.0, x + move)

    def trial(lam):
        return np.where(mask, np.clip(x - move * (sJ + lam * sV), lo, hi), x)

    def vol(lam):
        return volume_fraction(physical_field(trial(lam), mask, base, radius, beta, eta), mask)

    v0 = vol(0.0)
    if vmin <= v0 <= vmax:
        return trial(0.0), v0, 0.0
    if v0 > vmax:
        sign, feasible = 1.0, (lambda v: v <= vmax)
    else:
        sign, feasible = -1.0, (lambda v: v >= vmin)
    a, b = 0.0, sign
    for _ in range(60):
        if feasible(vol(b)):
            break
        a, b = b, 2.0 * b
    for _ in range(iters):
        c = 0.5 * (a + b)
        if feasible(vol(c)):
            b = c
        else:
            a = c
    return trial(b), vol(b), b
