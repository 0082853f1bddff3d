"""Forward regularized LBM-LES solver with partial bounce-back (oracle).

Written from Sec. 2 and Sec. 3.1 of the paper, in the order of Algorithm
"LES solver": equilibrium (Eq. feq) -> non-equilibrium moment Pi (Eq. Pi) ->
effective relaxation time (Eq. tau_eff) -> regularized collision
(Eq. modified_collision) -> fluid-solid treatment (Eq. external_force) ->
streaming (Eq. streaming_step) -> boundary rules (Eqs. wall, inlet, outlet)
-> sampling of the window averages (Eq. weighted_temporal_sampling) ->
consecutive-window test (Eq. statistical_criterion).

All arithmetic is FP64 (or complex128 for complex-step differentiation);
arrays are vectorised over nodes with shape (Q, nx, ny[, nz]) for
populations, i.e. f[alpha, x, y] is f_alpha(x_i, t).

Readings of the paper where it is silent or ambiguous (each is listed in the
design notes of the repository):
  * design field: gamma per node, 1 = solid; the bounce-back fraction is
    s = gamma ("linear") or s = g(1 - gamma; q) with the paper's convex
    interpolation g ("paper").
  * ||Pi|| = sqrt(2 Pi:Pi), the only reading under which Eq. tau_eff follows
    from Eqs. nu_t - Pi.
  * the wall rule of Eq. wall is a halfway bounce-back of post-collision
    values: a population that would be pulled from outside through a wall is
    the node's own post-collision population of the opposite direction.
  * nodes where an open face meets a wall are wall nodes; Zou-He acts only on
    open rows; the inlet speed u0 may vary per row.
  * a pressure outlet on the west face is the x-mirror of the printed east
    outlet.
  * pressure p = c_s^2 rho; the objective is sampled on the post-boundary
    populations of the sampled step; the sampling instants are end-aligned
    (the last step of each window is sampled).
  * window i is the |W| transitions ending at step i|W|; the criterion is
    strict, window 1 never converges, a zero current mean converges only if
    the previous mean is zero too.
  * drag (Sec. 3.1, Eq. C_d and the drag objective of the cylinder example):
    the force of Eq. external_force summed over the nodes of a box and the
    directions, F = sum_i sum_alpha c_alpha F_alpha, acts on the fluid; the
    drag is its negative x component, D = -F_x, the force the flow exerts on
    the porous solid (positive for flow along +x). C_d = D / d_ref with
    d_ref = rho_0 u_0^2 L_ref / 2 given.
  * wake recovery (Sec. "Wake flow recovery"): the window value is
    J = sum_{i in M} |u_bar_i - u_ref_i|^2 with u_bar the dW/|W|-weighted sum
    of the sampled velocities u = j / rho over the window; M is a box and
    u_ref is given (zero unless set).
"""

import numpy as np

from .lattice import D2Q9, D3Q19

WALL, VELOCITY, PRESSURE = 0, 1, 2


class Problem:
    """Plain container of everything one solve needs.

    shape       (nx, ny) for D2Q9, (nx, ny, nz) for D3Q19
    tau, c_smag relaxation time of the molecular viscosity, Smagorinsky C_s
    periodic    per-axis periodicity (x, y[, z])
    west, east  int arrays of length ny: kind of each row of the x faces
                (WALL / VELOCITY / PRESSURE); ignored when x is periodic
    u_in        float array of length ny: inlet x-velocity u0 per row
    rho_out     prescribed outlet density rho_0
    s_map, s_q  'linear' (s = gamma) or 'paper' (s = g(1 - gamma; q))
    objective   'dp' (inlet-outlet pressure drop) or 'diss_dp'
                (dissipation plus pressure drop)
    monitor     quantity averaged for the window test ('dp' or 'diss_dp')
    sec_in, sec_out  (x, ylo, yhi) pressure sections (all z in 3D)
    objective   also 'drag' (drag force over force_box) or 'wake' (wake
                recovery over meas_box); monitor also 'cd' (drag / drag_ref)
    force_box   ((x0, x1), (y0, y1)[, (z0, z1)]) half-open, None = whole grid
    drag_ref    rho_0 u_0^2 L_ref / 2, the denominator of C_d
    meas_box    measurement region M of the wake objective (as force_box)
    u_ref       reference mean velocity on M, shape (d, *box shape); None = 0
    window_len, sample_every, eps, max_windows   window parameters
    rho_init, u_init   initial macroscopic fields (scalar / (d, *shape))
    """

    def __init__(self, shape, tau, c_smag, *, periodic=None, west=None, east=None,
                 u_in=None, rho_out=1.0, s_map="linear", s_q=0.1,
                 objective="dp", monitor=None, sec_in=None, sec_out=None,
                 window_len=1, sample_every=1, eps=-1.0, max_windows=1,
                 rho_init=1.0, u_init=None, force_box=None, drag_ref=1.0, meas_box=None,
                 u_ref=None):
        self.shape = tuple(int(n) for n in shape)
        self.lat = D2Q9 if len(self.shape) == 2 else D3Q19
        d = self.lat.d
        self.tau = float(tau)
        self.c_smag = float(c_smag)
        self.periodic = tuple(periodic) if periodic is not None else (False,) * d
        ny = self.shape[1]
        self.west = np.zeros(ny, np.int64) if west is None else np.asarray(west, np.int64)
        self.east = np.zeros(ny, np.int64) if east is None else np.asarray(east, np.int64)
        self.u_in = np.zeros(ny) if u_in is None else np.asarray(u_in, np.float64)
        self.rho_out = float(rho_out)
        self.s_map = s_map
        self.s_q = float(s_q)
        self.objective = objective
        if monitor is None:
            monitor = "dp" if objective == "wake" else objective
        self.monitor = monitor
        self.sec_in = sec_in if sec_in is not None else (0, 0, ny)
        self.sec_out = sec_out if sec_out is not None else (self.shape[0] - 1, 0, ny)
        self.window_len = int(window_len)
        self.sample_every = int(sample_every)
        self.eps = float(eps)
        self.max_windows = int(max_windows)
        self.rho_init = rho_init
        self.u_init = np.zeros((d,) + self.shape) if u_init is None else np.asarray(u_init)
        full = tuple((0, n) for n in self.shape)
        self.force_box = full if force_box is None else tuple(tuple(b) for b in force_box)
        self.drag_ref = float(drag_ref)
        self.meas_box = full if meas_box is None else tuple(tuple(b) for b in meas_box)
        mshape = tuple(hi - lo for lo, hi in self.meas_box)
        self.u_ref = np.zeros((d,) + mshape) if u_ref is None else np.asarray(u_ref)
        self._geom = None
        self._check()

    def _check(self):
        assert self.tau > 0.5
        assert self.window_len % self.sample_every == 0
        for box in (self.force_box, self.meas_box):
            assert len(box) == len(self.shape)
            assert all(0 <= lo < hi <= n for (lo, hi), n in zip(box, self.shape))
        assert self.u_ref.shape == (self.lat.d,) + tuple(hi - lo for lo, hi in self.meas_box)
        ny = self.shape[1]
        if not self.periodic[0]:
            for kinds in (self.west, self.east):
                assert kinds.shape == (ny,)
                if not self.periodic[1]:
                    # rows touching a y wall are wall nodes
                    assert kinds[0] == WALL and kinds[-1] == WALL
            assert np.all(self.east != VELOCITY), "east velocity faces are not modelled"


# ---------------------------------------------------------------- moments

def density(f):
    """rho = sum_alpha f_alpha (Sec. 2.1.1, moment equations)."""
    return f.sum(axis=0)


def momentum(lat, f):
    """rho u = sum_alpha c_alpha f_alpha, shape (d, ...)."""
    return np.tensordot(lat.c.T.astype(np.float64), f, axes=([1], [0]))


def equilibrium(lat, rho, u):
    """Eq. feq: w rho [1 + c.u/cs^2 + (c.u)^2/(2 cs^4) - u.u/(2 cs^2)]."""
    cs2 = lat.cs2
    cu = np.tensordot(lat.c.astype(np.float64), u, axes=([1], [0]))
    uu = (u * u).sum(axis=0)
    wb = lat.w.reshape((-1,) + (1,) * rho.ndim)
    return wb * rho * (1.0 + cu / cs2 + cu * cu / (2 * cs2 * cs2) - uu / (2 * cs2))


def noneq_moment(lat, f, feq):
    """Eq. Pi: Pi_pq = sum_alpha c_ap c_aq (f_alpha - f^eq_alpha), shape (d, d, ...)."""
    c = lat.c.astype(np.float64)
    fne = f - feq
    d = lat.d
    Pi = np.empty((d, d) + f.shape[1:], dtype=fne.dtype)
    for p in range(d):
        for q in range(d):
            Pi[p, q] = np.tensordot(c[:, p] * c[:, q], fne, axes=([0], [0]))
    return Pi


def pi_norm(Pi):
    """||Pi|| = sqrt(2 Pi_pq Pi_pq), the norm of Eq. nu_t carried over to Pi."""
    return np.sqrt(2.0 * (Pi * Pi).sum(axis=(0, 1)))


def tau_effective(tau, c_smag, rho, norm, cs2):
    """Eq. tau_eff with filter width l_f = dx = 1."""
    return 0.5 * (tau + np.sqrt(tau * tau + 2.0 * c_smag * c_smag * norm / (rho * cs2 * cs2)))


def regularized_noneq(lat, Pi):
    """First-order non-equilibrium part of Eq. modified_collision:
    w_alpha / (2 cs^4) sum_pq (c_ap c_aq - cs^2 delta_pq) Pi_pq."""
    c = lat.c.astype(np.float64)
    cs2 = lat.cs2
    d = lat.d
    out = np.zeros((lat.Q,) + Pi.shape[2:], dtype=Pi.dtype)
    for a in range(lat.Q):
        acc = 0.0
        for p in range(d):
            for q in range(d):
                acc = acc + (c[a, p] * c[a, q] - cs2 * (p == q)) * Pi[p, q]
        out[a] = lat.w[a] / (2 * cs2 * cs2) * acc
    return out


def collide(prob, f):
    """Regularized LES collision, Eqs. feq, Pi, tau_eff, modified_collision.

    Returns f* and a dict of the intermediate node fields.
    """
    lat = prob.lat
    rho = density(f)
    u = momentum(lat, f) / rho
    feq = equilibrium(lat, rho, u)
    Pi = noneq_moment(lat, f, feq)
    norm = pi_norm(Pi)
    tau_e = tau_effective(prob.tau, prob.c_smag, rho, norm, lat.cs2)
    fneq = regularized_noneq(lat, Pi)
    fstar = feq + (1.0 - 1.0 / tau_e) * fneq
    aux = dict(rho=rho, u=u, feq=feq, Pi=Pi, norm=norm, tau_e=tau_e, fneq=fneq)
    return fstar, aux


def design_map(prob, gamma):
    """Bounce-back fraction s(gamma).

    'linear': s = gamma.  'paper': s = g(phi) = 0.5 (1 - phi (1+q)/(phi+q))
    with phi = 1 - gamma (Sec. 2.2, the convex interpolation of Eq.
    external_force; the paper's interpolation parameter is called q here).
    """
    if prob.s_map == "linear":
        return gamma * 1.0
    q = prob.s_q
    phi = 1.0 - gamma
    return 0.5 * (1.0 - phi * (1.0 + q) / (phi + q))


def design_map_derivative(prob, gamma):
    """ds/dgamma of design_map (the factor in Eq. sensitivity, with dphi/dgamma = -1)."""
    if prob.s_map == "linear":
        return np.ones_like(gamma)
    q = prob.s_q
    phi = 1.0 - gamma
    return 0.5 * q * (1.0 + q) / ((phi + q) ** 2)


def partial_bounce_back(lat, fstar, s):
    """Eq. external_force: F_alpha = s (f*_opp(alpha) - f*_alpha); returns f* + F."""
    F = s * (fstar[lat.opp] - fstar)
    return fstar + F


# --------------------------------------------------------------- geometry

def _geometry(prob):
    """Per-direction pull sources and the boundary classification of nodes."""
    if prob._geom is not None:
        return prob._geom
    lat = prob.lat
    shape = prob.shape
    d = lat.d
    idx = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    # open (Zou-He) nodes: x faces, rows whose kind is not WALL; in 3D the
    # nodes on a non-periodic z face are wall nodes
    open_kind = np.zeros(shape, np.int64)     # 0 none, else 1 + face*3 + kind
    if not prob.periodic[0]:
        okz = np.ones(shape, bool)
        if d == 3 and not prob.periodic[2]:
            okz = (idx[2] > 0) & (idx[2] < shape[2] - 1)
        for face, kinds in ((0, prob.west), (1, prob.east)):
            xface = 0 if face == 0 else shape[0] - 1
            k = kinds[idx[1]]
            sel = (idx[0] == xface) & (k != WALL) & okz
            open_kind[sel] = 1 + face * 3 + k[sel]
    src = []
    for a in range(lat.Q):
        s_idx = []
        outside = np.zeros(shape, bool)
        for ax in range(d):
            si = idx[ax] - lat.c[a, ax]
            if prob.periodic[ax]:
                si = si % shape[ax]
            else:
                outside |= (si < 0) | (si >= shape[ax])
                si = np.clip(si, 0, shape[ax] - 1)
            s_idx.append(si)
        src.append((tuple(s_idx), outside))
    prob._geom = dict(idx=idx, open_kind=open_kind, src=src)
    return prob._geom


def stream(prob, fpost):
    """Eq. streaming_step in pull form with the halfway wall rule (Eq. wall).

    f_alpha(x) = fpost_alpha(x - c_alpha) when x - c_alpha is in the domain
    (wrapping periodic axes); otherwise, at a wall node, the node's own
    post-collision population of the opposite direction; at an open node the
    value is unknown (NaN) until the Zou-He rule fills it in.
    """
    lat = prob.lat
    g = _geometry(prob)
    openm = g["open_kind"] > 0
    f = np.empty_like(fpost)
    for a in range(lat.Q):
        s_idx, outside = g["src"][a]
        fa = fpost[a][s_idx]
        refl = outside & ~openm
        fa = np.where(refl, fpost[lat.opp[a]], fa)
        fa = np.where(outside & openm, np.nan, fa)
        f[a] = fa
    return f


def _zou_he_2d(prob, f):
    """Eqs. inlet and outlet, printed D2Q9 forms, at every open node."""
    g = _geometry(prob)
    ok = g["open_kind"]
    ix, iy = g["idx"]
    # west velocity inlet (Eq. inlet) with u0 = u_in(row)
    sel = ok == 1 + 0 * 3 + VELOCITY
    if sel.any():
        f0, f2, f3, f4, f6, f7 = (f[a][sel] for a in (0, 2, 3, 4, 6, 7))
        u0 = prob.u_in[iy[sel]]
        rho = (f0 + f2 + f4 + 2 * (f3 + f6 + f7)) / (1 - u0)
        f[1][sel] = f3 + 2.0 / 3.0 * rho * u0
        f[5][sel] = f7 + 0.5 * (f4 - f2) + 1.0 / 6.0 * rho * u0
        f[8][sel] = f6 + 0.5 * (f2 - f4) + 1.0 / 6.0 * rho * u0
    # east pressure outlet (Eq. outlet) with rho_0 = rho_out
    sel = ok == 1 + 1 * 3 + PRESSURE
    if sel.any():
        f0, f1, f2, f4, f5, f8 = (f[a][sel] for a in (0, 1, 2, 4, 5, 8))
        r0 = prob.rho_out
        u = (f0 + f2 + f4 + 2 * (f1 + f5 + f8)) / r0 - 1
        f[3][sel] = f1 - 2.0 / 3.0 * r0 * u
        f[6][sel] = f8 + 0.5 * (f4 - f2) - 1.0 / 6.0 * r0 * u
        f[7][sel] = f5 + 0.5 * (f2 - f4) - 1.0 / 6.0 * r0 * u
    # west pressure outlet: the x-mirror of Eq. outlet (1<->3, 5<->6, 8<->7)
    sel = ok == 1 + 0 * 3 + PRESSURE
    if sel.any():
        f0, f2, f3, f4, f6, f7 = (f[a][sel] for a in (0, 2, 3, 4, 6, 7))
        r0 = prob.rho_out
        ux = 1 - (f0 + f2 + f4 + 2 * (f3 + f6 + f7)) / r0
        f[1][sel] = f3 + 2.0 / 3.0 * r0 * ux
        f[5][sel] = f7 + 0.5 * (f4 - f2) + 1.0 / 6.0 * r0 * ux
        f[8][sel] = f6 + 0.5 * (f2 - f4) + 1.0 / 6.0 * r0 * ux
    return f


def zou_he_general(lat, fn, face, kind, u0=None, rho0=None):
    """Zou-He on an x face for any velocity set, for nodes given as columns.

    fn: (Q, m) populations after streaming (unknowns arbitrary). The unknown
    populations (those entering the domain through the face) are
        f_a = f_opp(a) + 2 w_a rho (c_a . u) / cs^2 - 1/2 sum_perp c_ap N_p,
    N_p = sum over c_x = 0 of c_p f: the mass balance of Eqs. inlet / outlet
    fixes rho (velocity face) or u_x (pressure face), and the transverse
    correction makes the tangential momentum zero. For D2Q9 this is exactly
    the printed Eqs. inlet and outlet.
    """
    c = lat.c
    sgn = 1 if face == 0 else -1            # inward normal along x
    unknown = np.nonzero(c[:, 0] == sgn)[0]
    tang = np.nonzero(c[:, 0] == 0)[0]
    leaving = np.nonzero(c[:, 0] == -sgn)[0]
    base = fn[tang].sum(axis=0) + 2 * fn[leaving].sum(axis=0)
    if kind == VELOCITY:
        ux = u0
        rho = base / (1 - sgn * ux)
    else:
        rho = rho0 * np.ones_like(base)
        ux = sgn * (1 - base / rho0)
    out = fn.copy()
    for a in unknown:
        acc = fn[lat.opp[a]] + 2 * lat.w[a] * rho * (c[a, 0] * ux) / lat.cs2
        for p in range(1, lat.d):
            Np = (c[tang, p][:, None] * fn[tang]).sum(axis=0)
            acc = acc - 0.5 * c[a, p] * Np
        out[a] = acc
    return out


def _zou_he_3d(prob, f):
    g = _geometry(prob)
    ok = g["open_kind"]
    iy = g["idx"][1]
    for face in (0, 1):
        for kind in (VELOCITY, PRESSURE):
            sel = ok == 1 + face * 3 + kind
            if not sel.any():
                continue
            fn = np.stack([f[a][sel] for a in range(prob.lat.Q)])
            out = zou_he_general(prob.lat, fn, face, kind,
                                 u0=prob.u_in[iy[sel]], rho0=prob.rho_out)
            for a in range(prob.lat.Q):
                f[a][sel] = out[a]
    return f


def apply_boundaries(prob, f):
    """Open-face rules after streaming (walls were applied while streaming)."""
    if prob.lat.d == 2:
        return _zou_he_2d(prob, f)
    return _zou_he_3d(prob, f)


def step(prob, f, s):
    """One time step of Algorithm "LES solver": collide, fluid-solid, stream, BC."""
    fstar, _ = collide(prob, f)
    fpost = partial_bounce_back(prob.lat, fstar, s)
    return apply_boundaries(prob, stream(prob, fpost))


def initial_state(prob):
    """f(x, 0) = f^eq(rho(x, 0), u(x, 0)) (Sec. 2.1.3)."""
    rho = np.broadcast_to(np.asarray(prob.rho_init, np.float64), prob.shape).copy()
    return equilibrium(prob.lat, rho, prob.u_init.astype(np.float64))


# ------------------------------------------------------------- objectives

def _section_mean(prob, rho, sec):
    x, lo, hi = sec
    return rho[x, lo:hi].mean()


def pressure_drop(prob, f):
    """Mean inlet minus mean outlet pressure, p = cs^2 rho, over the sections."""
    rho = density(f)
    cs2 = prob.lat.cs2
    return cs2 * (_section_mean(prob, rho, prob.sec_in) - _section_mean(prob, rho, prob.sec_out))


def dissipation(prob, f):
    """Sum over nodes of 2 rho nu_eff S:S with S from Eq. Lallemand_equation
    and nu_eff from Eqs. nu_eff / effective_viscosity_relation:
    (tau_e - 1/2) Pi:Pi / (2 rho cs^2 tau_e^2)."""
    _, aux = collide(prob, f)
    Pi, rho, te = aux["Pi"], aux["rho"], aux["tau_e"]
    PP = (Pi * Pi).sum(axis=(0, 1))
    return ((te - 0.5) * PP / (2 * rho * prob.lat.cs2 * te * te)).sum()


def box_slices(box):
    """Index slices of a half-open box ((x0, x1), (y0, y1)[, (z0, z1)])."""
    return tuple(slice(lo, hi) for lo, hi in box)


def solid_force(prob, f, s):
    """Eq. external_force summed over the directions: F = sum_alpha c_alpha
    F_alpha at every node, F_alpha = s (f*_opp(alpha) - f*_alpha) on the
    post-collision populations f* of the post-boundary state f. Shape
    (d, *shape)."""
    lat = prob.lat
    fstar, _ = collide(prob, f)
    F = s * (fstar[lat.opp] - fstar)
    return momentum(lat, F)


def drag_force(prob, f, s):
    """D = -sum_{i in force_box} F_x(x_i): the x force that the fluid exerts
    on the porous solid in the box (the negative of the x momentum that the
    fluid-solid term removes from the fluid)."""
    return -solid_force(prob, f, s)[0][box_slices(prob.force_box)].sum()


def velocity(prob, f):
    """u = j / rho, shape (d, *shape)."""
    return momentum(prob.lat, f) / density(f)


def wake_value(prob, u_bar):
    """Wake-recovery objective J = sum_{i in M} |u_bar_i - u_ref_i|^2 for a
    window-mean velocity u_bar given on M, shape (d, *box shape)."""
    return ((u_bar - prob.u_ref) ** 2).sum()


def sample(prob, f, kind, s=None):
    """Instantaneous objective / monitor value j(t) on a post-boundary state
    (s, the bounce-back fraction, is needed by 'drag' and 'cd')."""
    if kind == "dp":
        return pressure_drop(prob, f)
    if kind == "diss_dp":
        return dissipation(prob, f) + pressure_drop(prob, f)
    if kind == "drag":
        return drag_force(prob, f, s)
    if kind == "cd":
        return drag_force(prob, f, s) / prob.drag_ref
    raise ValueError(kind)


# ---------------------------------------------------------------- windows

def window_test(m_prev, m_cur, eps):
    """Eq. statistical_criterion with the strict inequality.

    Returns (relative change, converged). A zero current mean converges only
    when the previous mean is zero as well.
    """
    if m_cur == 0:
        return (0.0 if m_prev == 0 else float("inf")), (m_prev == 0 and eps >= 0)
    rel = abs((m_cur - m_prev) / m_cur)
    return rel, (eps >= 0 and rel < eps)


def run(prob, gamma, n_steps, stop_on_converge=False, keep=()):
    """Algorithm "LES solver": windows of |W| steps, end-aligned samples every
    dW steps weighted dW/|W| (Eq. weighted_temporal_sampling), criterion at
    each window end.

    Returns a dict: f (final state), steps, J and M (per-window objective and
    monitor means), rel, converged (per window), w_eff (1-based index of the
    converged window, or of the last window), states (copies at the steps in
    `keep`).
    """
    f = initial_state(prob)
    s = design_map(prob, gamma)
    W, dW = prob.window_len, prob.sample_every
    wgt = dW / W
    Jacc = Macc = 0.0
    wake = prob.objective == "wake"
    msl = (slice(None),) + box_slices(prob.meas_box)
    ubar = 0.0
    out = dict(J=[], M=[], rel=[], converged=[], states={}, u_bar=None)
    if 0 in keep:
        out["states"][0] = f.copy()
    k = 0
    for k in range(1, n_steps + 1):
        f = step(prob, f, s)
        if k in keep:
            out["states"][k] = f.copy()
        if k % dW == 0:
            if wake:
                ubar = ubar + wgt * velocity(prob, f)[msl]
            else:
                Jacc += wgt * sample(prob, f, prob.objective, s)
            Macc += wgt * sample(prob, f, prob.monitor, s)
        if k % W == 0:
            if wake:
                Jacc = wake_value(prob, ubar)
                out["u_bar"] = ubar
                ubar = 0.0
            out["J"].append(Jacc)
            out["M"].append(Macc)
            if len(out["M"]) == 1:
                rel, conv = float("nan"), False
            else:
                rel, conv = window_test(out["M"][-2], out["M"][-1], prob.eps)
            out["rel"].append(rel)
            out["converged"].append(conv)
            Jacc = Macc = 0.0
            if stop_on_converge and (conv or len(out["M"]) >= prob.max_windows):
                break
    out["f"] = f
    out["steps"] = k
    out["w_eff"] = len(out["J"])
    return out


def window_objective(prob, gamma, f_start):
    """J over one window replayed from the fixed start state f^{n_s - 1}:
    the window-restricted subproblem that the adjoint differentiates."""
    s = design_map(prob, gamma)
    W, dW = prob.window_len, prob.sample_every
    f = f_start
    J = 0.0
    ubar = 0.0
    msl = (slice(None),) + box_slices(prob.meas_box)
    for m in range(1, W + 1):
        f = step(prob, f, s)
        if m % dW == 0:
            if prob.objective == "wake":
                ubar = ubar + dW / W * velocity(prob, f)[msl]
            else:
                J = J + dW / W * sample(prob, f, prob.objective, s)
    return wake_value(prob, ubar) if prob.objective == "wake" else J
