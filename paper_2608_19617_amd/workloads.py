"""Seeded synthetic inputs: geometries, design fields, inlet profiles and
window parameters of the benchmark and test configurations.

This module holds no solver arithmetic. It only describes problems (numbers
and numpy arrays) so that the HIP path and the CPU oracle can be fed the
same inputs. Arrays are indexed [x, y] (2D) or [x, y, z] (3D); the binding
converts them to the library's x-fastest node order.

Readings used for the inputs (the paper does not fix them):
  * Re = U L / nu with U the peak inlet speed and L the obstacle diameter,
    step height or channel width; nu = (tau - 1/2) / 3 (Eq.
    viscosity_relation), so tau = 1/2 + 3 U L / Re.
  * parabolic inlet rows: u0(y) = 4 U (y - a)(b - y) / (b - a)^2 with the
    halfway walls at y = a and y = b (half a node outside the open rows);
  * an obstacle given as gamma = 1 inside, 0 outside, with a linear ramp two
    nodes wide: gamma = clip((R + 1 - r) / 2, 0, 1);
  * the initial state is rho = 1 and u = (u0(y), 0) along x unless stated.
"""

from dataclasses import dataclass, field

import numpy as np

WALL, VELOCITY, PRESSURE = 0, 1, 2


@dataclass
class Workload:
    name: str
    shape: tuple                     # (nx, ny) or (nx, ny, nz)
    tau: float
    c_smag: float
    gamma: np.ndarray                # design field, 1 = solid
    west: np.ndarray                 # row kinds of the x = 0 face
    east: np.ndarray                 # row kinds of the x = nx-1 face
    u_in: np.ndarray                 # inlet speed per row
    periodic: tuple = (False, False, False)
    rho_out: float = 1.0
    rho_init: float = 1.0
    u_init_mode: int = 1             # 1: u = (u_in(y), 0) everywhere at t = 0
    objective: str = "dp"            # "dp", "diss_dp", "drag" or "wake"
    monitor: str = "dp"              # "dp", "diss_dp" or "cd"
    sec_in: tuple = (0, 0, 1)        # (x, ylo, yhi)
    sec_out: tuple = (0, 0, 1)
    window_len: int = 100
    sample_every: int = 1
    ckpt_every: int = 10
    eps: float = -1.0
    max_windows: int = 1
    n_steps: int = 100               # forward steps of the workload
    s_map: str = "linear"
    s_q: float = 0.1
    full_history: bool = False       # keep every window's start state (full-time adjoint)
    force_box: tuple = None          # ((x0, x1), (y0, y1)[, (z0, z1)]) of the drag; None: whole grid
    drag_ref: float = 1.0            # rho_0 u_0^2 L_ref / 2 of the C_d monitor
    meas_box: tuple = None           # measurement region of the wake objective; None: whole grid
    notes: dict = field(default_factory=dict)

    @property
    def nodes(self):
        return int(np.prod(self.shape))

    @property
    def lattice(self):
        return "D2Q9" if len(self.shape) == 2 else "D3Q19"


def tau_from_re(u, length, re):
    return 0.5 + 3.0 * u * length / re


def parabola(ny, lo, hi, u_max):
    """u0 on rows [lo, hi) with walls half a node outside them; 0 elsewhere."""
    y = np.arange(ny, dtype=np.float64)
    a, b = lo - 0.5, hi - 0.5
    u = 4 * u_max * (y - a) * (b - y) / (b - a) ** 2
    u[(y < lo) | (y >= hi)] = 0.0
    return u


def disk(shape, cx, cy, radius):
    """gamma of a disk (a cylinder along z in 3D) with a 2-node linear ramp."""
    X, Y = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    r = np.hypot(X - cx, Y - cy)
    g = np.clip((radius + 1 - r) / 2, 0.0, 1.0)
    if len(shape) == 3:
        g = np.repeat(g[:, :, None], shape[2], axis=2)
    return g


def _rows(ny, lo, hi, kind):
    k = np.zeros(ny, np.int64)
    k[lo:hi] = kind
    return k


def cylinder_channel(nx=160, ny=64, radius=8, center=(40, 32), u_max=0.05, re=100.0,
                     window_len=500, sample_every=1, ckpt_every=50, n_windows=4, c_smag=0.1):
    """Cylinder in a channel: parabolic Zou-He inlet, pressure outlet, walls
    top and bottom, J = mean inlet-outlet pressure drop over each window."""
    return Workload(
        name=f"cylinder_channel_{nx}x{ny}",
        shape=(nx, ny), tau=tau_from_re(u_max, 2 * radius, re), c_smag=c_smag,
        gamma=disk((nx, ny), center[0], center[1], radius),
        west=_rows(ny, 1, ny - 1, VELOCITY), east=_rows(ny, 1, ny - 1, PRESSURE),
        u_in=_channel_parabola(ny, u_max),
        sec_in=(0, 1, ny - 1), sec_out=(nx - 1, 1, ny - 1),
        window_len=window_len, sample_every=sample_every, ckpt_every=ckpt_every,
        eps=-1.0, max_windows=n_windows, n_steps=n_windows * window_len)


def _channel_parabola(ny, u_max):
    """Parabola between the halfway walls y = -1/2 and y = ny - 1/2."""
    y = np.arange(ny, dtype=np.float64)
    u = 4 * u_max * (y + 0.5) * (ny - 0.5 - y) / ny ** 2
    u[0] = u[-1] = 0.0      # corner rows are wall nodes
    return u


def backward_facing_step(nx=800, ny=200, step_len=100, step_h=100, u_max=0.05, re=800.0,
                         window_len=2000, sample_every=100, eps=1e-3, max_windows=20,
                         ckpt_every=100, c_smag=0.1):
    """Backward-facing step: the step (gamma = 1) fills x < step_len,
    y < step_h; the inlet rows above it carry a parabola between the step top
    and the upper wall; pressure outlet; consecutive windows with the
    criterion on the window-mean pressure drop."""
    g = np.zeros((nx, ny))
    g[:step_len, :step_h] = 1.0
    u = parabola(ny, step_h, ny, u_max)
    u[ny - 1] = 0.0
    return Workload(
        name=f"backward_facing_step_{nx}x{ny}",
        shape=(nx, ny), tau=tau_from_re(u_max, step_h, re), c_smag=c_smag, gamma=g,
        west=_rows(ny, step_h, ny - 1, VELOCITY), east=_rows(ny, 1, ny - 1, PRESSURE), u_in=u,
        sec_in=(0, step_h, ny - 1), sec_out=(nx - 1, 1, ny - 1),
        window_len=window_len, sample_every=sample_every, ckpt_every=ckpt_every,
        eps=eps, max_windows=max_windows, n_steps=max_windows * window_len)


def cylinder_wake(nx=2048, ny=512, radius=32, u_max=0.04, re=1000.0, window_len=20000,
                  sample_every=20, ckpt_every=500, max_windows=5, eps=1e-3, c_smag=0.1):
    """Cylinder wake at high Reynolds number (LES regime)."""
    w = cylinder_channel(nx, ny, radius, (nx // 4, ny // 2), u_max, re, window_len, sample_every,
                         ckpt_every, max_windows, c_smag)
    w.name = f"cylinder_wake_{nx}x{ny}"
    w.eps = eps
    return w


def u_bend(n=1024, width=128, u0=0.03, re=2000.0, window_len=10000, sample_every=20,
           ckpt_every=500, seed=0, sigma=4.0, c_smag=0.1, max_windows=2):
    """U-bend: inlet and outlet legs on the west face joined by a half
    annulus; the channel is fluid (gamma = 0) and every other node is a
    design node with gamma drawn uniform in [0, 1] from the seed,
    Gaussian-smoothed (sigma nodes) and rescaled to [0, 1]. Uniform inlet
    speed u0; J = dissipation plus the pressure drop between sections at
    x = width across each leg."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    raw = rng.random((n, n))
    sm = gaussian_filter(raw, sigma, mode="nearest")
    g = (sm - sm.min()) / (sm.max() - sm.min())
    c = n // 2
    in_lo, in_hi = c + width // 2, c + width // 2 + width           # upper (inlet) leg
    out_lo, out_hi = c - width // 2 - width, c - width // 2         # lower (outlet) leg
    x_bend = 3 * width
    X, Y = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    chan = np.zeros((n, n), bool)
    chan[:x_bend, in_lo:in_hi] = True
    chan[:x_bend, out_lo:out_hi] = True
    r = np.hypot(X - x_bend, Y - (c - 0.5))
    r_in, r_out = c - 0.5 - (out_hi - 0.5), c - 0.5 - (out_lo - 0.5)
    chan |= (X >= x_bend) & (r >= r_in) & (r <= r_out)
    g[chan] = 0.0
    west = np.zeros(n, np.int64)
    west[in_lo:in_hi] = VELOCITY
    west[out_lo:out_hi] = PRESSURE
    u = np.zeros(n)
    u[in_lo:in_hi] = u0
    return Workload(
        name=f"u_bend_{n}x{n}", shape=(n, n), tau=tau_from_re(u0, width, re), c_smag=c_smag,
        gamma=g, west=west, east=np.zeros(n, np.int64), u_in=u, u_init_mode=0,
        objective="diss_dp", monitor="diss_dp",
        sec_in=(width, in_lo, in_hi), sec_out=(width, out_lo, out_hi),
        window_len=window_len, sample_every=sample_every, ckpt_every=ckpt_every,
        eps=0.05, max_windows=max_windows, n_steps=max_windows * window_len)


def cylinder_3d(nx=384, ny=128, nz=128, radius=16, center=(96, 64), u_max=0.05, re=1000.0,
                window_len=5000, sample_every=20, ckpt_every=250, n_windows=4, c_smag=0.1):
    """D3Q19 channel with a cylinder along z: parabolic inlet in y, uniform
    in z; pressure outlet; walls in y; periodic in z."""
    w = Workload(
        name=f"cylinder_3d_{nx}x{ny}x{nz}", shape=(nx, ny, nz),
        tau=tau_from_re(u_max, 2 * radius, re), c_smag=c_smag,
        gamma=disk((nx, ny, nz), center[0], center[1], radius),
        west=_rows(ny, 1, ny - 1, VELOCITY), east=_rows(ny, 1, ny - 1, PRESSURE),
        u_in=_channel_parabola(ny, u_max), periodic=(False, False, True),
        sec_in=(0, 1, ny - 1), sec_out=(nx - 1, 1, ny - 1),
        window_len=window_len, sample_every=sample_every, ckpt_every=ckpt_every,
        eps=-1.0, max_windows=n_windows, n_steps=n_windows * window_len)
    return w


def cylinder_drag(re=51.2, nx=200, ny=100, radius=8, u0=0.05, window_len=5000, sample_every=50, eps=1e-3,
                  max_windows=20, ckpt_every=250, c_smag=0.1, s_q=0.1):
    """Flow around a circular cylinder (Sec. "Flow around a circular
    cylinder"): a 200 x 100 lattice with a cylinder of radius 8 at its centre
    holding the initial design phi = 0.5 (gamma = 0.5 inside, fluid
    outside); uniform inlet speed u0 on the west face, pressure outlet, walls
    top and bottom; tau from Re = u0 2r / nu. Drag objective over the whole
    domain with the C_d monitor (L_ref = 2r, rho_0 = 1) and the paper's
    interpolation g(phi; q); |W| = 5000, dW = 50, eps = 1e-3."""
    cx, cy = nx // 2, ny // 2
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    g = np.where(np.hypot(X - cx, Y - cy) <= radius, 0.5, 0.0)
    u = np.full(ny, u0)
    u[0] = u[-1] = 0.0
    return Workload(
        name=f"cylinder_drag_{nx}x{ny}_re{re:g}", shape=(nx, ny), tau=tau_from_re(u0, 2 * radius, re),
        c_smag=c_smag, gamma=g, west=_rows(ny, 1, ny - 1, VELOCITY), east=_rows(ny, 1, ny - 1, PRESSURE),
        u_in=u, objective="drag", monitor="cd", drag_ref=0.5 * u0 ** 2 * 2 * radius, s_map="paper", s_q=s_q,
        sec_in=(0, 1, ny - 1), sec_out=(nx - 1, 1, ny - 1),
        window_len=window_len, sample_every=sample_every, ckpt_every=ckpt_every,
        eps=eps, max_windows=max_windows, n_steps=max_windows * window_len,
        notes={"center": (cx, cy), "radius": radius, "re": re})


def wake_recovery(re=60.0, d=10, l_measure=33, nx=200, ny=50, l_m=6, u0=0.05, window_len=6000,
                  sample_every=20, eps=5e-4, max_windows=20, ckpt_every=300, c_smag=0.1, s_q=0.1,
                  reference=False, v0=0.5):
    """Wake-flow recovery (Sec. "Wake flow recovery", Table wfr): a 200 x 50
    channel with walls and a uniform inlet; the design domain D is 3d x 2d,
    centred across the channel, its front edge at x = 3d; the measurement
    square M of L_M x L_M nodes is centred across the channel with its centre
    L_measure downstream of D's back edge. reference=True places a cylinder
    of diameter d at the centre of D (gamma = 1 inside), the flow whose
    window-mean velocity on M is u_ref; otherwise D holds the constant
    initial design gamma = v0. Wake objective on M, C_d monitor of the drag
    over D (L_ref = d)."""
    x0, x1 = 3 * d, 6 * d
    y0, y1 = ny // 2 - d, ny // 2 + d
    xm = x1 + l_measure - l_m // 2
    ym = ny // 2 - l_m // 2
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    if reference:
        cx, cy = (x0 + x1 - 1) / 2.0, (y0 + y1 - 1) / 2.0
        g = np.where(np.hypot(X - cx, Y - cy) <= d / 2.0, 1.0, 0.0)
    else:
        g = np.zeros((nx, ny))
        g[x0:x1, y0:y1] = v0
    u = np.full(ny, u0)
    u[0] = u[-1] = 0.0
    box = ((x0, x1), (y0, y1))
    return Workload(
        name=f"wake_recovery_{nx}x{ny}_re{re:g}" + ("_reference" if reference else ""), shape=(nx, ny),
        tau=tau_from_re(u0, d, re), c_smag=c_smag, gamma=g, west=_rows(ny, 1, ny - 1, VELOCITY),
        east=_rows(ny, 1, ny - 1, PRESSURE), u_in=u, objective="wake", monitor="cd",
        force_box=box, drag_ref=0.5 * u0 ** 2 * d, meas_box=((xm, xm + l_m), (ym, ym + l_m)),
        s_map="paper", s_q=s_q, sec_in=(0, 1, ny - 1), sec_out=(nx - 1, 1, ny - 1),
        window_len=window_len, sample_every=sample_every, ckpt_every=ckpt_every,
        eps=eps, max_windows=max_windows, n_steps=max_windows * window_len,
        notes={"design_box": box, "re": re, "d": d, "l_measure": l_measure})


def u_bend_paper(re=400.0, u0=0.05, window_len=20000, sample_every=20, eps=0.05, max_windows=20,
                 ckpt_every=500, c_smag=0.1, s_q=0.1):
    """U-bend of the paper (Sec. "U-bend flow", Table ubend_parameters): Re 400
    on 240 x 192 (L_d = 24, L_f = L_m = L_p = 48, L_r = 144) or Re 750 on
    300 x 240 (30, 60, 60, 60, 180). The inlet leg (rows L_d + L_f + L_m ..
    L_y - L_d) and the outlet leg (rows L_d .. L_d + L_f) open on the west
    face and are joined beyond x = L_r by a half annulus of radii L_m / 2 and
    L_m / 2 + L_f around (L_r, L_y / 2). Design domain: x >= L_r, and the box
    L_p <= x < L_r, y < L_d + L_f. Initial design: the channel is fluid,
    the rest solid (gamma = 1, also off the design domain). Uniform inlet u0,
    west pressure outlet, walls elsewhere; J = window mean of the pressure
    drop between sections at x = L_p across the legs; tau from Re on L_f."""
    if re == 750.0:
        nx, ny, ld, lf, lm, lp, lr = 300, 240, 30, 60, 60, 60, 180
    else:
        nx, ny, ld, lf, lm, lp, lr = 240, 192, 24, 48, 48, 48, 144
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    out_lo, out_hi = ld, ld + lf
    in_lo, in_hi = ld + lf + lm, ny - ld
    yc = ny / 2.0 - 0.5
    r = np.hypot(X - lr, Y - yc)
    chan = np.zeros((nx, ny), bool)
    chan[:lr, in_lo:in_hi] = True
    chan[:lr, out_lo:out_hi] = True
    chan |= (X >= lr) & (r >= lm / 2.0) & (r <= lm / 2.0 + lf)
    design = (X >= lr) | ((X >= lp) & (Y < out_hi))
    g = np.where(chan, 0.0, 1.0)
    west = np.zeros(ny, np.int64)
    west[in_lo:in_hi] = VELOCITY
    west[out_lo:out_hi] = PRESSURE
    u = np.zeros(ny)
    u[in_lo:in_hi] = u0
    return Workload(
        name=f"u_bend_paper_{nx}x{ny}_re{re:g}", shape=(nx, ny), tau=tau_from_re(u0, lf, re), c_smag=c_smag,
        gamma=g, west=west, east=np.zeros(ny, np.int64), u_in=u, u_init_mode=0,
        objective="dp", monitor="dp", s_map="paper", s_q=s_q,
        sec_in=(lp, in_lo, in_hi), sec_out=(lp, out_lo, out_hi),
        window_len=window_len, sample_every=sample_every, ckpt_every=ckpt_every,
        eps=eps, max_windows=max_windows, n_steps=max_windows * window_len,
        notes={"design_mask": design, "re": re, "l_f": lf})


def random_design(shape, seed, lo=0.0, hi=1.0):
    """Uniform random design field (test input)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)
