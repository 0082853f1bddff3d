"""Discrete adjoint of the windowed solver (oracle).

Written from Sec. 3.2 of the paper: the adjoint equation (Eq.
adjoint_equation) split into the adjoint collision (Eq. adjoint_collision)
and the adjoint streaming (Eq. adjoint_streaming), the adjoint wall rule and
the adjoint Zou-He inlet and outlet rules (Eqs. adjoint_inlet_bc,
adjoint_outlet_bc), the sensitivity (Eq. sensitivity), and the sampled
objective source of Eq. weighted_temporal_sampling, solved backward from the
end of the representative window to its beginning. The paper's own
objectives are included: the drag of the cylinder example, whose samples
depend on the design directly (an explicit dD/ds term beside the sources),
and the wake-recovery objective, a function of the window-mean velocity
whose sources carry 2 (u_bar - u_ref).

Sign convention: the paper's multiplier lambda multiplies
(f^{n+1} - f** ) in the Lagrangian, so the adjoint carried here is
kappa = -lambda, the derivative of J with respect to the post-collision,
post-fluid-solid populations; nu is the derivative of J with respect to the
post-boundary populations of a step. Only dJ/dgamma is compared with the GPU.

The window-restricted subproblem: the state f^{n_s - 1} entering the window
is held fixed; the |W| transitions inside the window and the samples taken
on their post-boundary states are differentiated (Sec. 3.2, "treated as
fixed ... window-restricted subproblem").
"""

import numpy as np

from . import forward as fw


# ----------------------------------------------------- adjoint boundaries

def _adjoint_inlet_2d(lam, u0):
    """Eq. adjoint_inlet_bc (printed), chi = u0 / (1 - u0)."""
    chi = u0 / (1 - u0)
    l0, l1, l2, l3, l4, l5, l6, l7, l8 = lam
    out = np.array(lam, copy=True)
    out[0] = l0 + 2 * chi / 3 * l1 + chi / 6 * l5 + chi / 6 * l8
    out[2] = l2 + 2 * chi / 3 * l1 + (-0.5 + chi / 6) * l5 + (0.5 + chi / 6) * l8
    out[4] = l4 + 2 * chi / 3 * l1 + (0.5 + chi / 6) * l5 + (-0.5 + chi / 6) * l8
    out[3] = l3 + (1 + 4 * chi / 3) * l1 + chi / 3 * l5 + chi / 3 * l8
    out[6] = l6 + 4 * chi / 3 * l1 + chi / 3 * l5 + (1 + chi / 3) * l8
    out[7] = l7 + 4 * chi / 3 * l1 + (1 + chi / 3) * l5 + chi / 3 * l8
    out[1] = out[5] = out[8] = 0.0
    return out


def _adjoint_outlet_east_2d(lam):
    """Eq. adjoint_outlet_bc (printed)."""
    l0, l1, l2, l3, l4, l5, l6, l7, l8 = lam
    out = np.array(lam, copy=True)
    out[0] = l0 - 2 / 3 * l3 - 1 / 6 * l6 - 1 / 6 * l7
    out[1] = l1 - 1 / 3 * l3 - 1 / 3 * l6 - 1 / 3 * l7
    out[2] = l2 - 2 / 3 * l3 - 2 / 3 * l6 + 1 / 3 * l7
    out[4] = l4 - 2 / 3 * l3 + 1 / 3 * l6 - 2 / 3 * l7
    out[5] = l5 - 4 / 3 * l3 - 1 / 3 * l6 + 2 / 3 * l7
    out[8] = l8 - 4 / 3 * l3 + 2 / 3 * l6 - 1 / 3 * l7
    out[3] = out[6] = out[7] = 0.0
    return out


def _adjoint_outlet_west_2d(lam):
    """x-mirror of Eq. adjoint_outlet_bc (1<->3, 5<->6, 8<->7) for the
    west-facing pressure outlet."""
    l0, l1, l2, l3, l4, l5, l6, l7, l8 = lam
    out = np.array(lam, copy=True)
    out[0] = l0 - 2 / 3 * l1 - 1 / 6 * l5 - 1 / 6 * l8
    out[3] = l3 - 1 / 3 * l1 - 1 / 3 * l5 - 1 / 3 * l8
    out[2] = l2 - 2 / 3 * l1 - 2 / 3 * l5 + 1 / 3 * l8
    out[4] = l4 - 2 / 3 * l1 + 1 / 3 * l5 - 2 / 3 * l8
    out[6] = l6 - 4 / 3 * l1 - 1 / 3 * l5 + 2 / 3 * l8
    out[7] = l7 - 4 / 3 * l1 + 2 / 3 * l5 - 1 / 3 * l8
    out[1] = out[5] = out[8] = 0.0
    return out


def boundary_matrix(lat, face, kind, u0=0.0, rho0=1.0):
    """Jacobian of the general Zou-He rule at one node (Q x Q, post <- pre).

    Built column by column from unit inputs (the rule is affine in the
    populations); its transpose is the adjoint rule for any velocity set.
    """
    Q = lat.Q
    eye = np.eye(Q)
    zero = np.zeros((Q, 1))
    u0v = np.full(Q, u0)
    base = fw.zou_he_general(lat, zero, face, kind, u0=np.array([u0]), rho0=rho0)
    cols = fw.zou_he_general(lat, eye, face, kind, u0=u0v, rho0=rho0)
    return cols - base


def adjoint_boundaries(prob, nu):
    """Transpose of the open-face rules, at open nodes only."""
    g = fw._geometry(prob)
    ok = g["open_kind"]
    iy = g["idx"][1]
    lat = prob.lat
    out = nu.copy()
    for face in (0, 1):
        for kind in (fw.VELOCITY, fw.PRESSURE):
            sel = ok == 1 + face * 3 + kind
            if not sel.any():
                continue
            lam = [nu[a][sel] for a in range(lat.Q)]
            if lat.d == 2:
                if face == 0 and kind == fw.VELOCITY:
                    res = _adjoint_inlet_2d(lam, prob.u_in[iy[sel]])
                elif face == 1 and kind == fw.PRESSURE:
                    res = _adjoint_outlet_east_2d(lam)
                else:
                    res = _adjoint_outlet_west_2d(lam)
            else:
                lamv = np.stack(lam)
                res = np.empty_like(lamv)
                u0s = prob.u_in[iy[sel]]
                cache = {}
                for j in range(lamv.shape[1]):
                    key = float(u0s[j])
                    if key not in cache:
                        cache[key] = boundary_matrix(lat, face, kind, key, prob.rho_out)
                    res[:, j] = cache[key].T @ lamv[:, j]
            for a in range(lat.Q):
                out[a][sel] = res[a]
    return out


def adjoint_stream(prob, nu_hat):
    """Eq. adjoint_streaming together with the adjoint wall rule.

    kappa_alpha(y) = nu_hat_alpha(y + c_alpha) inside the domain; where
    y + c_alpha is outside through a wall, the forward halfway rule read the
    population into direction opp(alpha) at y itself, so kappa_alpha(y) =
    nu_hat_opp(alpha)(y) (the printed adjoint bounce-back lambda_2 = lambda_4,
    ...); a population leaving through an open face is never read (0).
    """
    lat = prob.lat
    g = fw._geometry(prob)
    openm = g["open_kind"] > 0
    idx = g["idx"]
    shape = prob.shape
    kappa = np.empty_like(nu_hat)
    for a in range(lat.Q):
        t_idx = []
        outside = np.zeros(shape, bool)
        for ax in range(lat.d):
            ti = idx[ax] + lat.c[a, ax]
            if prob.periodic[ax]:
                ti = ti % shape[ax]
            else:
                outside |= (ti < 0) | (ti >= shape[ax])
                ti = np.clip(ti, 0, shape[ax] - 1)
            t_idx.append(ti)
        ka = nu_hat[a][tuple(t_idx)]
        ka = np.where(outside & ~openm, nu_hat[lat.opp[a]], ka)
        ka = np.where(outside & openm, 0.0, ka)
        kappa[a] = ka
    return kappa


# ------------------------------------------------ node-local derivatives

def equilibrium_jacobian(lat, rho, u):
    """d f^eq_beta / d f_alpha as printed in Sec. 3.2, shape (Q, Q, ...)."""
    cs2 = lat.cs2
    c = lat.c.astype(np.float64)
    cu = np.tensordot(c, u, axes=([1], [0]))               # (Q, ...)
    uu = (u * u).sum(axis=0)
    cc = c @ c.T                                            # c_b . c_a
    Q = lat.Q
    out = np.empty((Q, Q) + rho.shape, dtype=np.result_type(rho, u))
    for b in range(Q):
        phi_b = 1 + cu[b] / cs2 + cu[b] ** 2 / (2 * cs2 * cs2) - uu / (2 * cs2)
        for a in range(Q):
            # (c_b - u).(c_a - u) and (c_b.u)(c_b.(c_a - u))
            t1 = cc[b, a] - cu[b] - cu[a] + uu
            t2 = cu[b] * (cc[b, a] - cu[b])
            out[b, a] = lat.w[b] * phi_b + lat.w[b] * (t1 / cs2 + t2 / (cs2 * cs2))
    return out


def noneq_moment_jacobian(lat, dfeq):
    """d Pi_pq / d f_alpha = -sum_beta c_bp c_bq d f^eq_beta/d f_alpha + c_ap c_aq."""
    c = lat.c.astype(np.float64)
    d = lat.d
    out = np.empty((d, d) + dfeq.shape[1:], dtype=dfeq.dtype)
    for p in range(d):
        for q in range(d):
            w = c[:, p] * c[:, q]
            term = -np.tensordot(w, dfeq, axes=([0], [0]))
            cap = (c[:, p] * c[:, q]).reshape((-1,) + (1,) * (dfeq.ndim - 2))
            out[p, q] = term + cap
    return out


def _safe_div(num, den):
    zero = den == 0
    return np.where(zero, 0.0, num / np.where(zero, 1.0, den))


def tau_jacobian(prob, rho, Pi, norm, dPi):
    """d tau_eff / d f_alpha as printed in Sec. 3.2; d||Pi||/df = 2 Pi:dPi/||Pi||,
    taken as 0 where ||Pi|| = 0 (the term multiplies f^neq, which vanishes there)."""
    cs2 = prob.lat.cs2
    C2 = prob.c_smag ** 2
    R = np.sqrt(prob.tau ** 2 + 2 * C2 * norm / (rho * cs2 * cs2))
    dnorm = _safe_div(2 * (Pi[:, :, None] * dPi).sum(axis=(0, 1)), norm)
    return C2 / (2 * cs2 * cs2 * R) * (-norm / rho ** 2 + dnorm / rho)


def collision_jacobian(prob, f, s):
    """d f**_beta / d f_alpha of collision + fluid-solid treatment, assembled
    term by term as the bracket of Eq. adjoint_collision (with the
    interpolation g replaced by the bounce-back fraction s). Shape (Q, Q, ...),
    first index beta (output), second alpha (input)."""
    lat = prob.lat
    cs2 = lat.cs2
    c = lat.c.astype(np.float64)
    _, aux = fw.collide(prob, f)
    rho, u, Pi, norm, te, fneq = (aux[k] for k in ("rho", "u", "Pi", "norm", "tau_e", "fneq"))
    dfeq = equilibrium_jacobian(lat, rho, u)
    dPi = noneq_moment_jacobian(lat, dfeq)
    dtau = tau_jacobian(prob, rho, Pi, norm, dPi)
    Q, d = lat.Q, lat.d
    dfneq = np.zeros_like(dfeq)
    for b in range(Q):
        acc = 0.0
        for p in range(d):
            for q in range(d):
                acc = acc + (c[b, p] * c[b, q] - cs2 * (p == q)) * dPi[p, q]
        dfneq[b] = lat.w[b] / (2 * cs2 * cs2) * acc
    a_fac = 1 - 1 / te
    jac = np.empty_like(dfeq)
    opp = lat.opp
    for b in range(Q):
        bb = opp[b]
        plain = dfeq[b] + a_fac * dfneq[b] + fneq[b] * dtau / te ** 2
        fs = (dfeq[bb] - dfeq[b]) + (fneq[bb] - fneq[b]) * dtau / te ** 2 \
            + a_fac * (dfneq[bb] - dfneq[b])
        jac[b] = plain + s * fs
    return jac


def sensitivity_term(prob, f, kappa):
    """Per-node contribution of one step to dJ/ds (Eq. sensitivity without the
    interpolation factor): sum_alpha kappa_alpha ((f^eq_opp - f^eq_alpha) +
    (1 - 1/tau_eff)(f^neq_opp - f^neq_alpha))."""
    lat = prob.lat
    _, aux = fw.collide(prob, f)
    feq, fneq, te = aux["feq"], aux["fneq"], aux["tau_e"]
    opp = lat.opp
    diff = (feq[opp] - feq) + (1 - 1 / te) * (fneq[opp] - fneq)
    return (kappa * diff).sum(axis=0)


def objective_gradient(prob, f, kind=None, s=None, u_bar=None):
    """d j / d f on a post-boundary state, for j = 'dp', 'diss_dp', 'drag'
    (needs the bounce-back fraction s) or 'wake' (the derivative of the
    window value with respect to one sample's velocity, without the sample
    weight; needs the window-mean velocity u_bar on M)."""
    kind = prob.objective if kind is None else kind
    lat = prob.lat
    cs2 = lat.cs2
    g = np.zeros(f.shape, dtype=np.result_type(f, 0.0 if s is None else s))
    if kind == "drag":
        # D = -sum_box sum_alpha c_x,alpha s (f*_opp(alpha) - f*_alpha), with
        # d f* / d f the collision Jacobian without the fluid-solid term
        jac = collision_jacobian(prob, f, 0.0)
        cx = lat.c[:, 0].astype(np.float64)
        box = fw.box_slices(prob.force_box)
        for a in range(lat.Q):
            dFx = sum(cx[b] * (jac[lat.opp[b], a] - jac[b, a]) for b in range(lat.Q))
            g[a][box] = -(s * dFx)[box]
        return g
    if kind == "wake":
        # J = sum_M |u_bar - u_ref|^2, d u / d f_alpha = (c_alpha - u) / rho
        msl = (slice(None),) + fw.box_slices(prob.meas_box)
        rho = fw.density(f)[msl[1:]]
        u = fw.velocity(prob, f)[msl]
        r = 2.0 * (u_bar - prob.u_ref)
        c = lat.c.astype(np.float64)
        for a in range(lat.Q):
            g[a][msl[1:]] = sum(r[p] * (c[a, p] - u[p]) for p in range(lat.d)) / rho
        return g
    xi, lo, hi = prob.sec_in
    n_in = (hi - lo) * (prob.shape[2] if lat.d == 3 else 1)
    g[:, xi, lo:hi] += cs2 / n_in
    xo, lo, hi = prob.sec_out
    n_out = (hi - lo) * (prob.shape[2] if lat.d == 3 else 1)
    g[:, xo, lo:hi] -= cs2 / n_out
    if kind == "diss_dp":
        _, aux = fw.collide(prob, f)
        rho, u, Pi, norm, te = (aux[k] for k in ("rho", "u", "Pi", "norm", "tau_e"))
        dfeq = equilibrium_jacobian(lat, rho, u)
        dPi = noneq_moment_jacobian(lat, dfeq)
        dtau = tau_jacobian(prob, rho, Pi, norm, dPi)
        Z = (Pi * Pi).sum(axis=(0, 1))
        dZ = 2 * (Pi[:, :, None] * dPi).sum(axis=(0, 1))
        # D = (te - 1/2) Z / (2 cs2 rho te^2)
        h = (te - 0.5) / (rho * te * te)
        dh = dtau * (1 / (rho * te * te) - 2 * (te - 0.5) / (rho * te ** 3)) \
            - (te - 0.5) / (rho * rho * te * te)
        g = g + (dZ * h + Z * dh) / (2 * cs2)
    elif kind != "dp":
        raise ValueError(kind)
    return g


def objective_design_gradient(prob, f, kind=None):
    """Explicit d j / d s of a sample at fixed populations: nonzero for the
    drag only, dD/ds = -sum_alpha c_x,alpha (f*_opp(alpha) - f*_alpha) on the
    force box."""
    kind = prob.objective if kind is None else kind
    g = np.zeros(prob.shape, dtype=f.dtype)
    if kind == "drag":
        box = fw.box_slices(prob.force_box)
        g[box] = -fw.solid_force(prob, f, 1.0)[0][box]
    return g


# ---------------------------------------------------------- reverse sweep

def adjoint_step(prob, f_pre, s, nu_next):
    """One reverse step: from nu^{n} (adjoint of the post-boundary state f^n)
    to the collision-adjoint at step n-1 and the sensitivity increment.

    Returns (mu, dsens): mu = (d f^n / d f^{n-1})^T nu^n, dsens = d<nu^n,
    f^n>/ds with f^{n-1} fixed.
    """
    nu_hat = adjoint_boundaries(prob, nu_next)
    kappa = adjoint_stream(prob, nu_hat)
    dsens = sensitivity_term(prob, f_pre, kappa)
    jac = collision_jacobian(prob, f_pre, s)
    mu = np.einsum("ba...,b...->a...", jac, kappa)
    return mu, dsens


def window_gradient(prob, gamma, f_start):
    """J and dJ/dgamma over one window from the fixed state f_start.

    Forward: |W| steps from f_start, samples at end-aligned instants
    m = dW, 2 dW, ..., |W| weighted dW/|W|. Reverse: from m = |W| down to 1
    (the adjoint equations are solved at every step, the objective source
    only enters at sampling instants). Returns (J, dJ/dgamma, nu_start) where
    nu_start = dJ/d f_start (unused by the window method).
    """
    s = fw.design_map(prob, gamma)
    W, dW = prob.window_len, prob.sample_every
    wgt = dW / W
    states = [f_start]
    for m in range(1, W + 1):
        states.append(fw.step(prob, states[-1], s))
    u_bar = None
    if prob.objective == "wake":
        msl = (slice(None),) + fw.box_slices(prob.meas_box)
        u_bar = sum(wgt * fw.velocity(prob, states[m])[msl] for m in range(dW, W + 1, dW))
        J = fw.wake_value(prob, u_bar)
    else:
        J = 0.0
        for m in range(dW, W + 1, dW):
            J = J + wgt * fw.sample(prob, states[m], prob.objective, s)

    def source(m):
        return wgt * objective_gradient(prob, states[m], prob.objective, s, u_bar)

    nu = source(W)
    sens = wgt * objective_design_gradient(prob, states[W])
    for m in range(W, 0, -1):
        nu, dsens = adjoint_step(prob, states[m - 1], s, nu)
        sens = sens + dsens
        if m - 1 >= 1 and (m - 1) % dW == 0:
            nu = nu + source(m - 1)
            sens = sens + wgt * objective_design_gradient(prob, states[m - 1])
    return J, fw.design_map_derivative(prob, gamma) * sens, nu


def full_gradient(prob, gamma, n_windows):
    """J of window n_windows (the last) and dJ/dgamma through the whole
    history from f^0: the full-time adjoint that Sec. "Comparison with
    full-time adjoint optimization" compares against. The reverse sweep of
    the last window (with its objective sources) continues from the adjoint
    of that window's start state through every earlier step down to the
    first transition, with no objective source there; f^0 does not depend
    on gamma."""
    s = fw.design_map(prob, gamma)
    W = prob.window_len
    states = [fw.initial_state(prob)]
    for _ in range((n_windows - 1) * W):
        states.append(fw.step(prob, states[-1], s))
    J, g_window, nu = window_gradient(prob, gamma, states[-1])
    sens = np.zeros(prob.shape, dtype=np.result_type(states[0], s))
    for m in range(len(states) - 1, 0, -1):
        nu, dsens = adjoint_step(prob, states[m - 1], s, nu)
        sens = sens + dsens
    return J, g_window + fw.design_map_derivative(prob, gamma) * sens
