"""Pins of three oracle functions by balance laws and closed-form flows:

* forward.dissipation (the U-bend objective's D = sum 2 rho nu_eff S:S, built
  from Eqs. nu_t, Pi, tau_eff and Lallemand_equation): in a periodic
  Taylor-Green vortex the kinetic energy E = sum rho |u|^2 / 2 falls at the
  rate dE/dt = -D, with the molecular viscosity (C_s = 0) and with the eddy
  viscosity of the LES closure (C_s > 0), in 2D and in 3D;
* forward.zou_he_general in 3D (the any-lattice form of Eqs. inlet and
  outlet used on D3Q19 x faces): after the rule a velocity node carries
  momentum (rho u0, 0, 0) with rho its own density, a pressure node has
  density rho_0 and no tangential momentum, and the normal unknown obeys the
  non-equilibrium bounce-back; a 3D Poiseuille channel develops the inlet
  parabola with no transverse flow;
* forward.pressure_drop (c_s^2 times the difference of the section means of
  rho, Sec. 4.4): in developed Poiseuille flow the drop between two sections
  L apart is the Hagen-Poiseuille gradient 12 rho nu u_bar L / H^2 of a
  channel of width H.

Each pin is also run against copies of the oracle function with a planted
mistake (a dropped factor, a flipped sign, a dropped transverse term), which
it must reject; the copies live only inside these CPU tests.
"""

import inspect
import textwrap

import numpy as np
import pytest

from oracle import forward as fw
from oracle.lattice import D2Q9, D3Q19


def _mutant(fn, old, new):
    """A copy of oracle function `fn` whose source has `old` replaced by `new`
    (exactly one occurrence), compiled against the same module globals."""
    src = textwrap.dedent(inspect.getsource(fn))
    assert src.count(old) == 1, (fn.__name__, old)
    ns = dict(fn.__globals__)
    exec(compile(src.replace(old, new), f"<planted mistake in {fn.__name__}>", "exec"), ns)
    return ns[fn.__name__]


# ------------------------------------------------ dissipation: energy budget

def _taylor_green(shape, plane, tau, c_smag, u0, rho0, steps):
    """States of a decaying Taylor-Green vortex in the (plane[0], plane[1])
    coordinate plane of a periodic box (uniform along a third axis in 3D)."""
    d = len(shape)
    a, b = plane
    n = shape[a]
    assert shape[b] == n
    k = 2 * np.pi / n
    grids = np.meshgrid(*[np.arange(m) for m in shape], indexing="ij")
    xa, xb = grids[a], grids[b]
    u = np.zeros((d,) + tuple(shape))
    u[a] = -u0 * np.cos(k * xa) * np.sin(k * xb)
    u[b] = u0 * np.sin(k * xa) * np.cos(k * xb)
    rho = rho0 * (1 - u0 ** 2 / (4 / 3) * (np.cos(2 * k * xa) + np.cos(2 * k * xb)))
    prob = fw.Problem(shape, tau, c_smag, periodic=(True,) * d, u_init=u, rho_init=rho)
    f = fw.initial_state(prob)
    s = np.zeros(shape)
    states = []
    for _ in range(steps):
        states.append(f)
        f = fw.step(prob, f, s)
    return prob, states


def _kinetic_energy(prob, f):
    rho = fw.density(f)
    u = fw.momentum(prob.lat, f) / rho
    return 0.5 * (rho * (u * u).sum(axis=0)).sum()


@pytest.fixture(scope="module")
def tg_runs():
    """2D molecular (rho_0 = 2, so that a misplaced density shows), 2D LES
    (C_s = 1: the eddy part is about twice the molecular one) and 3D (the
    vortex in the x-z plane, so the off-diagonal Pi_xz carries the stress)."""
    return [
        _taylor_green((32, 32), (0, 1), 0.8, 0.0, 0.01, 2.0, 152),
        _taylor_green((32, 32), (0, 1), 0.52, 1.0, 0.05, 1.5, 152),
        _taylor_green((24, 2, 24), (0, 2), 0.7, 0.0, 0.01, 2.0, 82),
    ]


def _budget_error(tg_runs):
    """max over the runs and sample times of |D(t) / (-dE/dt) - 1|, dE/dt by
    a central difference over one step."""
    worst = 0.0
    for prob, states in tg_runs:
        for t in (40, 80, 150):
            if t + 1 >= len(states):
                continue
            dEdt = (_kinetic_energy(prob, states[t + 1]) - _kinetic_energy(prob, states[t - 1])) / 2
            D = fw.dissipation(prob, states[t])
            assert D > 0
            worst = max(worst, abs(D / -dEdt - 1))
    return worst


def test_dissipation_is_the_kinetic_energy_loss(tg_runs):
    """dE/dt = -D to 2% (measured 0.4-1.1%: the lattice's O(k^2) and O(Ma^2)
    departures from the continuum budget)."""
    assert _budget_error(tg_runs) < 0.02


def test_dissipation_zero_at_equilibrium():
    """A uniform flow at equilibrium has Pi = 0, hence D = 0 exactly."""
    prob = fw.Problem((6, 5), 0.7, 0.3, periodic=(True, True))
    u = np.zeros((2, 6, 5))
    u[0] = 0.04
    u[1] = -0.01
    f = fw.equilibrium(prob.lat, np.full((6, 5), 1.1), u)
    assert abs(fw.dissipation(prob, f)) < 1e-30


@pytest.mark.parametrize("old,new", [
    ("(te - 0.5) * PP", "te * PP"),                       # nu_eff without the -1/2
    ("(2 * rho * prob.lat.cs2 * te * te)", "(4 * rho * prob.lat.cs2 * te * te)"),   # factor 2
    ("(2 * rho * prob.lat.cs2 * te * te)", "(2 * prob.lat.cs2 * te * te)"),         # rho dropped
    ("(2 * rho * prob.lat.cs2 * te * te)", "(2 * rho * te * te)"),                  # cs^2 dropped
    ("(2 * rho * prob.lat.cs2 * te * te)", "(2 * rho * prob.lat.cs2 * te)"),        # tau_e^1
])
def test_dissipation_pin_rejects_planted_mistakes(tg_runs, monkeypatch, old, new):
    monkeypatch.setattr(fw, "dissipation", _mutant(fw.dissipation, old, new))
    assert _budget_error(tg_runs) > 0.05


# --------------------------------------------- pressure drop: Poiseuille

def _poiseuille(shape, tau, steps):
    """Channel with walls at y = -1/2 and ny - 1/2, the parabolic Zou-He inlet
    and a pressure outlet (periodic z in 3D), run to its developed state."""
    d = len(shape)
    nx, ny = shape[:2]
    y = np.arange(ny)
    u_in = 4 * 0.05 * (y + 0.5) * (ny - 0.5 - y) / ny ** 2
    u_in[0] = u_in[-1] = 0.0
    west = np.zeros(ny, int)
    west[1:-1] = fw.VELOCITY
    east = np.zeros(ny, int)
    east[1:-1] = fw.PRESSURE
    u_init = np.zeros((d,) + tuple(shape))
    u_init[0] = u_in.reshape((1, -1) + (1,) * (d - 2))
    per = (False, False) + ((True,) if d == 3 else ())
    prob = fw.Problem(shape, tau, 0.0, periodic=per, west=west, east=east, u_in=u_in, u_init=u_init)
    f = fw.initial_state(prob)
    s = np.zeros(shape)
    for _ in range(steps):
        f = fw.step(prob, f, s)
    return prob, f, u_in


@pytest.fixture(scope="module")
def poiseuille_runs():
    return {2: _poiseuille((64, 16), 0.8, 3000), 3: _poiseuille((48, 12, 3), 0.8, 2000)}


def _gradient_error(run):
    """|pressure_drop between x = nx/4 and 3 nx/4 / (12 rho nu u_bar L / H^2) - 1|
    with u_bar the mean speed across the mid section and H = ny."""
    prob, f, _ = run
    nx, ny = prob.shape[:2]
    x1, x2 = nx // 4, 3 * nx // 4
    prob.sec_in, prob.sec_out = (x1, 0, ny), (x2, 0, ny)
    rho = fw.density(f)
    u = fw.momentum(prob.lat, f) / rho
    u_bar = u[0, nx // 2].mean()
    nu = (prob.tau - 0.5) * prob.lat.cs2
    expect = 12 * rho.mean() * nu * u_bar * (x2 - x1) / ny ** 2
    return abs(fw.pressure_drop(prob, f) / expect - 1)


@pytest.mark.slow
@pytest.mark.parametrize("d", [2, 3])
def test_pressure_drop_is_the_poiseuille_gradient(poiseuille_runs, d):
    """Measured 0.37% (2D) and 0.33% (3D): the halfway walls' slip at
    tau = 0.8 and compressibility."""
    assert _gradient_error(poiseuille_runs[d]) < 0.01


@pytest.mark.slow
@pytest.mark.parametrize("target,old,new", [
    ("pressure_drop", "return cs2 * (", "return ("),                                 # p = rho
    ("pressure_drop", "prob.sec_in) - _section_mean(prob, rho, prob.sec_out)",
     "prob.sec_out) - _section_mean(prob, rho, prob.sec_in)"),                        # sign
    ("_section_mean", "rho[x, lo:hi].mean()", "rho[x, lo:hi].sum()"),                 # sum, not mean
])
def test_pressure_drop_pin_rejects_planted_mistakes(poiseuille_runs, monkeypatch, target, old, new):
    monkeypatch.setattr(fw, target, _mutant(getattr(fw, target), old, new))
    assert _gradient_error(poiseuille_runs[2]) > 0.05


@pytest.mark.slow
def test_d3q19_poiseuille_profile(poiseuille_runs):
    """3D channel (periodic z): the developed mid-channel profile is the
    inlet parabola (shape to 1e-3), uniform in z, with no transverse flow."""
    prob, f, _ = poiseuille_runs[3]
    nx, ny = prob.shape[:2]
    rho = fw.density(f)
    u = fw.momentum(prob.lat, f) / rho
    mid = u[:, nx // 2]
    prof = mid[0].mean(axis=1)
    y = np.arange(ny)
    par = (y + 0.5) * (ny - 0.5 - y)          # walls half a node outside rows 0 and ny - 1
    err = np.linalg.norm(prof / prof.mean() - par / par.mean()) / np.linalg.norm(par / par.mean())
    assert err < 1e-3
    assert np.ptp(mid[0], axis=1).max() < 1e-12
    assert np.abs(mid[1]).max() < 1e-6 and np.abs(mid[2]).max() < 1e-12


# ------------------------------------------------- 3D Zou-He post-conditions

def _random_columns(lat, m, rng):
    """m random near-equilibrium nodes with tangential momentum in y and z."""
    rho = 1.0 + 0.05 * rng.standard_normal(m)
    u = 0.05 * rng.standard_normal((lat.d, m))
    f = fw.equilibrium(lat, rho, u)
    return f + 0.01 * lat.w[:, None] * rng.standard_normal(f.shape)


def _zou_he_errors(lat, rng, m=64):
    """Largest violation of the rule's post-conditions on random columns, for
    both x faces and both kinds."""
    c = lat.c.astype(np.float64)
    worst = 0.0
    for face in (0, 1):
        sgn = 1 if face == 0 else -1
        normal = int(np.nonzero((lat.c[:, 0] == sgn) & (np.abs(lat.c).sum(axis=1) == 1))[0][0])
        for kind in (fw.VELOCITY, fw.PRESSURE):
            fn = _random_columns(lat, m, rng)
            u0 = 0.06 * rng.random(m)
            out = fw.zou_he_general(lat, fn, face, kind, u0=u0, rho0=1.03)
            rho = out.sum(axis=0)
            j = c.T @ out
            known = lat.c[:, 0] != sgn
            errs = [np.abs(out[known] - fn[known]).max()]            # known populations kept
            if kind == fw.VELOCITY:
                errs.append(np.abs(j[0] - rho * u0).max())
            else:
                errs.append(np.abs(rho - 1.03).max())
            errs += [np.abs(j[p]).max() for p in range(1, lat.d)]    # no tangential momentum
            feq = fw.equilibrium(lat, rho, j / rho)
            errs.append(np.abs((out[normal] - feq[normal]) - (out[lat.opp[normal]] - feq[lat.opp[normal]])).max())
            worst = max(worst, max(errs))
    return worst


@pytest.mark.parametrize("lat", [D2Q9, D3Q19], ids=lambda l: l.name)
def test_zou_he_general_postconditions(lat, rng):
    """Velocity faces: j = (rho u0, 0[, 0]); pressure faces: sum f = rho_0 and
    zero tangential momentum; the normal unknown is the bounce-back of the
    non-equilibrium part; populations leaving the domain are unchanged."""
    assert _zou_he_errors(lat, rng) < 1e-15


@pytest.mark.parametrize("old,new", [
    ("acc = acc - 0.5 * c[a, p] * Np", "acc = acc + 0.5 * c[a, p] * Np"),     # transverse sign
    ("acc = acc - 0.5 * c[a, p] * Np", "acc = acc - c[a, p] * Np"),           # transverse factor
    ("for p in range(1, lat.d):", "for p in range(1, 2):"),                   # z correction dropped
    ("+ 2 * lat.w[a] * rho", "+ lat.w[a] * rho"),                             # equilibrium factor
    ("rho = base / (1 - sgn * ux)", "rho = base / (1 + sgn * ux)"),           # mass balance sign
    ("ux = sgn * (1 - base / rho0)", "ux = (1 - base / rho0)"),               # outlet direction
])
def test_zou_he_pin_rejects_planted_mistakes(rng, monkeypatch, old, new):
    monkeypatch.setattr(fw, "zou_he_general", _mutant(fw.zou_he_general, old, new))
    assert _zou_he_errors(D3Q19, rng) > 1e-6
