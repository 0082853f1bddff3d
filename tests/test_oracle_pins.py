"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the part of the oracle it pins and the passage it follows.
None of them re-types the formula under test: they check identities,
conservation laws, closed-form flows, transposes and complex-step
derivatives that a dropped term, a wrong sign or index, or a transposed
operand would break.
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle import adjoint as ad
from oracle import forward as fw
from oracle.lattice import D2Q9, D3Q19

LATTICES = [D2Q9, D3Q19]


def _frac_weights(lat):
    table = {4 / 9: Fraction(4, 9), 1 / 9: Fraction(1, 9), 1 / 36: Fraction(1, 36),
             1 / 3: Fraction(1, 3), 1 / 18: Fraction(1, 18)}
    return [table[float(w)] for w in lat.w]


# ---------------------------------------------------------------- P1 lattice

@pytest.mark.parametrize("lat", LATTICES, ids=lambda l: l.name)
def test_lattice_isotropy_exact(lat):
    """Sec. 2.1.1 velocity set: moments of the weights up to fourth order,
    exactly in rationals (c_s^2 = 1/3)."""
    w = _frac_weights(lat)
    c = lat.c
    d = lat.d
    cs2 = Fraction(1, 3)
    assert sum(w) == 1
    for p in range(d):
        assert sum(w[a] * c[a, p] for a in range(lat.Q)) == 0
        for q in range(d):
            m2 = sum(w[a] * c[a, p] * c[a, q] for a in range(lat.Q))
            assert m2 == (cs2 if p == q else 0)
            for r in range(d):
                assert sum(w[a] * c[a, p] * c[a, q] * c[a, r] for a in range(lat.Q)) == 0
                for s in range(d):
                    m4 = sum(w[a] * c[a, p] * c[a, q] * c[a, r] * c[a, s] for a in range(lat.Q))
                    dd = (p == q) * (r == s) + (p == r) * (q == s) + (p == s) * (q == r)
                    assert m4 == cs2 * cs2 * dd
    for a in range(lat.Q):
        assert np.all(c[lat.opp[a]] == -c[a])


def test_d2q9_order_matches_printed_boundary_indices():
    """The printed wall rule f4=f2, f7=f5, f8=f6 pairs opposite directions and
    the inlet unknowns 1, 5, 8 are the directions with c_x = +1."""
    assert list(D2Q9.opp[[2, 5, 6]]) == [4, 7, 8]
    assert sorted(np.nonzero(D2Q9.c[:, 0] == 1)[0]) == [1, 5, 8]
    assert sorted(np.nonzero(D2Q9.c[:, 0] == -1)[0]) == [3, 6, 7]


# ------------------------------------------------------------- P2 equilibrium

@pytest.mark.parametrize("lat", LATTICES, ids=lambda l: l.name)
def test_equilibrium_moments(lat, rng):
    """Eq. feq reproduces rho, rho u and rho cs^2 I + rho u u."""
    n = 50
    rho = 1 + 0.1 * rng.standard_normal(n)
    u = 0.05 * rng.standard_normal((lat.d, n))
    feq = fw.equilibrium(lat, rho, u)
    c = lat.c.astype(float)
    assert np.allclose(feq.sum(0), rho, rtol=0, atol=1e-15)
    assert np.allclose(c.T @ feq, rho * u, rtol=0, atol=1e-15)
    for p in range(lat.d):
        for q in range(lat.d):
            m2 = (c[:, p] * c[:, q]) @ feq
            ref = rho * (lat.cs2 * (p == q) + u[p] * u[q])
            assert np.allclose(m2, ref, rtol=0, atol=1e-15)


# --------------------------------------------------------------- P3 collision

def _random_state(lat, n, rng, amp=0.02):
    rho = 1 + 0.05 * rng.standard_normal(n)
    u = 0.05 * rng.standard_normal((lat.d, n))
    feq = fw.equilibrium(lat, rho, u)
    return feq + amp * lat.w[:, None] * rng.standard_normal((lat.Q, n))


class _NodeProblem:
    """Minimal stand-in carrying what collide() reads."""

    def __init__(self, lat, tau, c_smag):
        self.lat, self.tau, self.c_smag = lat, tau, c_smag


@pytest.mark.parametrize("lat", LATTICES, ids=lambda l: l.name)
def test_collision_conserves_and_relaxes(lat, rng):
    """Eq. modified_collision: mass and momentum unchanged; the non-equilibrium
    moment of f* is (1 - 1/tau_eff) Pi; with C_s = 0, tau_eff = tau."""
    f = _random_state(lat, 40, rng)
    prob = _NodeProblem(lat, 0.56, 0.1)
    fstar, aux = fw.collide(prob, f)
    c = lat.c.astype(float)
    assert np.allclose(fstar.sum(0), f.sum(0), rtol=0, atol=1e-15)
    assert np.allclose(c.T @ fstar, c.T @ f, rtol=0, atol=1e-15)
    feq2 = fw.equilibrium(lat, fstar.sum(0), (c.T @ fstar) / fstar.sum(0))
    Pi2 = fw.noneq_moment(lat, fstar, feq2)
    assert np.allclose(Pi2, (1 - 1 / aux["tau_e"]) * aux["Pi"], rtol=0, atol=1e-15)
    assert np.all(aux["tau_e"] > prob.tau)
    _, aux0 = fw.collide(_NodeProblem(lat, 0.56, 0.0), f)
    assert np.allclose(aux0["tau_e"], 0.56, rtol=0, atol=1e-15)


@pytest.mark.parametrize("lat", LATTICES, ids=lambda l: l.name)
def test_les_closure_solves_implicit_relation(lat, rng):
    """Eqs. nu_t, nu_eff, effective_viscosity_relation and Lallemand_equation
    define tau_eff implicitly: tau_eff = tau + C_s^2 ||S|| / cs^2 with
    S = -Pi / (2 rho cs^2 tau_eff) and ||S|| = sqrt(2 S:S). The closed form of
    Eq. tau_eff must satisfy it (this also fixes the reading of ||Pi||)."""
    f = _random_state(lat, 40, rng, amp=0.2)
    prob = _NodeProblem(lat, 0.507, 0.17)
    _, aux = fw.collide(prob, f)
    te, Pi, rho = aux["tau_e"], aux["Pi"], aux["rho"]
    S = -Pi / (2 * rho * lat.cs2 * te)
    normS = np.sqrt(2 * (S * S).sum(axis=(0, 1)))
    nu = (prob.tau - 0.5) * lat.cs2
    nu_t = prob.c_smag ** 2 * normS
    assert np.allclose(te, (nu + nu_t) / lat.cs2 + 0.5, rtol=1e-14, atol=0)
    assert np.max(te - prob.tau) > 1e-4      # the LES term is active


@pytest.mark.parametrize("lat", LATTICES, ids=lambda l: l.name)
def test_regularized_part_is_even(lat, rng):
    """The regularized first-order part is even under c -> -c, so the
    (f^neq_opp - f^neq) terms of Eqs. adjoint_collision and sensitivity vanish."""
    f = _random_state(lat, 30, rng)
    _, aux = fw.collide(_NodeProblem(lat, 0.6, 0.1), f)
    fneq = aux["fneq"]
    assert np.max(np.abs(fneq[lat.opp] - fneq)) < 1e-17
    assert np.max(np.abs(fneq)) > 1e-5


# --------------------------------------------------------- P5 partial bounce

@pytest.mark.parametrize("lat", LATTICES, ids=lambda l: l.name)
def test_partial_bounce_back_momentum(lat, rng):
    """Eq. external_force on f*: F_alpha = s(f*_opp - f*_alpha) equals
    -2 w s rho (c.u)/cs^2, so the node momentum becomes (1 - 2s) rho u and the
    mass is unchanged; s = 1 reverses the momentum."""
    f = _random_state(lat, 30, rng)
    fstar, aux = fw.collide(_NodeProblem(lat, 0.6, 0.1), f)
    s = rng.random(30)
    fpost = fw.partial_bounce_back(lat, fstar, s)
    c = lat.c.astype(float)
    rho, u = aux["rho"], aux["u"]
    cu = c @ u
    assert np.allclose(fpost - fstar, -2 * lat.w[:, None] * s * rho * cu / lat.cs2, rtol=0, atol=1e-16)
    assert np.allclose(c.T @ fpost, (1 - 2 * s) * rho * u, rtol=0, atol=1e-16)
    assert np.allclose(fpost.sum(0), rho, rtol=0, atol=1e-15)


def test_paper_interpolation_endpoints():
    """Sec. 2.2 interpolation g(phi) = 0.5(1 - phi(1+q)/(phi+q)): fluid
    (phi = 1, gamma = 0) gives 0, solid (phi = 0, gamma = 1) gives 1/2; its
    derivative matches a complex-step derivative."""
    prob = fw.Problem((4, 4), 0.6, 0.1, s_map="paper", s_q=0.3)
    g = np.array([0.0, 1.0, 0.37])
    s = fw.design_map(prob, g)
    assert s[0] == 0.0 and abs(s[1] - 0.5) < 1e-16
    h = 1e-30
    cs = fw.design_map(prob, g + 1j * h).imag / h
    assert np.allclose(fw.design_map_derivative(prob, g), cs, rtol=1e-15, atol=0)


@pytest.mark.parametrize("dims", [(12, 10), (6, 5, 4)])
def test_periodic_box_momentum_decay(dims, rng):
    """Periodic box, uniform s: the total momentum obeys P(t+1) = (1-2s) P(t)
    exactly and the total mass is conserved (collision conserves both,
    streaming is a permutation)."""
    d = len(dims)
    u_init = 0.03 * rng.standard_normal((d,) + dims)
    prob = fw.Problem(dims, 0.57, 0.1, periodic=(True,) * d, u_init=u_init)
    f = fw.initial_state(prob)
    s = np.full(dims, 0.013)
    c = prob.lat.c.astype(float)
    P = np.tensordot(c.T, f, axes=([1], [0])).reshape(d, -1).sum(1)
    m = f.sum()
    for _ in range(6):
        f = fw.step(prob, f, s)
        P_new = np.tensordot(c.T, f, axes=([1], [0])).reshape(d, -1).sum(1)
        assert np.allclose(P_new, (1 - 2 * 0.013) * P, rtol=1e-12, atol=1e-15)
        assert abs(f.sum() - m) < 1e-12 * m
        P = P_new


# ----------------------------------------------------------------- P7 Zou-He

def _open_problem(rng, west_kind, east_kind, u0=0.04):
    nx, ny = 5, 5
    west = np.zeros(ny, int)
    east = np.zeros(ny, int)
    west[1:-1] = west_kind
    east[1:-1] = east_kind
    return fw.Problem((nx, ny), 0.6, 0.1, west=west, east=east,
                      u_in=np.full(ny, u0), rho_out=1.02)


def test_zou_he_postconditions(rng):
    """Eqs. inlet and outlet: after the rule the inlet node carries momentum
    (rho u0, 0) with rho from the rule's mass balance; the outlet node has
    density rho_0 and zero tangential momentum; same for the west outlet."""
    lat = D2Q9
    c = lat.c.astype(float)
    for wk, ek in ((fw.VELOCITY, fw.PRESSURE), (fw.PRESSURE, fw.WALL)):
        prob = _open_problem(rng, wk, ek)
        f = _random_state(lat, 25, rng).reshape(9, 5, 5)
        f = fw.apply_boundaries(prob, f.copy())
        for y in range(1, 4):
            node = f[:, 0, y]
            rho = node.sum()
            j = c.T @ node
            if wk == fw.VELOCITY:
                assert abs(j[0] - rho * 0.04) < 1e-15 and abs(j[1]) < 1e-15
            else:
                assert abs(rho - 1.02) < 1e-15 and abs(j[1]) < 1e-15
            if ek == fw.PRESSURE:
                node = f[:, -1, y]
                assert abs(node.sum() - 1.02) < 1e-15
                assert abs((c.T @ node)[1]) < 1e-15


def test_general_zou_he_reduces_to_printed(rng):
    """The any-lattice Zou-He rule used in 3D gives the printed D2Q9 rules."""
    for wk, ek in ((fw.VELOCITY, fw.PRESSURE), (fw.PRESSURE, fw.WALL)):
        prob = _open_problem(rng, wk, ek)
        f = _random_state(D2Q9, 25, rng).reshape(9, 5, 5)
        printed = fw.apply_boundaries(prob, f.copy())
        for face, kind in ((0, wk), (1, ek)):
            if kind == fw.WALL:
                continue
            x = 0 if face == 0 else 4
            cols = f[:, x, 1:4]
            gen = fw.zou_he_general(D2Q9, cols, face, kind, u0=np.full(3, 0.04), rho0=1.02)
            assert np.allclose(gen, printed[:, x, 1:4], rtol=0, atol=1e-15)


# -------------------------------------------------- P8 adjoint boundary rules

def _bc_jacobian(prob, x, y):
    """Jacobian of the forward open-face rule at node (x, y), column by column
    (the rule is affine in the populations)."""
    f0 = np.full((9,) + prob.shape, 0.1)
    base = fw.apply_boundaries(prob, f0.copy())[:, x, y]
    M = np.zeros((9, 9))
    for b in range(9):
        f1 = f0.copy()
        f1[b, x, y] += 1.0
        M[:, b] = fw.apply_boundaries(prob, f1)[:, x, y] - base
    return M


def test_printed_adjoint_boundaries_are_transposes(rng):
    """Eqs. adjoint_inlet_bc and adjoint_outlet_bc (and the mirrored west
    outlet) are the exact transposes of the forward rules Eqs. inlet / outlet,
    and the outlet adjoint annihilates the constant vector."""
    for wk, ek, u0 in ((fw.VELOCITY, fw.PRESSURE, 0.04), (fw.PRESSURE, fw.WALL, 0.0),
                       (fw.VELOCITY, fw.PRESSURE, 0.11)):
        prob = _open_problem(rng, wk, ek, u0=u0)
        for x, kind in ((0, wk), (4, ek)):
            if kind == fw.WALL:
                continue
            M = _bc_jacobian(prob, x, 2)
            lam = rng.standard_normal((9,) + prob.shape)
            out = ad.adjoint_boundaries(prob, lam)
            assert np.allclose(out[:, x, 2], M.T @ lam[:, x, 2], rtol=0, atol=1e-14)
            if kind == fw.PRESSURE:
                ones = np.ones((9,) + prob.shape)
                assert np.allclose(ad.adjoint_boundaries(prob, ones)[:, x, 2], 0, atol=1e-15)
        # interior and wall nodes are untouched
        lam = rng.standard_normal((9,) + prob.shape)
        out = ad.adjoint_boundaries(prob, lam)
        assert np.array_equal(out[:, 2, :], lam[:, 2, :])
        assert np.array_equal(out[:, 0, 0], lam[:, 0, 0])


def test_boundary_matrix_matches_printed_2d(rng):
    """The generic transposed-Jacobian route (used in 3D) reproduces the printed
    2D adjoint rules."""
    for face, kind, u0 in ((0, fw.VELOCITY, 0.05), (1, fw.PRESSURE, 0.0), (0, fw.PRESSURE, 0.0)):
        M = ad.boundary_matrix(D2Q9, face, kind, u0, 1.0)
        lam = rng.standard_normal(9)
        if face == 0 and kind == fw.VELOCITY:
            ref = ad._adjoint_inlet_2d(list(lam), u0)
        elif face == 1:
            ref = ad._adjoint_outlet_east_2d(list(lam))
        else:
            ref = ad._adjoint_outlet_west_2d(list(lam))
        assert np.allclose(M.T @ lam, ref, rtol=0, atol=1e-14)


# --------------------------------------------------------- P9 dPi/df closed form

@pytest.mark.parametrize("lat", LATTICES, ids=lambda l: l.name)
def test_pi_jacobian_closed_form(lat, rng):
    """The printed dPi/df (via d f^eq / d f) equals (c_a - u)(c_a - u) - cs^2 I."""
    n = 7
    rho = 1 + 0.05 * rng.standard_normal(n)
    u = 0.05 * rng.standard_normal((lat.d, n))
    dPi = ad.noneq_moment_jacobian(lat, ad.equilibrium_jacobian(lat, rho, u))
    c = lat.c.astype(float)
    for a in range(lat.Q):
        for p in range(lat.d):
            for q in range(lat.d):
                ref = (c[a, p] - u[p]) * (c[a, q] - u[q]) - lat.cs2 * (p == q)
                assert np.allclose(dPi[p, q, a], ref, rtol=0, atol=1e-15)


# ---------------------------------------------------------- P10 Poiseuille

@pytest.mark.slow
def test_poiseuille_profile():
    """Walls at y = -1/2 and ny - 1/2 (halfway reading of Eq. wall), Zou-He
    velocity inlet with the parabolic profile, pressure outlet: the developed
    profile mid-channel is that parabola (shape to 1e-3; the halfway-wall slip
    is O((tau - 1/2)^2)) with no transverse flow."""
    nx, ny = 64, 16
    y = np.arange(ny)
    u_in = 4 * 0.05 * (y + 0.5) * (ny - 0.5 - y) / ny ** 2
    west = np.zeros(ny, int)
    west[1:-1] = fw.VELOCITY
    east = np.zeros(ny, int)
    east[1:-1] = fw.PRESSURE
    u_init = np.zeros((2, nx, ny))
    u_init[0] = u_in[None, :]
    prob = fw.Problem((nx, ny), 0.8, 0.0, west=west, east=east, u_in=u_in, u_init=u_init)
    f = fw.initial_state(prob)
    s = np.zeros((nx, ny))
    for _ in range(3000):
        f = fw.step(prob, f, s)
    rho = fw.density(f)
    u = fw.momentum(prob.lat, f) / rho
    prof = u[0, nx // 2]
    err = np.linalg.norm(prof / prof.mean() - u_in / u_in.mean()) / np.linalg.norm(u_in / u_in.mean())
    assert err < 1e-3
    assert np.abs(u[1, nx // 2]).max() < 1e-6
    # a linear pressure drop along the channel drives it
    p = rho.mean(axis=1) / 3
    assert p[5] > p[nx // 2] > p[nx - 6]


# --------------------------------------------------------- P11 Taylor-Green

@pytest.mark.slow
def test_taylor_green_decay():
    """Periodic Taylor-Green vortex with C_s = 0: the velocity amplitude decays
    as exp(-nu (kx^2 + ky^2) t) with nu = (tau - 1/2) cs^2
    (Eq. viscosity_relation); mass is conserved to round-off."""
    n = 32
    tau = 0.8
    k = 2 * np.pi / n
    x = np.arange(n)[:, None]
    y = np.arange(n)[None, :]
    u0 = 0.01
    u = np.stack([-u0 * np.cos(k * x) * np.sin(k * y) + 0 * y,
                  u0 * np.sin(k * x) * np.cos(k * y) + 0 * x])
    rho = 1 - u0 ** 2 / (4 * (1 / 3)) * (np.cos(2 * k * x) + np.cos(2 * k * y))
    prob = fw.Problem((n, n), tau, 0.0, periodic=(True, True), u_init=u, rho_init=rho)
    f = fw.initial_state(prob)
    s = np.zeros((n, n))
    m0 = f.sum()

    def amp(f):
        r = fw.density(f)
        v = fw.momentum(prob.lat, f) / r
        return np.sqrt((v * v).sum(axis=0).mean())

    a = []
    for t in range(401):
        if t in (100, 400):
            a.append(amp(f))
        f = fw.step(prob, f, s)
    rate = -np.log(a[1] / a[0]) / 300
    nu = (tau - 0.5) / 3
    assert abs(rate / (2 * nu * k * k) - 1) < 0.01
    assert abs(f.sum() - m0) < 1e-13 * m0


# ---------------------------------------------- P12 node-local derivatives

@pytest.mark.parametrize("lat", LATTICES, ids=lambda l: l.name)
def test_collision_jacobian_complex_step(lat, rng):
    """The explicit per-node Jacobian assembled from the printed terms of
    Eq. adjoint_collision equals the complex-step derivative of collision +
    fluid-solid treatment."""
    n = 6
    f = _random_state(lat, n, rng, amp=0.1)
    prob = _NodeProblem(lat, 0.53, 0.16)
    s = rng.random(n)
    jac = ad.collision_jacobian(prob, f, s)
    h = 1e-30
    for a in range(lat.Q):
        fc = f.astype(complex)
        fc[a] += 1j * h
        fs, _ = fw.collide(prob, fc)
        col = fw.partial_bounce_back(lat, fs, s).imag / h
        assert np.allclose(jac[:, a], col, rtol=1e-13, atol=1e-15)


def test_zero_stress_jacobian_is_finite():
    """At Pi = 0 the d||Pi||/df term is 0/0; the guard keeps the Jacobian
    finite and equal to the C_s = 0 Jacobian there (the term multiplies f^neq)."""
    lat = D2Q9
    rho = np.array([1.0])
    u = np.array([[0.03], [-0.01]])
    f = fw.equilibrium(lat, rho, u)
    jac = ad.collision_jacobian(_NodeProblem(lat, 0.6, 0.1), f, np.array([0.2]))
    jac0 = ad.collision_jacobian(_NodeProblem(lat, 0.6, 0.0), f, np.array([0.2]))
    assert np.all(np.isfinite(jac))
    assert np.allclose(jac, jac0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("kind", ["dp", "diss_dp"])
def test_objective_gradient_complex_step(kind, rng):
    """d j / d f of the sampled objective against complex-step."""
    nx, ny = 6, 5
    prob = fw.Problem((nx, ny), 0.55, 0.12, objective=kind, sec_in=(1, 1, 4), sec_out=(4, 0, 5),
                      periodic=(True, True))
    f = _random_state(D2Q9, nx * ny, rng, amp=0.1).reshape(9, nx, ny)
    g = ad.objective_gradient(prob, f)
    h = 1e-30
    for a, x, y in ((0, 1, 2), (3, 4, 0), (7, 2, 2), (5, 4, 4)):
        fc = f.astype(complex)
        fc[a, x, y] += 1j * h
        cs = fw.sample(prob, fc, kind).imag / h
        assert abs(g[a, x, y] - cs) <= 1e-14 * max(1.0, abs(cs))


# --------------------------------------------------- P13 whole window adjoint

def _window_cases():
    rng = np.random.default_rng(7)
    cases = []
    nx, ny = 16, 8
    y = np.arange(ny)
    west = np.zeros(ny, int)
    west[1:-1] = fw.VELOCITY
    east = np.zeros(ny, int)
    east[1:-1] = fw.PRESSURE
    u_in = 4 * 0.05 * (y + 0.5) * (ny - 0.5 - y) / ny ** 2
    u_init = np.stack([u_in[None, :] + 0.01 * rng.standard_normal((nx, ny)),
                       0.01 * rng.standard_normal((nx, ny))])
    cases.append(("channel_dp_linear", fw.Problem(
        (nx, ny), 0.56, 0.1, west=west, east=east, u_in=u_in, window_len=12, sample_every=3,
        u_init=u_init, rho_init=1 + 0.01 * rng.standard_normal((nx, ny))),
        0.6 * rng.random((nx, ny))))
    nx, ny = 12, 10
    west = np.zeros(ny, int)
    west[1:4] = fw.VELOCITY
    west[5:9] = fw.PRESSURE
    cases.append(("west_in_out_diss_paper", fw.Problem(
        (nx, ny), 0.53, 0.15, west=west, u_in=np.full(ny, 0.03), objective="diss_dp",
        s_map="paper", s_q=0.2, sec_in=(2, 1, 4), sec_out=(2, 5, 9), window_len=10,
        sample_every=2, u_init=0.02 * rng.standard_normal((2, nx, ny))), rng.random((nx, ny))))
    nx, ny = 12, 6
    cases.append(("periodic_y", fw.Problem(
        (nx, ny), 0.6, 0.1, periodic=(False, True), west=np.ones(ny, int),
        east=np.full(ny, 2), u_in=np.full(ny, 0.04), window_len=8, sample_every=4,
        u_init=0.02 * rng.standard_normal((2, nx, ny))), 0.3 * rng.random((nx, ny))))
    nx, ny, nz = 6, 5, 4
    west = np.zeros(ny, int)
    west[1:-1] = fw.VELOCITY
    east = np.zeros(ny, int)
    east[1:-1] = fw.PRESSURE
    cases.append(("d3q19_channel_diss", fw.Problem(
        (nx, ny, nz), 0.55, 0.1, periodic=(False, False, True), west=west, east=east,
        u_in=np.full(ny, 0.04), objective="diss_dp", window_len=6, sample_every=2,
        u_init=0.02 * rng.standard_normal((3, nx, ny, nz))), 0.5 * rng.random((nx, ny, nz))))
    return cases


@pytest.mark.parametrize("name,prob,gamma", _window_cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_window_gradient_complex_step(name, prob, gamma):
    """The hand-derived reverse sweep (adjoint BCs, adjoint streaming with the
    adjoint wall rule, explicit collision Jacobian, sensitivity, sampled
    sources) equals the complex-step derivative of the window objective with
    respect to every design entry (relative L2 <= 1e-12)."""
    f0 = fw.initial_state(prob)
    J, g, _ = ad.window_gradient(prob, gamma, f0)
    assert np.isclose(J, fw.window_objective(prob, gamma, f0), rtol=1e-15, atol=0)
    h = 1e-30
    cs = np.zeros_like(g)
    for idx in np.ndindex(*gamma.shape):
        gc = gamma.astype(complex)
        gc[idx] += 1j * h
        cs[idx] = fw.window_objective(prob, gc, f0).imag / h
    assert np.linalg.norm(g - cs) <= 1e-12 * np.linalg.norm(cs)
    assert np.linalg.norm(cs) > 0


@pytest.mark.parametrize("name,prob,gamma", _window_cases()[:3], ids=lambda v: v if isinstance(v, str) else "")
def test_full_gradient_complex_step(name, prob, gamma):
    """Full-time adjoint (Sec. "Comparison with full-time adjoint
    optimization"): the last window's objective with the whole history from
    f^0 depending on gamma, differentiated by the chained reverse sweep,
    equals its complex-step derivative on every design entry; it differs from
    the window-restricted gradient, whose start state is held fixed."""
    n = 3
    J, g = ad.full_gradient(prob, gamma, n)

    def start(gm):
        s = fw.design_map(prob, gm)
        f = fw.initial_state(prob).astype(complex if np.iscomplexobj(gm) else float)
        for _ in range((n - 1) * prob.window_len):
            f = fw.step(prob, f, s)
        return f

    assert J == pytest.approx(fw.window_objective(prob, gamma, start(gamma)), rel=1e-15, abs=0)
    h = 1e-30
    cs = np.zeros_like(g)
    for idx in np.ndindex(*gamma.shape):
        gc = gamma.astype(complex)
        gc[idx] += 1j * h
        cs[idx] = fw.window_objective(prob, gc, start(gc)).imag / h
    assert np.linalg.norm(g - cs) <= 1e-12 * np.linalg.norm(cs)
    _, g_win, _ = ad.window_gradient(prob, gamma, start(gamma))
    assert np.linalg.norm(g - g_win) > 1e-6 * np.linalg.norm(g)


@pytest.mark.parametrize("name,prob,gamma", _window_cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_step_dot_product(name, prob, gamma, rng):
    """<L df, nu> = <df, L^T nu> for one step, with L df by complex step."""
    s = fw.design_map(prob, gamma)
    f = fw.initial_state(prob)
    f = fw.step(prob, f, s)
    df = rng.standard_normal(f.shape)
    nu = rng.standard_normal(f.shape)
    h = 1e-30
    Ldf = fw.step(prob, f + 1j * h * df, s).imag / h
    mu, _ = ad.adjoint_step(prob, f, s, nu)
    lhs = (Ldf * nu).sum()
    rhs = (df * mu).sum()
    assert abs(lhs - rhs) <= 1e-13 * np.abs(Ldf * nu).sum()


@pytest.mark.slow
def test_finite_difference_cylinder_window():
    """Central finite differences (h = 1e-4, one of the paper's perturbation
    sizes) of the replayed window objective on a small cylinder channel agree
    with the adjoint to 1e-6 relative; the paper's own check reached < 1%
    (Sec. 4.2.1)."""
    nx, ny = 48, 20
    y = np.arange(ny)
    u_in = 4 * 0.05 * (y + 0.5) * (ny - 0.5 - y) / ny ** 2
    west = np.zeros(ny, int)
    west[1:-1] = fw.VELOCITY
    east = np.zeros(ny, int)
    east[1:-1] = fw.PRESSURE
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    r = np.hypot(X - 12, Y - 10)
    gamma = np.clip((4 + 1 - r) / 2, 0, 1)
    u_init = np.zeros((2, nx, ny))
    u_init[0] = u_in[None, :]
    prob = fw.Problem((nx, ny), 0.55, 0.1, west=west, east=east, u_in=u_in,
                      window_len=40, sample_every=1, u_init=u_init)
    f = fw.initial_state(prob)
    s = fw.design_map(prob, gamma)
    for _ in range(60):
        f = fw.step(prob, f, s)
    J, g, _ = ad.window_gradient(prob, gamma, f)
    for idx in ((16, 10), (9, 10), (13, 13), (20, 8)):
        gp = gamma.copy()
        gm = gamma.copy()
        gp[idx] += 1e-4
        gm[idx] -= 1e-4
        fd = (fw.window_objective(prob, gp, f) - fw.window_objective(prob, gm, f)) / 2e-4
        assert abs(fd - g[idx]) <= 1e-6 * abs(g[idx])


# -------------------------------------------------- window criterion (A12)

def test_window_criterion_edges():
    """Eq. statistical_criterion: strict inequality; zero mean handled; a
    negative tolerance disables the test."""
    assert fw.window_test(1.0, 1.0005, 1e-3)[1] is True
    rel, conv = fw.window_test(1.0, 1.0011, 1e-3)
    assert not conv and abs(rel - 0.0011 / 1.0011) < 1e-15
    rel, conv = fw.window_test(1.0, 1.001, 1e-3)     # |1 - 1.001| / 1.001 < 1e-3
    assert conv
    assert fw.window_test(0.0, 0.0, 1e-3)[1] is True
    assert fw.window_test(1.0, 0.0, 1e-3)[1] is False
    assert fw.window_test(1.0, 1.0, -1.0)[1] is False
    rel, conv = fw.window_test(2.0, -2.0, 1e-3)
    assert rel == 2.0 and not conv


def test_run_windows_and_sampling(rng):
    """End-aligned sampling with weights dW/|W| (Eq. weighted_temporal_sampling):
    the window objective equals the mean of the sampled instantaneous values,
    and window 1 never counts as converged."""
    nx, ny = 8, 6
    west = np.zeros(ny, int)
    west[1:-1] = fw.VELOCITY
    east = np.zeros(ny, int)
    east[1:-1] = fw.PRESSURE
    prob = fw.Problem((nx, ny), 0.6, 0.1, west=west, east=east, u_in=np.full(ny, 0.03),
                      window_len=6, sample_every=3, eps=1e9, max_windows=5,
                      u_init=0.01 * rng.standard_normal((2, nx, ny)))
    res = fw.run(prob, np.zeros((nx, ny)), 18, keep=(3, 6, 9, 12))
    st = res["states"]
    assert len(res["J"]) == 3
    assert np.isclose(res["J"][0], 0.5 * (fw.pressure_drop(prob, st[3]) + fw.pressure_drop(prob, st[6])),
                      rtol=1e-15, atol=0)
    assert np.isclose(res["J"][1], 0.5 * (fw.pressure_drop(prob, st[9]) + fw.pressure_drop(prob, st[12])),
                      rtol=1e-15, atol=0)
    assert res["converged"] == [False, True, True]
    res2 = fw.run(prob, np.zeros((nx, ny)), 30, stop_on_converge=True)
    assert res2["steps"] == 12 and res2["w_eff"] == 2
