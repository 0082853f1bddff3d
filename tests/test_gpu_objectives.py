"""Parity of the paper's own objectives on the GPU (through the C ABI) with
the FP64 oracle: the drag objective and the C_d monitor (Sec. 3.1 Eq. C_d,
the drag objective of the cylinder example) and the wake-recovery objective
(Sec. "Wake flow recovery"), in D2Q9 and D3Q19, single-step and blocked
launches, window-restricted and full-time adjoints, replays, and argument
errors.

Tolerances as for the other objectives: FP64 window values <= 1e-12
relative, dJ/dgamma <= 1e-11 relative L2 (1e-10 for the full-time
adjoint); FP32 J <= 1e-5 and dJ/dgamma <= 1e-4; FP16 weight-shifted storage
J <= 1e-2 and dJ/dgamma <= 1e-2."""

import numpy as np
import pytest

from oracle import adjoint as ad
from oracle import forward as fw
from paper_2608_19617_amd import workloads as W

from helpers import oracle_problem, random_start_state, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Solver():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_19617_amd.solver import Solver
    return Solver


def _u_ref(w, seed):
    shape = tuple(hi - lo for lo, hi in w.meas_box)
    return 0.02 * np.random.default_rng(seed).standard_normal((len(w.shape),) + shape)


def _cases():
    """Ragged grids and boxes: a drag box around the cylinder with the C_d
    monitor, a drag box on the inlet face with the paper's interpolation, a
    wake measurement box behind the cylinder, and D3Q19 drag and wake boxes
    (walls in y, periodic z)."""
    cases = []
    w = W.cylinder_channel(nx=70, ny=23, radius=5, center=(20, 11), window_len=24, sample_every=3,
                           ckpt_every=8, n_windows=1)
    w.gamma = np.clip(w.gamma + 0.3 * W.random_design(w.shape, 1), 0, 1)
    w.objective, w.monitor = "drag", "cd"
    w.force_box, w.drag_ref = ((13, 28), (4, 19)), 0.5 * 0.05 ** 2 * 10
    cases.append(("drag_cd", w))
    w = W.cylinder_channel(nx=45, ny=30, radius=4, center=(15, 15), window_len=20, sample_every=2,
                           ckpt_every=5, n_windows=1)
    w.s_map, w.s_q = "paper", 0.2
    w.gamma = W.random_design(w.shape, 2)
    w.objective, w.monitor = "drag", "dp"
    w.force_box = ((0, 9), (1, 29))
    cases.append(("drag_inlet_paper", w))
    w = W.cylinder_channel(nx=70, ny=23, radius=5, center=(20, 11), window_len=24, sample_every=3,
                           ckpt_every=8, n_windows=1)
    w.gamma = np.clip(w.gamma + 0.3 * W.random_design(w.shape, 3), 0, 1)
    w.objective, w.monitor = "wake", "cd"
    w.force_box, w.meas_box = ((13, 28), (4, 19)), ((33, 62), (2, 21))
    cases.append(("wake", w))
    for kind in ("drag", "wake"):
        w = W.cylinder_3d(nx=21, ny=11, nz=6, radius=3, center=(6, 5), window_len=8, sample_every=2,
                          ckpt_every=4, n_windows=1)
        w.gamma = np.clip(w.gamma + 0.2 * W.random_design(w.shape, 9), 0, 1)
        w.objective, w.monitor = kind, "cd"
        w.force_box, w.drag_ref = ((2, 11), (1, 10), (0, 6)), 0.7
        w.meas_box = ((10, 19), (2, 9), (1, 5))
        cases.append((f"d3q19_{kind}", w))
    return cases


def _oracle_window(w, f0, u_ref):
    """J, monitor mean, u_bar (wake) and dJ/dgamma of one window from f0."""
    prob = oracle_problem(w, u_ref=u_ref)
    J, g, _ = ad.window_gradient(prob, w.gamma, f0)
    s = fw.design_map(prob, w.gamma)
    wgt = w.sample_every / w.window_len
    f, M, ubar = f0, 0.0, 0.0
    msl = (slice(None),) + fw.box_slices(prob.meas_box)
    for m in range(1, w.window_len + 1):
        f = fw.step(prob, f, s)
        if m % w.sample_every == 0:
            M += wgt * fw.sample(prob, f, prob.monitor, s)
            ubar = ubar + wgt * fw.velocity(prob, f)[msl]
    return prob, J, M, ubar, g


def _gpu_window(Solver, w, prec, f0, u_ref, blocking=None):
    sv = Solver(w, prec)
    if blocking is not None:
        fwd, adj = blocking
        if len(w.shape) == 3:
            sv.set_blocking_3d(*fwd)
            sv.set_adjoint_blocking_3d(*adj)
        else:
            sv.set_blocking(*fwd)
            sv.set_adjoint_blocking(*adj)
    if w.objective == "wake":
        sv.set_wake_reference(u_ref)
    sv.set_state(f0, 0)
    rep = sv.forward(w.window_len)
    ubar = sv.wake_mean_velocity() if w.objective == "wake" else None
    g, J = sv.adjoint()
    sv.close()
    return rep, ubar, g.cpu().numpy(), J


@pytest.mark.parametrize("name,w", _cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_objective_window_fp64(Solver, name, w):
    """One window from a shared random start state: the window objective,
    the monitor mean, the wake's u_bar and dJ/dgamma of the FP64 GPU path
    against the oracle."""
    u_ref = _u_ref(w, 4) if w.objective == "wake" else None
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=31)
    _, J_o, M_o, ubar_o, g_o = _oracle_window(w, f0, u_ref)
    rep, ubar, g, J = _gpu_window(Solver, w, "f64", f0, u_ref)
    assert abs(rep["J_eff"] - J_o) <= 1e-12 * abs(J_o)
    assert abs(rep["monitor"] - M_o) <= 1e-12 * abs(M_o)
    assert J == rep["J_eff"]
    if ubar is not None:
        assert rel_l2(ubar, ubar_o) <= 1e-13
    assert rel_l2(g, g_o) <= 1e-11
    assert np.linalg.norm(g_o) > 0


@pytest.mark.parametrize("prec,tol_J,tol_g", [("f32", 1e-5, 1e-4), ("f16s", 1e-2, 1e-2)])
@pytest.mark.parametrize("case", [0, 2, 3, 4])
def test_objective_window_reduced(Solver, case, prec, tol_J, tol_g):
    name, w = _cases()[case]
    u_ref = _u_ref(w, 5) if w.objective == "wake" else None
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=32)
    _, J_o, M_o, _, g_o = _oracle_window(w, f0, u_ref)
    rep, _, g, J = _gpu_window(Solver, w, prec, f0, u_ref)
    assert abs(J - J_o) <= tol_J * abs(J_o)
    assert abs(rep["monitor"] - M_o) <= tol_J * abs(M_o)
    assert rel_l2(g, g_o) <= tol_g


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", [0, 2, 3, 4])
def test_objective_blocked_launches(Solver, case, prec):
    """Temporally blocked forward launches (D2Q9 tiles in LDS; D3Q19
    two-step z-marching blocks) sample the drag, C_d and u_bar on their last
    step, and blocked adjoint launches apply the drag and wake sources: same
    results as single-step launches (FP64 also against the oracle)."""
    name, w = _cases()[case]
    w.window_len, w.sample_every, w.ckpt_every = 12, 3, 6
    u_ref = _u_ref(w, 6) if w.objective == "wake" else None
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=33)
    single = ((1,), (1,))
    blocked = (((2, 8, 8, 4), (2, 8, 8, 4)) if len(w.shape) == 3 else ((3, 16, 16), (3, 16, 16)))
    r1, u1, g1, J1 = _gpu_window(Solver, w, prec, f0, u_ref, single)
    r2, u2, g2, J2 = _gpu_window(Solver, w, prec, f0, u_ref, blocked)
    tol = 1e-13 if prec == "f64" else 1e-5
    assert abs(J2 - J1) <= tol * abs(J1)
    assert abs(r2["monitor"] - r1["monitor"]) <= tol * abs(r1["monitor"])
    assert rel_l2(g2, g1) <= 10 * tol
    if u1 is not None:
        assert rel_l2(u2, u1) <= tol
    if prec == "f64":
        _, J_o, _, _, g_o = _oracle_window(w, f0, u_ref)
        assert abs(J2 - J_o) <= 1e-12 * abs(J_o)
        assert rel_l2(g2, g_o) <= 1e-11


@pytest.mark.parametrize("case", [0, 2, 4])
def test_objective_windows_from_rest(Solver, case):
    """Three consecutive windows from t = 0: per-window objective (the wake
    accumulator restarts at each window) and C_d means against the oracle's
    window loop, and the last window's u_bar."""
    name, w = _cases()[case]
    w.window_len, w.sample_every, w.ckpt_every, w.max_windows = 12, 3, 4, 3
    w.eps = -1.0
    u_ref = _u_ref(w, 7) if w.objective == "wake" else None
    prob = oracle_problem(w, u_ref=u_ref)
    out = fw.run(prob, w.gamma, 3 * w.window_len)
    sv = Solver(w, "f64")
    if u_ref is not None:
        sv.set_wake_reference(u_ref)
    sv.forward(3 * w.window_len)
    J, M, _ = sv.history()
    np.testing.assert_allclose(J, out["J"], rtol=1e-11, atol=0)
    np.testing.assert_allclose(M, out["M"], rtol=1e-11, atol=0)
    if u_ref is not None:
        assert rel_l2(sv.wake_mean_velocity(), out["u_bar"]) <= 1e-12
    sv.close()


@pytest.mark.parametrize("case", [0, 2])
def test_objective_replay(Solver, case):
    """lbm_window_replay with another design: the oracle's window objective
    from the same window-start state; the forward's u_bar is unchanged."""
    name, w = _cases()[case]
    u_ref = _u_ref(w, 8) if w.objective == "wake" else None
    prob = oracle_problem(w, u_ref=u_ref)
    f0 = random_start_state(prob, seed=34)
    sv = Solver(w, "f64")
    if u_ref is not None:
        sv.set_wake_reference(u_ref)
    sv.set_state(f0, 0)
    rep = sv.forward(w.window_len)
    ub = sv.wake_mean_velocity() if u_ref is not None else None
    assert sv.replay(w.gamma) == pytest.approx(rep["J_eff"], rel=1e-14)
    g2 = np.clip(w.gamma + 0.1 * W.random_design(w.shape, 12), 0, 1)
    J_o = fw.window_objective(prob, g2, f0)
    assert sv.replay(g2) == pytest.approx(J_o, rel=1e-12)
    if ub is not None:
        assert np.array_equal(sv.wake_mean_velocity(), ub)
    sv.close()


@pytest.mark.parametrize("case", [0, 2])
def test_objective_full_time_adjoint(Solver, case):
    """Full-time adjoint of the drag (explicit dD/ds of the last window only)
    and of the wake objective against the oracle's chained sweep from f^0."""
    name, w = _cases()[case]
    w.window_len, w.sample_every, w.ckpt_every, w.max_windows = 12, 3, 4, 3
    w.eps = -1.0
    w.full_history = True
    u_ref = _u_ref(w, 9) if w.objective == "wake" else None
    prob = oracle_problem(w, u_ref=u_ref)
    J_o, g_o = ad.full_gradient(prob, w.gamma, 3)
    sv = Solver(w, "f64")
    if u_ref is not None:
        sv.set_wake_reference(u_ref)
    sv.forward(3 * w.window_len)
    g, J = sv.adjoint_full()
    assert abs(J - J_o) <= 1e-12 * abs(J_o)
    assert rel_l2(g.cpu().numpy(), g_o) <= 1e-10
    sv.close()


def test_wake_reference_from_a_reference_design(Solver):
    """The paper's recipe: u_ref is the window-mean velocity of a reference
    design; the same design then gives J = 0 and dJ/dgamma = 0."""
    name, w = _cases()[2]
    sv = Solver(w, "f64")
    sv.forward(w.window_len)
    u_ref = sv.wake_mean_velocity()
    sv.close()
    sv = Solver(w, "f64")
    sv.set_wake_reference(u_ref)
    rep = sv.forward(w.window_len)
    g, J = sv.adjoint()
    assert J == 0.0 and rep["J_eff"] == 0.0
    assert np.max(np.abs(g.cpu().numpy())) == 0.0
    sv.close()


def test_objective_errors(Solver):
    """C_d monitor without drag_ref, boxes outside the grid or empty, wake
    calls with another objective or before a window: LBM_E_INVALID /
    LBM_E_STATE."""
    from paper_2608_19617_amd.binding import LbmError
    name, w = _cases()[0]
    w.drag_ref = 0.0
    with pytest.raises(LbmError, match="drag_ref"):
        Solver(w, "f32")
    w.drag_ref = 1.0
    for box in (((0, 71), (0, 23)), ((5, 10), (7, 7)), ((-1, 5), (0, 5))):
        w.force_box = box
        with pytest.raises(LbmError, match="force_box"):
            Solver(w, "f32")
    w.force_box = ((13, 28), (4, 19))
    sv = Solver(w, "f32")
    with pytest.raises(LbmError, match="LBM_E_STATE"):
        sv.set_wake_reference(np.zeros((2, 70, 23)))
    with pytest.raises(LbmError, match="LBM_E_STATE"):
        sv.wake_mean_velocity()
    sv.close()
    name, w = _cases()[2]
    w.meas_box = ((60, 80), (2, 21))
    with pytest.raises(LbmError, match="meas_box"):
        Solver(w, "f32")
    w.meas_box = ((33, 62), (2, 21))
    sv = Solver(w, "f32")
    with pytest.raises(LbmError, match="no completed window"):
        sv.wake_mean_velocity()
    sv.close()


def test_drag_and_wake_full_size(Solver):
    """Cylinder-wake grid 2048 x 512 (FP32, the library's default launches:
    a temporally blocked launch whose last step is the sampled step): a
    6-step window from a random state, with the drag over a box around the
    cylinder and the wake value over a box behind it, against the oracle's
    steps on the whole grid."""
    w = W.cylinder_wake()
    w.window_len = w.sample_every = w.ckpt_every = 6
    w.force_box = ((480, 545), (223, 289))
    w.meas_box = ((640, 1000), (160, 352))
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=35)
    s = fw.design_map(prob, w.gamma)
    f = f0
    for _ in range(6):
        f = fw.step(prob, f, s)
    D_o = fw.drag_force(prob, f, s)
    u_ref = _u_ref(w, 10)
    prob_w = oracle_problem(w, u_ref=u_ref)
    msl = (slice(None),) + fw.box_slices(prob_w.meas_box)
    Jw_o = fw.wake_value(prob_w, fw.velocity(prob_w, f)[msl])
    for kind, want in (("drag", D_o), ("wake", Jw_o)):
        w.objective, w.monitor = kind, "dp"
        sv = Solver(w, "f32")
        if kind == "wake":
            sv.set_wake_reference(u_ref)
        sv.set_state(f0, 0)
        rep = sv.forward(6)
        assert abs(rep["J_eff"] - want) <= 1e-4 * abs(want), (kind, rep["J_eff"], want)
        sv.close()


@pytest.mark.parametrize("kind", ["cylinder_drag", "wake_recovery", "u_bend_paper"])
def test_paper_examples_full_size(Solver, kind):
    """The paper's examples at their sizes with the paper's interpolation
    and their objectives (cylinder 200 x 100 at Re 51.2: drag with the C_d
    monitor; wake 200 x 50 at Re 60: wake value on the 6 x 6 measurement
    square; U-bend 240 x 192 at Re 400: pressure drop between the legs, west
    inlet and west outlet): one 20-step window (dW = 5) from a random state,
    FP64 J, monitor mean and dJ/dgamma against the oracle, FP32 within its
    tolerances."""
    if kind == "cylinder_drag":
        w = W.cylinder_drag(51.2, window_len=20, sample_every=5, ckpt_every=10)
    elif kind == "wake_recovery":
        w = W.wake_recovery(60.0, window_len=20, sample_every=5, ckpt_every=10)
    else:
        w = W.u_bend_paper(400.0, window_len=20, sample_every=5, ckpt_every=10)
    w.max_windows = 1
    u_ref = _u_ref(w, 13) if kind == "wake_recovery" else None
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=36)
    _, J_o, M_o, _, g_o = _oracle_window(w, f0, u_ref)
    for prec, tol_J, tol_g in (("f64", 1e-12, 1e-11), ("f32", 1e-5, 1e-4)):
        rep, _, g, J = _gpu_window(Solver, w, prec, f0, u_ref)
        assert abs(J - J_o) <= tol_J * abs(J_o), (prec, J, J_o)
        assert abs(rep["monitor"] - M_o) <= tol_J * abs(M_o)
        assert rel_l2(g, g_o) <= tol_g, (prec, rel_l2(g, g_o))


def test_u_bend_fd_on_a_developed_flow(Solver):
    """The paper's U-bend at Re 400 (240 x 192, FP64) after 60 000 steps from
    rest: dJ/dgamma of a 2000-step window against forward differences
    (h = 1e-6, the window replayed from its start state) at eight nodes
    within three nodes of the channel, fluid and solid, <= 1e-3 of the
    largest. (Over the paper's 20 000-step window this flow answers a
    perturbation of 1e-4 nonlinearly, so a finite-difference check needs the
    shorter window or a much smaller step.)"""
    from scipy.ndimage import binary_dilation
    w = W.u_bend_paper(400.0)
    w.window_len, w.ckpt_every, w.eps, w.max_windows = 2000, 500, -1.0, 30
    sv = Solver(w, "f64")
    sv.forward(30 * w.window_len)
    g, J = sv.adjoint()
    g = g.cpu().numpy()
    near = binary_dilation(w.gamma == 0.0, iterations=3) & w.notes["design_mask"]
    cand = np.argwhere(near)
    pts = [tuple(int(v) for v in cand[i]) for i in np.random.default_rng(0).choice(len(cand), 8, replace=False)]
    adj, fd = [], []
    for p in pts:
        gp = w.gamma.copy()
        h = 1e-6 if gp[p] + 1e-6 <= 1.0 else -1e-6
        gp[p] += h
        fd.append((sv.replay(gp) - J) / h)
        adj.append(g[p])
    sv.close()
    adj, fd = np.array(adj), np.array(fd)
    assert np.max(np.abs(adj - fd)) <= 1e-3 * np.max(np.abs(fd)), (adj, fd)
