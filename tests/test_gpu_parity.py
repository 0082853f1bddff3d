"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (relative L2 unless stated):
  FP64 storage: fields after 1000 steps <= 1e-12; window objective <= 1e-12;
                dJ/dgamma <= 1e-10 (the adjoint sums |W| steps of 9x9
                transposes in a different association order).
  FP32 storage: laminar fields <= 1e-5; dJ/dgamma <= 1e-4.
  FP16 weight-shifted storage: dJ/dgamma <= 1e-2.
"""

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


# ------------------------------------------------------------- small cases

def _small_cases():
    """Ragged grids spanning several 256-node blocks, every boundary kind."""
    cases = []
    w = W.cylinder_channel(nx=70, ny=23, radius=5, center=(20, 11), window_len=24, sample_every=3,
                           ckpt_every=8, n_windows=1)
    w.gamma = np.clip(w.gamma + 0.3 * W.random_design(w.shape, 1), 0, 1)
    cases.append(("channel_dp", w))
    w = W.cylinder_channel(nx=45, ny=30, radius=4, center=(15, 15), window_len=20, sample_every=2,
                           ckpt_every=5, n_windows=1)
    west = np.zeros(30, np.int64)
    west[2:12] = W.VELOCITY
    west[15:27] = W.PRESSURE
    w.west, w.east = west, np.zeros(30, np.int64)
    w.u_in = np.full(30, 0.03)
    w.objective = w.monitor = "diss_dp"
    w.sec_in, w.sec_out = (5, 2, 12), (5, 15, 27)
    w.s_map, w.s_q = "paper", 0.2
    w.gamma = W.random_design(w.shape, 2)
    cases.append(("west_in_out_diss_paper", w))
    w = W.cylinder_channel(nx=33, ny=12, radius=3, center=(10, 6), window_len=16, sample_every=4,
                           ckpt_every=4, n_windows=1)
    w.periodic = (False, True, False)
    w.west = np.full(12, W.VELOCITY)
    w.east = np.full(12, W.PRESSURE)
    w.u_in = np.full(12, 0.04)
    w.sec_in, w.sec_out = (0, 0, 12), (32, 0, 12)
    w.gamma = 0.4 * W.random_design(w.shape, 3)
    cases.append(("periodic_y", w))
    w = W.cylinder_channel(nx=30, ny=30, radius=4, center=(15, 15), window_len=10, sample_every=5,
                           ckpt_every=1, n_windows=1)
    w.periodic = (True, True, False)
    w.west = w.east = np.zeros(30, np.int64)
    w.gamma = 0.3 * W.random_design(w.shape, 4)
    w.objective = w.monitor = "diss_dp"
    cases.append(("periodic_box_K1", w))
    return cases


@pytest.mark.parametrize("name,w", _small_cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_small_window_fp64(Solver, name, w):
    """One window from a shared random start state: J and dJ/dgamma of the
    GPU FP64 path against the oracle's forward and hand-derived adjoint."""
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=11)
    J_o, g_o, _ = ad.window_gradient(prob, w.gamma, f0)
    sv = Solver(w, "f64")
    sv.set_state(f0, 0)
    f_back, step = sv.get_state()
    assert step == 0 and np.max(np.abs(f_back - f0)) == 0.0
    rep = sv.forward(w.window_len)
    assert rep["windows_done"] == 1 and rep["w_eff"] == 1
    assert abs(rep["J_eff"] - J_o) <= 1e-12 * abs(J_o) + 1e-18
    # the final state
    res = f0
    s = fw.design_map(prob, w.gamma)
    for _ in range(w.window_len):
        res = fw.step(prob, res, s)
    f_gpu, step = sv.get_state()
    assert step == w.window_len
    assert rel_l2(f_gpu, res) <= 1e-12
    g, J = sv.adjoint()
    assert abs(J - J_o) <= 1e-12 * abs(J_o) + 1e-18
    assert rel_l2(g.cpu().numpy(), g_o) <= 1e-11
    sv.close()


@pytest.mark.parametrize("prec,tol_f,tol_g", [("f32", 2e-5, 1e-4), ("f16s", 1e-4, 1e-2)])
def test_small_window_reduced(Solver, prec, tol_f, tol_g):
    name, w = _small_cases()[0]
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=5)
    J_o, g_o, _ = ad.window_gradient(prob, w.gamma, f0)
    sv = Solver(w, prec)
    sv.set_state(f0, 0)
    sv.forward(w.window_len)
    g, J = sv.adjoint()
    print(f"small window {prec}: J {abs(J - J_o) / abs(J_o):.2e}, dJ/dgamma {rel_l2(g.cpu().numpy(), g_o):.2e}")
    assert abs(J - J_o) <= tol_f * abs(J_o) + 1e-9
    assert rel_l2(g.cpu().numpy(), g_o) <= tol_g
    sv.close()


# --------------------------------------------------------- cylinder channel
#
# The cylinder channel (160 x 64, Re 100, tau = 0.524) amplifies round-off
# at the pressure outlet: a 1e-10 perturbation grows to 1.5e-8 of the field
# norm by step 2000 in the oracle itself, and the FP64 oracle differs from
# the same algorithm in extended precision by ~1e-11 after 1000 steps. So
# the fields are compared from t = 0 where two FP64 programs can agree
# (step 300), and at step 1000 against the extended-precision solution;
# window statistics and dJ/dgamma are compared from a shared window-start
# state (the GPU's FP64 state entering each window, handed to the oracle).

@pytest.fixture(scope="module")
def c1():
    w = W.cylinder_channel()
    prob = oracle_problem(w)
    res = fw.run(prob, w.gamma, 1000, keep=(300, 1000))
    s_ld = fw.design_map(prob, w.gamma).astype(np.longdouble)
    f_ld = fw.initial_state(prob).astype(np.longdouble)
    for _ in range(1000):
        f_ld = fw.step(prob, f_ld, s_ld)
    drift = rel_l2(res["states"][1000], f_ld.astype(np.float64))
    return dict(w=w, prob=prob, f300=res["states"][300], f1000=res["states"][1000],
                f1000_ld=f_ld.astype(np.float64), drift1000=drift)


@pytest.fixture(scope="module")
def c1_gpu64(Solver, c1):
    """GPU FP64 run over 4 windows: states entering each window, window
    means, and the adjoint of window 4."""
    w = c1["w"]
    sv = Solver(w, "f64")
    out = {"starts": {}}
    sv.forward(300)
    out["f300"], _ = sv.get_state()
    sv.forward(200)
    for k in range(3):
        f, step = sv.get_state()
        out["starts"][step] = f
        if step == 1000:
            out["f1000"] = f
        sv.forward(500)
    assert sv.get_state()[1] == 2000
    out["J"], out["M"], _ = sv.history()
    out["g4"], out["J4"] = sv.adjoint()
    out["g4"] = out["g4"].cpu().numpy()
    sv.close()
    return out


def test_c1_fp64_fields(c1, c1_gpu64):
    e300 = rel_l2(c1_gpu64["f300"], c1["f300"])
    e1000 = rel_l2(c1_gpu64["f1000"], c1["f1000"])
    e1000_ld = rel_l2(c1_gpu64["f1000"], c1["f1000_ld"])
    print(f"cylinder channel 160x64 FP64 fields: step 300 {e300:.2e}; step 1000 vs oracle {e1000:.2e}, vs extended "
          f"precision {e1000_ld:.2e} (FP64 oracle vs extended {c1['drift1000']:.2e})")
    assert e300 <= 1e-12
    # the outlet amplifies round-off, so two FP64 programs differ by about
    # 1e-11 at step 1000 (the FP64 oracle is 9.8e-12 from the
    # extended-precision solution); the GPU state is measured 8.6e-13 from
    # the extended-precision solution (1.15e-12 with an earlier build of the
    # kernels, whose multiply-add contraction differed) and 9.0e-12 from the
    # FP64 oracle
    assert e1000_ld <= 2e-12
    assert e1000 <= 2.5e-11


@pytest.fixture(scope="module")
def c1_window4(c1, c1_gpu64):
    """Oracle window objectives of windows 2-4 from the GPU's FP64
    window-start states and the oracle adjoint of window 4 from the state at
    step 1500."""
    prob = c1["prob"]
    w = c1["w"]
    J, M = [], []
    s = fw.design_map(prob, w.gamma)
    for step in sorted(c1_gpu64["starts"]):
        f = c1_gpu64["starts"][step]
        jacc = 0.0
        for m in range(1, 501):
            f = fw.step(prob, f, s)
            jacc += fw.sample(prob, f, "dp") / 500
        J.append(jacc)
    J4, g4, _ = ad.window_gradient(prob, w.gamma, c1_gpu64["starts"][1500])
    return dict(J=np.array(J), J4=J4, g4=g4)


def test_c1_fp64_windows_and_adjoint(c1_gpu64, c1_window4):
    assert len(c1_gpu64["J"]) == 4
    eJ = np.abs(c1_gpu64["J"][1:] - c1_window4["J"]) / np.abs(c1_window4["J"])
    eJ4 = abs(c1_gpu64["J4"] - c1_window4["J4"]) / abs(c1_window4["J4"])
    eg = rel_l2(c1_gpu64["g4"], c1_window4["g4"])
    print(f"cylinder channel 160x64 FP64 from shared window starts: window means {eJ.max():.2e}; J4 {eJ4:.2e}; dJ/dgamma {eg:.2e}")
    assert eJ.max() <= 1e-11
    assert eJ4 <= 1e-11
    assert eg <= 1e-10


@pytest.mark.parametrize("prec,tol_J,tol_g", [("f32", 1e-3, 1e-4), ("f16s", 3e-3, 1e-2)])
def test_c1_reduced_precision(Solver, c1, c1_gpu64, c1_window4, prec, tol_J, tol_g):
    """FP32 / FP16-shifted storage: laminar fields from t = 0 (step 300), and
    J and dJ/dgamma of window 4 from the shared FP64 window-start state."""
    w = c1["w"]
    sv = Solver(w, prec)
    sv.forward(300)
    f300, _ = sv.get_state()
    sv.set_state(c1_gpu64["starts"][1500], 1500)
    sv.forward(500)
    g, J = sv.adjoint()
    e300 = rel_l2(f300, c1["f300"])
    eJ = abs(J - c1_window4["J4"]) / abs(c1_window4["J4"])
    eg = rel_l2(g.cpu().numpy(), c1_window4["g4"])
    print(f"cylinder channel 160x64 {prec}: fields@300 {e300:.2e}; J4 {eJ:.2e}; dJ/dgamma {eg:.2e}")
    assert e300 <= (1e-5 if prec == "f32" else 1e-2)
    assert eJ <= tol_J
    assert eg <= tol_g
    sv.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("K", [2, 5, 8])
def test_d2q9_record_sweep_blocked_matches_oracle(Solver, prec, K):
    """The D2Q9 reverse sweep from moment records with blocked recompute
    launches (4 steps on 16 x 16 tiles, so segments end on a shorter launch)
    and blocked adjoint launches (3 steps), with K - 1 = 1, 4 and 7 records
    per segment, on a ragged 70 x 23 channel; J and dJ/dgamma against the
    oracle's window gradient (dJ/dgamma relative L2: FP64 1e-11, FP32 1e-4,
    FP16S 1e-2; J relative: 1e-12, 1e-3, 2e-4, the last measured at most
    2.2e-5)."""
    w = W.cylinder_channel(nx=70, ny=23, radius=5, center=(20, 11), window_len=(10 if K == 5 else 8),
                           sample_every=2, ckpt_every=K, n_windows=1)
    w.gamma = np.clip(w.gamma + 0.3 * W.random_design(w.shape, 5), 0, 1)
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=61 + K)
    J_o, g_o, _ = ad.window_gradient(prob, w.gamma, f0)
    tol_g, tol_J = {"f64": (1e-11, 1e-12), "f32": (1e-4, 1e-3), "f16s": (1e-2, 2e-4)}[prec]
    sv = Solver(w, prec)
    sv.set_blocking(4, 16, 16)
    sv.set_adjoint_blocking(3, 16, 16)
    sv.set_state(f0, 0)
    sv.forward(w.window_len)
    g, J = sv.adjoint()
    print(f"record sweep {prec} K={K}: J {abs(J - J_o) / abs(J_o):.2e}, dJ/dgamma {rel_l2(g.cpu().numpy(), g_o):.2e}")
    assert abs(J - J_o) <= tol_J * abs(J_o)
    assert rel_l2(g.cpu().numpy(), g_o) <= tol_g, rel_l2(g.cpu().numpy(), g_o)
    sv.close()


# ------------------------------------------------------------------ D3Q19

def _small_3d():
    w = W.cylinder_3d(nx=21, ny=11, nz=6, radius=3, center=(6, 5), window_len=8, sample_every=2,
                      ckpt_every=4, n_windows=1)
    w.gamma = np.clip(w.gamma + 0.2 * W.random_design(w.shape, 9), 0, 1)
    return w


@pytest.mark.parametrize("objective", ["dp", "diss_dp"])
def test_small_window_d3q19_fp64(Solver, objective):
    """D3Q19 channel (walls in y, periodic z, Zou-He on x faces): J and
    dJ/dgamma against the oracle from a shared random start state."""
    w = _small_3d()
    w.objective = w.monitor = objective
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=21)
    J_o, g_o, _ = ad.window_gradient(prob, w.gamma, f0)
    sv = Solver(w, "f64")
    sv.set_state(f0, 0)
    sv.forward(w.window_len)
    res = f0
    s = fw.design_map(prob, w.gamma)
    for _ in range(w.window_len):
        res = fw.step(prob, res, s)
    f_gpu, _ = sv.get_state()
    assert rel_l2(f_gpu, res) <= 1e-12
    g, J = sv.adjoint()
    assert abs(J - J_o) <= 1e-12 * abs(J_o)
    assert rel_l2(g.cpu().numpy(), g_o) <= 1e-11
    sv.close()


def test_small_window_d3q19_fp32(Solver):
    w = _small_3d()
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=22)
    J_o, g_o, _ = ad.window_gradient(prob, w.gamma, f0)
    sv = Solver(w, "f32")
    sv.set_state(f0, 0)
    sv.forward(w.window_len)
    g, J = sv.adjoint()
    assert abs(J - J_o) <= 1e-5 * abs(J_o)
    assert rel_l2(g.cpu().numpy(), g_o) <= 1e-4
    sv.close()


def _small_3d_cases():
    cases = [("periodic_z", _small_3d())]
    w = _small_3d()
    w.periodic = (False, False, False)        # walls on the z faces too
    cases.append(("walls_z", w))
    w = _small_3d()
    w.periodic = (True, False, True)          # no open faces
    w.west = np.zeros_like(w.west)
    w.east = np.zeros_like(w.east)
    cases.append(("periodic_xz", w))
    return cases


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("case", [0, 1, 2])
def test_blocked_d3q19_matches_single_steps(Solver, prec, case):
    """Two-step D3Q19 launches (z-marching blocks, xy tiles grown by one node
    in LDS, walls as ghost cells or z reflections, Zou-He faces, periodic
    wraps; 256 to 1024 threads, one cell each) give the states, window objectives
    and adjoint of single-step launches; FP64 also against the oracle."""
    name, w = _small_3d_cases()[case]
    w.window_len, w.sample_every, w.ckpt_every, w.max_windows = 8, 2, 4, 2
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=23 + case)
    tol = {"f64": 1e-13, "f32": 1e-6, "f16s": 1e-3}[prec]
    res = {}
    # 256-thread (a, b, c), 512-thread (e, FP64 d and f), 768-thread (d) and 1024-thread (f) launches
    blocks = (("single", (1,)), ("a", (2, 8, 8, 4)), ("b", (2, 16, 4, 4)), ("c", (2, 7, 5, 8)),
              ("d", (2, 16, 14, 2) if prec == "f64" else (2, 24, 24, 2)), ("e", (2, 16, 16, 1)),
              ("f", (2, 20, 12, 3) if prec == "f64" else (2, 30, 25, 2)))
    for key, blk in blocks:
        sv = Solver(w, prec)
        sv.set_blocking_3d(*blk) if len(blk) > 1 else sv.set_blocking_3d(1)
        sv.set_state(f0, 0)
        sv.forward(2 * w.window_len)
        f, step = sv.get_state()
        J, M, _ = sv.history()
        g, _ = sv.adjoint()
        assert step == 2 * w.window_len
        res[key] = (f, J, g.cpu().numpy())
        sv.close()
    f1, J1, g1 = res["single"]
    for key in ("a", "b", "c", "d", "e", "f"):
        f, J, g = res[key]
        assert rel_l2(f, f1) <= tol, (key, rel_l2(f, f1))
        assert np.max(np.abs(J - J1)) <= tol * np.max(np.abs(J1)) + 1e-15
        assert rel_l2(g, g1) <= 100 * tol
    if prec == "f64":
        s_ = fw.design_map(prob, w.gamma)
        f_o = f0
        for _ in range(2 * w.window_len):
            f_o = fw.step(prob, f_o, s_)
        assert rel_l2(res["a"][0], f_o) <= 1e-12


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("case", [0, 1, 2])
def test_blocked_d3q19_adjoint_matches_single_steps(Solver, prec, case):
    """Two-step D3Q19 adjoint launches (z-marching blocks, adjoint wall rule
    as ghost cells or z reflections, 0 behind open faces, one
    read-modify-write of the sensitivity per launch; 256-, 512- and, below
    FP64, 768-thread blocks) give the dJ/dgamma of single-step adjoint launches
    after the same forward launches (single and blocked)."""
    name, w = _small_3d_cases()[case]
    w.window_len, w.sample_every, w.ckpt_every, w.max_windows = 8, 2, 8, 2
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=41 + case)
    tol = {"f64": 1e-13, "f32": 1e-6, "f16s": 1e-5}[prec]
    blocks = [(8, 8, 4), (7, 5, 8), (14, 14, 2) if prec == "f64" else (16, 14, 2)]
    if prec == "f64":
        blocks.append((24, 14, 2))      # a 416-cell region: 512 threads
    else:
        blocks.append((48, 8, 4))       # 48 x 8, wider than the grid, ragged in y
        blocks.append((24, 24, 2))      # a 676-cell region: 768 threads, one input set in flight
    # each blocked adjoint against the single-step adjoint of the same forward
    # launches (forward blocking changes the rounding below FP64)
    runs = [((1,), (1,)), ((1,), (2,) + blocks[0]), ((2, 8, 8, 4), (1,))] + \
           [((2, 8, 8, 4), (2,) + blk) for blk in blocks]
    res = {}
    for fwd, adj in runs:
        sv = Solver(w, prec)
        sv.set_blocking_3d(*fwd) if len(fwd) > 1 else sv.set_blocking_3d(1)
        sv.set_adjoint_blocking_3d(*adj) if len(adj) > 1 else sv.set_adjoint_blocking_3d(1)
        sv.set_state(f0, 0)
        sv.forward(2 * w.window_len)
        g, J = sv.adjoint()
        res[(fwd, adj)] = (g.cpu().numpy(), J)
        sv.close()
    for (fwd, adj), (g, J) in res.items():
        g1, J1 = res[(fwd, (1,))]
        assert rel_l2(g, g1) <= tol, (fwd, adj, rel_l2(g, g1))
        assert J == J1, (fwd, adj, J, J1)


def _ragged_3d(walls_z):
    """100 x 37 x 9 channel: 48 x 16 x 4 blocks leave ragged tiles in x
    (100 = 2 x 48 + 4), y (37 = 2 x 16 + 5) and z (9 = 2 x 4 + 1)."""
    w = W.cylinder_3d(nx=100, ny=37, nz=9, radius=5, center=(25, 18), window_len=8, sample_every=2,
                      ckpt_every=4, n_windows=1)
    w.gamma = np.clip(w.gamma + 0.2 * W.random_design(w.shape, 17), 0, 1)
    if walls_z:
        w.periodic = (False, False, False)
    return w


# widest forward and adjoint blocks per storage precision (LDS and registers)
_WIDE_BLOCKS = {
    "f64": ([(2, 40, 8, 4), (2, 32, 10, 3)], [(2, 24, 14, 3), (2, 14, 14, 2)]),
    "f32": ([(2, 48, 16, 4), (2, 30, 25, 3)], [(2, 48, 13, 3), (2, 24, 24, 2)]),
    "f16s": ([(2, 48, 16, 4), (2, 30, 25, 3), (2, 30, 30, 2)], [(2, 48, 13, 3), (2, 24, 24, 2)]),
}


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("walls_z", [False, True])
def test_blocked_d3q19_large_regions_on_ragged_tiles(Solver, prec, walls_z):
    """The widest blocked launches on a grid that several tiles cover with
    ragged tails in x, y and z: below FP64 the 1024-thread forward and
    recompute (regions of 769-1024 cells: 48 x 16 and 30 x 25 tiles, and in
    FP16S the full 32 x 32 region) and the 768-thread adjoint (48 x 13,
    24 x 24); in FP64 the 512-thread forward and adjoint (regions of up to
    the LDS limit of about 450 and 430 cells). States, window objectives
    and dJ/dgamma equal those of single-step launches; in FP64 and FP32
    every run also matches the oracle (FP64: states 1e-12, J 1e-12,
    dJ/dgamma 1e-11; FP32: 1e-6, 1e-3, 1e-4)."""
    w = _ragged_3d(walls_z)
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=61 + walls_z)
    tol = {"f64": 1e-13, "f32": 1e-6, "f16s": 1e-3}[prec]
    tol_adj = {"f64": 1e-13, "f32": 1e-6, "f16s": 1e-5}[prec]
    fwd_wide, adj_wide = _WIDE_BLOCKS[prec]
    runs = [(fb, (1,)) for fb in [(1,)] + fwd_wide] + [(fwd_wide[0], ab) for ab in adj_wide]
    res = {}
    for fb, ab in runs:
        print(f"ragged 3D {prec} walls_z={walls_z}: forward blocks {fb}, adjoint blocks {ab}", flush=True)
        sv = Solver(w, prec)
        sv.set_blocking_3d(*fb)
        sv.set_adjoint_blocking_3d(*ab)
        sv.set_state(f0, 0)
        sv.forward(w.window_len)
        f, step = sv.get_state()
        J, _, _ = sv.history()
        g, Ja = sv.adjoint()
        assert step == w.window_len
        res[(fb, ab)] = (f, J, g.cpu().numpy(), Ja)
        sv.close()
    f1, J1, g1, _ = res[((1,), (1,))]
    for (fb, ab), (f, J, g, Ja) in res.items():
        # states and window objectives against single steps
        assert rel_l2(f, f1) <= tol, (fb, rel_l2(f, f1))
        assert np.max(np.abs(J - J1)) <= tol * np.max(np.abs(J1)) + 1e-15
        if ab == (1,):
            assert rel_l2(g, g1) <= 100 * tol, (fb, rel_l2(g, g1))
        else:
            # a blocked adjoint against the single-step adjoint after the same forward launches
            g2, _ = res[(fb, (1,))][2:]
            assert rel_l2(g, g2) <= tol_adj, (fb, ab, rel_l2(g, g2))
            assert Ja == res[(fb, (1,))][3]
    if prec in ("f64", "f32"):
        tf, tJ, tg = {"f64": (1e-12, 1e-12, 1e-11), "f32": (1e-6, 1e-3, 1e-4)}[prec]
        J_o, g_o, _ = ad.window_gradient(prob, w.gamma, f0)
        s_ = fw.design_map(prob, w.gamma)
        f_o = f0
        for _ in range(w.window_len):
            f_o = fw.step(prob, f_o, s_)
        for key, (f, J, g, Ja) in res.items():
            print(f"  {key}: state {rel_l2(f, f_o):.2e}, J {abs(Ja - J_o) / abs(J_o):.2e}, "
                  f"dJ/dgamma {rel_l2(g, g_o):.2e}")
            assert rel_l2(f, f_o) <= tf
            assert abs(Ja - J_o) <= tJ * abs(J_o)
            assert rel_l2(g, g_o) <= tg


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("K", [5, 8, 2])
def test_d3q19_record_sweep_blocked_matches_oracle(Solver, prec, K):
    """The reverse sweep from moment records with both D3Q19 blockings on:
    two-step recompute launches that store the records of both steps (and a
    single step for an odd remainder), two-step adjoint launches that read
    them, with K - 1 = 4, 7 and 1 records per segment; J and dJ/dgamma
    against the oracle's window gradient (dJ/dgamma relative L2: FP64
    1e-11, FP32 1e-4, FP16S 1e-2; J relative: 1e-12, 1e-3, 2e-4, the last
    measured at most 1.9e-5)."""
    w = _small_3d()
    w.window_len, w.sample_every, w.ckpt_every, w.max_windows = (10 if K == 5 else 8), 2, K, 1
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=51 + K)
    J_o, g_o, _ = ad.window_gradient(prob, w.gamma, f0)
    tol_g, tol_J = {"f64": (1e-11, 1e-12), "f32": (1e-4, 1e-3), "f16s": (1e-2, 2e-4)}[prec]
    sv = Solver(w, prec)
    sv.set_blocking_3d(2, 8, 8, 4)
    sv.set_adjoint_blocking_3d(2, 8, 8, 4)
    sv.set_state(f0, 0)
    sv.forward(w.window_len)
    g, J = sv.adjoint()
    print(f"record sweep {prec} K={K}: J {abs(J - J_o) / abs(J_o):.2e}, dJ/dgamma {rel_l2(g.cpu().numpy(), g_o):.2e}")
    assert abs(J - J_o) <= tol_J * abs(J_o)
    assert rel_l2(g.cpu().numpy(), g_o) <= tol_g, rel_l2(g.cpu().numpy(), g_o)
    sv.close()


def test_adjoint_blocking_3d_rejects_bad_blocks(Solver):
    """Adjoint blocks below 256 nodes, xy regions above 768 cells, FP64
    regions beyond the LDS (468 cells), three steps, and a D2Q9 context are
    refused."""
    from paper_2608_19617_amd.binding import LbmError
    name, w = _small_3d_cases()[0]
    for prec, bad in (("f32", ((2, 4, 4, 4), (2, 40, 20, 1), (3, 8, 8, 4))), ("f64", ((2, 24, 16, 2),))):
        sv = Solver(w, prec)
        for blk in bad:
            with pytest.raises(LbmError):
                sv.set_adjoint_blocking_3d(*blk)
        sv.set_adjoint_blocking_3d(2, 8, 8, 4)
        sv.close()
    w2 = W.cylinder_channel(nx=64, ny=24, radius=4, center=(16, 12), window_len=8, sample_every=2,
                            ckpt_every=4, n_windows=1)
    sv = Solver(w2, "f32")
    with pytest.raises(LbmError):
        sv.set_adjoint_blocking_3d(2, 8, 8, 4)
    sv.close()


def test_blocking_3d_rejects_bad_blocks(Solver):
    """Blocks below 256 nodes, xy regions above 1024 cells and blocks whose
    ring exceeds the LDS are refused; a D2Q9 context refuses 3D blocking."""
    from paper_2608_19617_amd.binding import LbmError
    name, w = _small_3d_cases()[0]
    sv = Solver(w, "f64")
    for blk in ((2, 4, 4, 4), (2, 40, 30, 1), (2, 30, 30, 1), (3, 8, 8, 8)):
        with pytest.raises(LbmError):
            sv.set_blocking_3d(*blk)
    sv.set_blocking_3d(2, 8, 8, 4)
    sv.close()
    w2 = W.cylinder_channel(nx=64, ny=24, radius=4, center=(16, 12), window_len=8, sample_every=2,
                            ckpt_every=4, n_windows=1)
    sv = Solver(w2, "f32")
    with pytest.raises(LbmError):
        sv.set_blocking_3d(2, 8, 8, 4)
    sv.close()


# ------------------------------------------------- replay, FD and autograd

def test_replay_matches_forward_and_fd(Solver):
    """lbm_window_replay with the unchanged design reproduces the window
    objective (to FMA-contraction differences between kernels); central finite differences of the replay (FP64,
    h = 1e-4) match the adjoint on seed-chosen entries."""
    w = W.cylinder_channel(nx=96, ny=32, radius=5, center=(24, 16), window_len=40, sample_every=2,
                           ckpt_every=10, n_windows=2)
    sv = Solver(w, "f64")
    rep = sv.forward(2 * w.window_len)
    J_fwd = rep["J_eff"]
    assert abs(sv.replay(w.gamma) - J_fwd) <= 1e-14 * abs(J_fwd)
    g, J = sv.adjoint()
    g = g.cpu().numpy()
    rng = np.random.default_rng(0)
    cand = np.argwhere((w.gamma > 0) & (w.gamma < 1))
    pick = cand[rng.choice(len(cand), 8, replace=False)]
    h = 1e-4
    for ix, iy in pick:
        gp = w.gamma.copy()
        gm = w.gamma.copy()
        gp[ix, iy] += h
        gm[ix, iy] -= h
        fd = (sv.replay(gp) - sv.replay(gm)) / (2 * h)
        assert abs(fd - g[ix, iy]) <= 1e-5 * abs(g[ix, iy]) + 1e-12
    # the forward state was not disturbed by the replays
    rep2 = sv.forward(w.window_len)
    assert rep2["windows_done"] == 3
    sv.close()


@pytest.mark.parametrize("case", ["channel_2d", "ragged_3d_blocked"])
def test_directional_derivative_matches_adjoint(Solver, case):
    """A dot-product check of the whole gradient (the validation protocol of
    Sec. 4.2.1, along one direction instead of one entry): for a seeded
    random direction v over every node (max |v| = 1), central differences
    of the replayed window objective, (J(gamma + h v) - J(gamma - h v)) / 2h,
    converge to <dJ/dgamma, v> from the adjoint as h falls (FP64, h = 1e-4
    and 1e-5: second-order convergence, and agreement to 1e-7 relative at
    1e-5). 2D: a cylinder channel in the default temporally blocked
    launches; 3D: the ragged 100 x 37 x 9 grid in the 512-thread two-step
    FP64 forward and adjoint launches from a random start state. Measured:
    2D 2.4e-7 and 2.4e-9, 3D 3.7e-9 and 5.3e-11 at h = 1e-4 and 1e-5."""
    if case == "channel_2d":
        w = W.cylinder_channel(nx=96, ny=32, radius=5, center=(24, 16), window_len=40, sample_every=2,
                               ckpt_every=10, n_windows=2)
        sv = Solver(w, "f64")
        sv.forward(2 * w.window_len)
    else:
        w = _ragged_3d(False)
        prob = oracle_problem(w)
        sv = Solver(w, "f64")
        fwd, adj = _WIDE_BLOCKS["f64"]
        sv.set_blocking_3d(*fwd[0])
        sv.set_adjoint_blocking_3d(*adj[0])
        sv.set_state(random_start_state(prob, seed=71), 0)
        sv.forward(w.window_len)
    g, J = sv.adjoint()
    g = g.cpu().numpy()
    v = np.random.default_rng(5).uniform(-1.0, 1.0, size=w.shape)
    gv = float(np.sum(g * v))
    errs = []
    for h in (1e-4, 1e-5):
        fd = (sv.replay(w.gamma + h * v) - sv.replay(w.gamma - h * v)) / (2 * h)
        errs.append(abs(fd - gv) / abs(gv))
    print(f"directional derivative {case}: <dJ/dgamma, v> = {gv:.6e}, relative FD error {errs[0]:.2e} "
          f"(h = 1e-4), {errs[1]:.2e} (h = 1e-5)")
    assert errs[1] <= 1e-7
    assert errs[1] <= errs[0] / 10 or errs[0] <= 1e-9
    sv.close()


def test_autograd_windowed_objective(Solver):
    """WindowedJ: the backward of gamma -> J is the adjoint gradient of the
    representative window (here the criterion never passes, so W_eff is the
    last of max_windows windows)."""
    import torch
    from paper_2608_19617_amd.autograd import windowed_objective
    w = W.cylinder_channel(nx=64, ny=24, radius=4, center=(16, 12), window_len=30, sample_every=3,
                           ckpt_every=10, n_windows=2)
    sv = Solver(w, "f64")
    gamma = torch.tensor(w.gamma, dtype=torch.float64, device="cuda", requires_grad=True)
    J = windowed_objective(gamma, sv, 10 * w.window_len)
    J.backward()
    sv2 = Solver(w, "f64")
    sv2.forward(2 * w.window_len)
    g_ref, J_ref = sv2.adjoint()
    assert float(J) == J_ref
    assert torch.equal(gamma.grad, g_ref)
    sv.close()
    sv2.close()


def test_error_states(Solver):
    """Calls in the wrong state report LBM_E_STATE without touching the GPU state."""
    from paper_2608_19617_amd.binding import LbmError
    w = W.cylinder_channel(nx=40, ny=16, radius=3, center=(10, 8), window_len=10, ckpt_every=5,
                           n_windows=1)
    sv = Solver(w, "f32")
    with pytest.raises(LbmError, match="LBM_E_STATE"):
        sv.adjoint()
    with pytest.raises(LbmError, match="LBM_E_STATE"):
        sv.replay(w.gamma)
    with pytest.raises(LbmError, match="LBM_E_INVALID"):
        sv.set_state(np.zeros((9,) + w.shape), 3)
    sv.forward(15)
    with pytest.raises(LbmError, match="LBM_E_STATE"):
        sv.adjoint(window=2)
    g, J = sv.adjoint(window=1)
    assert np.isfinite(g.cpu().numpy()).all()
    sv.close()


def test_unstable_run_is_reported(Solver):
    """A run that blows up (tau near 1/2, no LES, large inlet speed) reports
    LBM_E_UNSTABLE at the window end; further forward calls need a reset."""
    from paper_2608_19617_amd.binding import LbmError
    w = W.cylinder_channel(nx=64, ny=24, radius=4, center=(16, 12), window_len=50, ckpt_every=10,
                           n_windows=4, c_smag=0.0)
    w.tau = 0.5001
    w.u_in = w.u_in * 0.45 / w.u_in.max()
    sv = Solver(w, "f32")
    with pytest.raises(LbmError, match="LBM_E_UNSTABLE"):
        sv.forward(2000)
    with pytest.raises(LbmError, match="LBM_E_STATE"):
        sv.forward(1)
    sv.reset()
    sv.close()


# ------------------------------------------------------- temporal blocking

@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("case", [0, 1, 2, 3])
def test_blocked_launches_match_single_steps(Solver, prec, case):
    """Temporally blocked forward launches (several steps per launch, halos in
    LDS) give the states, window objectives and adjoint of single-step
    launches: to rounding in FP64 (multiply-add contraction may differ
    between the two kernels) and to the storage rounding in FP32 / FP16S."""
    name, w = _small_cases()[case]
    w.window_len, w.sample_every, w.ckpt_every, w.max_windows = 24, 12, 6, 2
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=3)
    tol = {"f64": 1e-13, "f32": 1e-6, "f16s": 1e-3}[prec]
    res = {}
    for nt, tile in ((1, (32, 16)), (3, (16, 16)), (4, (32, 8)), (6, (20, 13))):
        sv = Solver(w, prec)
        sv.set_blocking(nt, *tile)
        sv.set_state(f0, 0)
        sv.forward(2 * w.window_len)
        f, step = sv.get_state()
        J, M, _ = sv.history()
        g, _ = sv.adjoint()
        assert step == 2 * w.window_len
        res[nt] = (f, J, g.cpu().numpy())
        sv.close()
    f1, J1, g1 = res[1]
    for nt in (3, 4, 6):
        f, J, g = res[nt]
        assert rel_l2(f, f1) <= tol, (nt, rel_l2(f, f1))
        assert np.max(np.abs(J - J1)) <= tol * np.max(np.abs(J1)) + 1e-15
        assert rel_l2(g, g1) <= 100 * tol


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("case", [0, 1, 2, 3])
def test_long_blocks_match_single_steps(Solver, prec, case):
    """Long blocked launches (8 and 10 steps, halos of 7 and 9 nodes; FP64,
    whose LDS holds fewer values, 4 and 7 steps), so the ghost cells of the
    walls and the open-face column are reused over many LDS steps, and the
    blocked recompute of the adjoint sweep (segments of 20 steps) against
    single-step launches."""
    name, w = _small_cases()[case]
    w.window_len, w.sample_every, w.ckpt_every, w.max_windows = 40, 20, 20, 2
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=5)
    tol = {"f64": 1e-13, "f32": 1e-6, "f16s": 1e-3}[prec]
    res = {}
    blocks = ((4, (25, 25)), (7, (16, 16))) if prec == "f64" else ((8, (25, 25)), (10, (16, 16)))
    for nt, tile in ((1, (32, 16)),) + blocks:
        sv = Solver(w, prec)
        sv.set_blocking(nt, *tile)
        sv.set_state(f0, 0)
        sv.forward(2 * w.window_len)
        f, step = sv.get_state()
        J, M, _ = sv.history()
        g, _ = sv.adjoint()
        assert step == 2 * w.window_len
        res[nt] = (f, J, g.cpu().numpy())
        sv.close()
    f1, J1, g1 = res[1]
    for nt, _ in blocks:
        f, J, g = res[nt]
        assert rel_l2(f, f1) <= tol, (nt, rel_l2(f, f1))
        assert np.max(np.abs(J - J1)) <= tol * np.max(np.abs(J1)) + 1e-15
        assert rel_l2(g, g1) <= 100 * tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", [0, 1, 2, 3])
def test_adjoint_blocking_matches_single_steps(Solver, prec, case):
    """lbm_set_adjoint_blocking: blocked adjoint launches on tiles other than
    the forward's, with several depths, give the single-step adjoint's
    dJ/dgamma; bad arguments are rejected."""
    from paper_2608_19617_amd.binding import LbmError
    name, w = _small_cases()[case]
    w.window_len, w.sample_every, w.ckpt_every, w.max_windows = 40, 20, 20, 2
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=7)
    tol = {"f64": 1e-12, "f32": 1e-5}[prec]
    sv = Solver(w, prec)
    sv.set_state(f0, 0)
    sv.forward(2 * w.window_len)
    sv.set_adjoint_blocking(1)
    g1, J1 = sv.adjoint()
    g1 = g1.cpu().numpy()
    configs = {"f64": ((2, (16, 16)), (4, (25, 25)), (3, (32, 16)), (7, (16, 16))),
               "f32": ((2, (16, 16)), (5, (25, 25)), (3, (48, 24)), (10, (16, 16)))}[prec]
    with pytest.raises(LbmError, match="LBM_E_INVALID"):
        sv.set_adjoint_blocking(17, 16, 16)       # more than 16 steps
    for na, tile in configs:
        sv.set_adjoint_blocking(na, *tile)
        g, J = sv.adjoint()
        assert J == J1
        assert rel_l2(g.cpu().numpy(), g1) <= tol, (na, tile, rel_l2(g.cpu().numpy(), g1))
    with pytest.raises(LbmError, match="LBM_E_INVALID"):
        sv.set_adjoint_blocking(4, 8, 8)          # fewer than 256 nodes per tile
    with pytest.raises(LbmError, match="LBM_E_INVALID"):
        sv.set_adjoint_blocking(16, 64, 64)       # more LDS than a compute unit has
    sv.close()


# ------------------------------------------------- full-size configurations
#
# At full size the oracle cannot replay whole windows in a test, so the GPU
# (in the launch configuration the benchmark times) is compared with the
# oracle over a bounded number of steps from a shared state, and through
# properties that hold at any size.

def _share_state(Solver, w, steps, prec="f64"):
    """GPU state after `steps` steps (a multiple of the window length)."""
    sv = Solver(w, prec)
    sv.forward(steps)
    f, step = sv.get_state()
    sv.close()
    assert step == steps
    return f


def _oracle_steps(prob, gamma, f, n):
    s = fw.design_map(prob, gamma)
    for _ in range(n):
        f = fw.step(prob, f, s)
    return f


@pytest.mark.parametrize("prec,tol,tol_dp", [("f64", 1e-12, 1e-14), ("f32", 1e-5, 2e-7), ("f16s", 2e-4, 2e-5)])
def test_bfs_full_size_steps(Solver, prec, tol, tol_dp):
    """Backward-facing step 800 x 200 (benchmark workload, default blocked
    launches): 100 steps from a shared FP64 state at step 2000, against the
    oracle; and the single sampled pressure drop of a 100-step window,
    whose error is bounded relative to the pressure level c_s^2 rho_0 (the
    drop itself is 2.5e-4 of it; measured: fields 5.5e-15, 2.6e-8, 2.0e-5;
    pressure drop 6e-15, 5.1e-8, 4.0e-6 of the level)."""
    w = W.backward_facing_step()
    f0 = _share_state(Solver, w, 2000)
    w1 = W.backward_facing_step()
    w1.window_len, w1.sample_every, w1.ckpt_every, w1.max_windows = 100, 100, 100, 1
    prob = oracle_problem(w1)
    f_o = _oracle_steps(prob, w1.gamma, f0, 100)
    sv = Solver(w1, prec)
    sv.set_state(f0, 0)
    rep = sv.forward(100)
    f_g, _ = sv.get_state()
    J_o = fw.pressure_drop(prob, f_o)
    e_f = rel_l2(f_g, f_o)
    e_J = abs(rep["J_eff"] - J_o) / abs(J_o)
    print(f"BFS 800x200 {prec}: fields after 100 steps {e_f:.2e}, sampled dp {e_J:.2e} (dp = {J_o:.3e})")
    assert e_f <= tol
    assert abs(rep["J_eff"] - J_o) <= tol_dp / 3.0
    sv.close()


def test_bfs_window_criterion_fp32_vs_fp64(Solver):
    """The consecutive-window test on the benchmark workload: FP32 and FP64
    take the same decision for every window whose FP64 relative change is not
    within the FP32 error margin of eps (Eq. statistical_criterion)."""
    w = W.backward_facing_step()
    hist = {}
    for prec in ("f64", "f32"):
        sv = Solver(w, prec)
        rep = sv.forward(w.max_windows * w.window_len, stop_on_converge=True)
        hist[prec] = (rep, sv.history())
        sv.close()
    rep64, (J64, M64, R64) = hist["f64"]
    rep32, (J32, M32, R32) = hist["f32"]
    print(f"BFS windows: FP64 converged={rep64['converged']} w_eff={rep64['w_eff']}; "
          f"FP32 converged={rep32['converged']} w_eff={rep32['w_eff']}; "
          f"FP64 rel changes {np.round(R64[1:6], 4)}")
    n = min(len(R64), len(R32))
    for i in range(1, n):
        if abs(R64[i] - w.eps) > 0.5 * abs(R64[i]) + 1e-3:
            assert (R64[i] < w.eps) == (R32[i] < w.eps)
    assert np.all(np.isfinite(J32)) and np.all(np.isfinite(J64))


def test_cylinder_wake_full_size_fp32(Solver):
    """Cylinder wake 2048 x 512 (Re 1000, LES): 10 steps from a shared FP64
    state at step 1000 in FP32 against the oracle."""
    w = W.cylinder_wake(window_len=1000, ckpt_every=100, sample_every=20, max_windows=1)
    f0 = _share_state(Solver, w, 1000)
    w1 = W.cylinder_wake(window_len=10, ckpt_every=10, sample_every=10, max_windows=1)
    prob = oracle_problem(w1)
    f_o = _oracle_steps(prob, w1.gamma, f0, 10)
    sv = Solver(w1, "f32")
    sv.set_state(f0, 0)
    sv.forward(10)
    f_g, _ = sv.get_state()
    e = rel_l2(f_g, f_o)
    print(f"cylinder wake 2048x512 FP32: fields after 10 steps {e:.2e}")
    assert e <= 1e-5
    sv.close()


def test_cylinder_wake_fd_check(Solver):
    """Cylinder wake 2048 x 512, FP64: central finite differences (h = 1e-4)
    of the replayed window objective on 16 seed-chosen design entries (disk
    ramp and near wake) against the adjoint, with the paper's < 1% bar
    (Sec. 4.2.1). Window of 2000 steps after 2000 steps of spin-up: long
    enough for sound to carry the disk's influence to both pressure sections
    (a shorter window has dJ/dgamma = 0 there)."""
    w = W.cylinder_wake(window_len=2000, ckpt_every=100, sample_every=20, max_windows=2)
    sv = Solver(w, "f64")
    sv.forward(4000)
    g, J = sv.adjoint()
    g = g.cpu().numpy()
    rng = np.random.default_rng(0)
    X, Y = np.meshgrid(np.arange(2048), np.arange(512), indexing="ij")
    cand = np.argwhere(((w.gamma > 0) & (w.gamma < 1)) |
                       ((X >= 544) & (X < 704) & (np.abs(Y - 256) <= 64)))
    pick = cand[rng.choice(len(cand), 16, replace=False)]
    errs = []
    for ix, iy in pick:
        gp = w.gamma.copy()
        gm = w.gamma.copy()
        gp[ix, iy] += 1e-4
        gm[ix, iy] -= 1e-4
        fd = (sv.replay(gp) - sv.replay(gm)) / 2e-4
        assert g[ix, iy] != 0.0
        errs.append(abs(fd - g[ix, iy]) / abs(g[ix, iy]))
    errs = np.array(errs)
    print(f"cylinder wake FD check: max rel err {errs.max():.2e}, median {np.median(errs):.2e}, "
          f"|dJ/dgamma| of the entries {np.abs(g[tuple(pick.T)]).min():.2e}..{np.abs(g[tuple(pick.T)]).max():.2e}")
    assert errs.max() <= 1e-3
    sv.close()


@pytest.fixture(scope="module")
def wake_window_oracle(Solver):
    """Cylinder wake 2048 x 512: the GPU FP64 state after 1000 steps, and the
    oracle's J and window gradient of a 10-step window from it (samples at
    steps 5 and 10) with the pressure sections across the cylinder
    (x = 505 and 520, every open row), so the adjoint reaches the disk, its
    ramp and the flow around it."""
    w = W.cylinder_wake(window_len=1000, ckpt_every=100, sample_every=20, max_windows=1)
    f0 = _share_state(Solver, w, 1000)
    w1 = W.cylinder_wake(window_len=10, ckpt_every=10, sample_every=5, max_windows=1)
    w1.sec_in, w1.sec_out = (505, 1, 511), (520, 1, 511)
    J_o, g_o, _ = ad.window_gradient(oracle_problem(w1), w1.gamma, f0)
    return w1, f0, J_o, g_o


@pytest.mark.parametrize("prec,tol_J,tol_g", [("f64", 1e-15, 1e-10), ("f32", 1e-9, 1e-4), ("f16s", 1e-5, 1e-2)])
def test_cylinder_wake_full_size_adjoint_vs_oracle(Solver, wake_window_oracle, prec, tol_J, tol_g):
    """The library's default launches at 2048 x 512 (temporally blocked
    forward, recompute and adjoint) over a 10-step window from a shared
    state: J and dJ/dgamma on the whole grid against the oracle (Sec. 3.2,
    Eqs. adjoint_collision, adjoint_streaming, sensitivity). J here is a
    pressure drop of about 1e-4 of the pressure level c_s^2 rho_0, so its
    error is bounded relative to that level (measured: FP64 9e-17, FP32
    1.4e-10, FP16S 1.5e-6); dJ/dgamma relative L2 (measured 1e-15, 1.3e-7,
    1.0e-4) against the bars 1e-10, 1e-4, 1e-2."""
    w1, f0, J_o, g_o = wake_window_oracle
    sv = Solver(w1, prec)
    sv.set_state(f0, 0)
    sv.forward(w1.window_len)
    g, J = sv.adjoint()
    g = g.cpu().numpy()
    eJ = abs(J - J_o) / abs(J_o)
    eg = rel_l2(g, g_o)
    print(f"cylinder wake 2048x512 {prec}: 10-step window J {eJ:.2e} (J = {J_o:.3e}), dJ/dgamma {eg:.2e}, "
          f"nonzero entries {np.count_nonzero(g_o)}")
    assert np.count_nonzero(g_o) == 2 * 18 * 512       # 9 columns either side of each section
    assert abs(J - J_o) <= tol_J / 3.0
    assert eg <= tol_g
    sv.close()


# the oracle's crop of the D3Q19 channel: x 69-91, y 51-76, every z
_C3_X0, _C3_X1, _C3_Y0, _C3_Y1 = 69, 92, 51, 77


@pytest.fixture(scope="module")
def cylinder_3d_window_oracle(Solver):
    """D3Q19 channel 384 x 128 x 128: the GPU FP64 state after 200 steps and
    the oracle's J and window gradient of a 4-step window from it (samples
    at steps 2 and 4) with pressure sections at x = 78 and x = 82 over rows
    60-67 and every z, across the front of the cylinder (its surface at
    x = 80). Over 4 steps the gradient reaches at most 4 nodes from a
    section, and the forward state there depends on the start state at most
    4 nodes further, so the oracle computes J and the gradient exactly on a
    crop whose faces are 9 nodes from the sections (walls on the crop's
    faces change nothing within 4 steps of them); the full grid's gradient
    is exactly 0 outside the crop."""
    w = W.cylinder_3d(window_len=200, sample_every=20, ckpt_every=50, n_windows=1)
    f0 = _share_state(Solver, w, 200)
    w1 = W.cylinder_3d(window_len=4, sample_every=2, ckpt_every=4, n_windows=1)
    w1.sec_in, w1.sec_out = (78, 60, 68), (82, 60, 68)
    x0, x1, y0, y1 = _C3_X0, _C3_X1, _C3_Y0, _C3_Y1
    c = W.cylinder_3d(nx=x1 - x0, ny=y1 - y0, nz=w1.shape[2], window_len=4, sample_every=2, ckpt_every=4,
                      n_windows=1)
    c.tau, c.c_smag = w1.tau, w1.c_smag
    c.gamma = w1.gamma[x0:x1, y0:y1, :].copy()
    c.west, c.east = np.zeros_like(c.west), np.zeros_like(c.east)
    c.sec_in, c.sec_out = (78 - x0, 60 - y0, 68 - y0), (82 - x0, 60 - y0, 68 - y0)
    J_o, g_o, _ = ad.window_gradient(oracle_problem(c), c.gamma, np.ascontiguousarray(f0[:, x0:x1, y0:y1, :]))
    return w1, f0, J_o, g_o


@pytest.mark.parametrize("prec,tol_J,tol_g", [("f64", 1e-15, 1e-10), ("f32", 1e-9, 1e-4), ("f16s", 1e-5, 1e-2)])
def test_cylinder_3d_full_size_adjoint_vs_oracle(Solver, cylinder_3d_window_oracle, prec, tol_J, tol_g):
    """The library's default launches on the D3Q19 channel 384 x 128 x 128
    (two-step z-marching forward, recompute and adjoint in FP64 and FP32;
    single-step forward and recompute with the two-step adjoint in FP16S)
    over a 4-step window from a shared state: J against the oracle (bounded
    relative to the pressure level c_s^2 rho_0, as the pressure drop between
    sections 4 nodes apart is small; measured FP64 4.5e-17, FP32 1.6e-11,
    FP16S 1.6e-7), dJ/dgamma on the oracle's crop (relative L2, measured
    5.3e-15, 9.2e-8, 7.0e-5 against the bars 1e-10, 1e-4, 1e-2) and exactly 0
    on the rest of the grid (Sec. 3.2, Eqs. adjoint_collision,
    adjoint_streaming, sensitivity)."""
    w1, f0, J_o, g_o = cylinder_3d_window_oracle
    sv = Solver(w1, prec)
    sv.set_state(f0, 0)
    sv.forward(w1.window_len)
    g, J = sv.adjoint()
    g = g.cpu().numpy()
    sv.close()
    inside = g[_C3_X0:_C3_X1, _C3_Y0:_C3_Y1, :]
    outside = np.count_nonzero(g) - np.count_nonzero(inside)
    eg = rel_l2(inside, g_o)
    print(f"cylinder 3D 384x128x128 {prec}: 4-step window J {abs(J - J_o):.2e} absolute (J = {J_o:.3e}), "
          f"dJ/dgamma {eg:.2e} on the crop, nonzero entries {np.count_nonzero(g_o)} (oracle), "
          f"{outside} outside the crop")
    assert np.count_nonzero(g_o) > 20000
    assert outside == 0
    assert abs(J - J_o) <= tol_J / 3.0
    assert eg <= tol_g


@pytest.fixture(scope="module")
def u_bend_window_oracle(Solver):
    """U-bend 1024 x 1024: the GPU FP64 state after 1000 steps and the
    oracle's J and window gradient of a 4-step window from it (dissipation
    plus pressure drop, samples at steps 2 and 4): the dissipation sums over
    every node, so the gradient is nonzero on the whole grid."""
    w = W.u_bend(window_len=200, sample_every=20, ckpt_every=20, max_windows=1)
    f0 = _share_state(Solver, w, 1000)
    w1 = W.u_bend(window_len=4, sample_every=2, ckpt_every=4, max_windows=1)
    J_o, g_o, _ = ad.window_gradient(oracle_problem(w1), w1.gamma, f0)
    return w1, f0, J_o, g_o


@pytest.mark.parametrize("prec,tol_J,tol_g", [("f64", 1e-13, 1e-10), ("f32", 2e-6, 1e-4), ("f16s", 5e-4, 1e-2)])
def test_u_bend_full_size_adjoint_vs_oracle(Solver, u_bend_window_oracle, prec, tol_J, tol_g):
    """The U-bend in the default launches of each precision (west inlet and
    west outlet rows, dissipation objective), 4-step window from a shared
    state: J and dJ/dgamma on all 1M nodes against the oracle (J relative,
    measured 6e-15, 1.6e-7, 6.7e-5; dJ/dgamma relative L2, measured 7e-15,
    3.5e-7, 7.7e-4). The gradient is nonzero wherever the flow has reached
    by step 1000 (u = 0 makes the node's sensitivity term vanish)."""
    w1, f0, J_o, g_o = u_bend_window_oracle
    sv = Solver(w1, prec)
    sv.set_state(f0, 0)
    sv.forward(w1.window_len)
    g, J = sv.adjoint()
    g = g.cpu().numpy()
    eJ = abs(J - J_o) / abs(J_o)
    eg = rel_l2(g, g_o)
    print(f"U-bend 1024x1024 {prec}: 4-step window J {eJ:.2e} (J = {J_o:.3e}), dJ/dgamma {eg:.2e}, "
          f"nonzero entries {np.count_nonzero(g_o)}")
    assert np.count_nonzero(g_o) > 200000
    assert eJ <= tol_J
    assert eg <= tol_g
    sv.close()


def test_u_bend_full_size_precisions(Solver):
    """U-bend 1024 x 1024 (dissipation + pressure drop objective, west inlet
    and west outlet): dJ/dgamma over a 200-step window from a shared FP64
    state, FP32 and FP16S against FP64 (<= 1e-4 and <= 1e-2)."""
    w = W.u_bend(window_len=200, sample_every=20, ckpt_every=20, max_windows=1)
    f0 = _share_state(Solver, w, 1000)
    res = {}
    for prec in ("f64", "f32", "f16s"):
        sv = Solver(w, prec)
        sv.set_state(f0, 0)
        sv.forward(w.window_len)
        g, J = sv.adjoint()
        res[prec] = (g.cpu().numpy(), J)
        sv.close()
    g64, J64 = res["f64"]
    e32 = rel_l2(res["f32"][0], g64)
    e16 = rel_l2(res["f16s"][0], g64)
    print(f"U-bend 1024x1024 dJ/dgamma vs FP64: FP32 {e32:.2e}, FP16S {e16:.2e}; J FP32 "
          f"{abs(res['f32'][1] - J64) / abs(J64):.2e}, FP16S {abs(res['f16s'][1] - J64) / abs(J64):.2e}")
    assert e32 <= 1e-4
    assert e16 <= 1e-2


def test_u_bend_oracle_one_step(Solver):
    """U-bend at full size: one step from a shared state against the oracle
    (FP64), covering the west velocity and west pressure rows at scale."""
    w = W.u_bend(window_len=200, sample_every=20, ckpt_every=20, max_windows=1)
    f0 = _share_state(Solver, w, 200)
    w1 = W.u_bend(window_len=2, sample_every=2, ckpt_every=2, max_windows=1)
    prob = oracle_problem(w1)
    f_o = _oracle_steps(prob, w1.gamma, f0, 2)
    sv = Solver(w1, "f64")
    sv.set_state(f0, 0)
    rep = sv.forward(2)
    f_g, _ = sv.get_state()
    assert rel_l2(f_g, f_o) <= 1e-13
    J_o = fw.sample(prob, f_o, "diss_dp")
    assert abs(rep["J_eff"] - J_o) <= 1e-11 * abs(J_o)
    sv.close()


def test_cylinder_3d_full_size(Solver):
    """D3Q19 channel 384 x 128 x 128 in the default (two-step) launches: 2
    steps from a shared FP64 state against the oracle (FP64 and FP32), and
    dJ/dgamma of a 40-step window from the shared state, FP64 against the
    FP64 single-step launches (<= 1e-12) and FP32 against FP64 (<= 1e-4)."""
    w = W.cylinder_3d(window_len=40, sample_every=20, ckpt_every=10, n_windows=1)
    f0 = _share_state(Solver, w, 200)
    w1 = W.cylinder_3d(window_len=2, sample_every=2, ckpt_every=2, n_windows=1)
    prob = oracle_problem(w1)
    f_o = _oracle_steps(prob, w1.gamma, f0, 2)
    for prec, tol in (("f64", 1e-13), ("f32", 1e-6)):
        sv = Solver(w1, prec)
        sv.set_state(f0, 0)
        sv.forward(2)
        f_g, _ = sv.get_state()
        e = rel_l2(f_g, f_o)
        print(f"cylinder 3D {prec}: 2 steps {e:.2e}")
        assert e <= tol
        sv.close()
    del f_o
    res = {}
    for prec, single in (("f64", False), ("f64", True), ("f32", False)):
        sv = Solver(w, prec)
        if single:
            sv.set_blocking_3d(1)
            sv.set_adjoint_blocking_3d(1)
        sv.set_state(f0, 0)
        sv.forward(w.window_len)
        g, J = sv.adjoint()
        res[(prec, single)] = (g.cpu().numpy(), J)
        sv.close()
    g64, J64 = res[("f64", False)]
    g64s, J64s = res[("f64", True)]
    e64 = rel_l2(g64, g64s)
    e = rel_l2(res[("f32", False)][0], g64)
    print(f"cylinder 3D dJ/dgamma: FP64 two-step vs single-step launches {e64:.2e}, "
          f"J {abs(J64 - J64s) / abs(J64s):.2e}; FP32 vs FP64 {e:.2e}")
    assert e64 <= 1e-12
    assert abs(J64 - J64s) <= 1e-12 * abs(J64s)
    assert e <= 1e-4


# ------------------------------------------------------ full-time adjoint

def _full_cases():
    w = W.cylinder_channel(nx=40, ny=18, radius=3, center=(12, 9), window_len=12, sample_every=3,
                           ckpt_every=4, n_windows=3)
    w.gamma = np.clip(w.gamma + 0.3 * W.random_design(w.shape, 2), 0, 1)
    cases = [("channel", w)]
    w3 = _small_3d_cases()[1][1]
    w3.window_len, w3.sample_every, w3.ckpt_every, w3.max_windows = 6, 2, 3, 3
    cases.append(("d3q19_walls_z", w3))
    return cases


@pytest.mark.parametrize("name,w", _full_cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_full_time_adjoint_matches_oracle(Solver, name, w):
    """lbm_adjoint_full (every window's start state kept; earlier windows
    replayed to rebuild their checkpoints; their reverse sweeps chained from
    the adjoint of the next window's start state, with no objective source)
    against the oracle's full-time gradient from f^0 (FP64 <= 1e-10), FP32
    against FP64 (<= 1e-4); the window-restricted adjoint is unchanged by it
    and differs from it."""
    w.eps = -1.0
    w.full_history = True
    n = 3
    prob = oracle_problem(w)
    J_o, g_o = ad.full_gradient(prob, w.gamma, n)
    res = {}
    for prec in ("f64", "f32"):
        sv = Solver(w, prec)
        rep = sv.forward(n * w.window_len)
        assert rep["windows_done"] == n
        g_win, J_win = sv.adjoint()
        g, J = sv.adjoint_full()
        g_win2, _ = sv.adjoint()
        assert np.array_equal(g_win.cpu().numpy(), g_win2.cpu().numpy())
        res[prec] = (g.cpu().numpy(), J, g_win.cpu().numpy())
        sv.close()
    g64, J64, gw64 = res["f64"]
    assert abs(J64 - J_o) <= 1e-12 * abs(J_o) + 1e-18
    assert rel_l2(g64, g_o) <= 1e-10
    assert rel_l2(g64, gw64) > 1e-6
    assert rel_l2(res["f32"][0], g64) <= 1e-4


def test_full_time_adjoint_errors(Solver):
    """Without full history, before a window ends, or with more windows than
    max_windows since the start of the history: LBM_E_STATE."""
    from paper_2608_19617_amd.binding import LbmError
    w = W.cylinder_channel(nx=40, ny=18, radius=3, center=(12, 9), window_len=8, sample_every=2,
                           ckpt_every=4, n_windows=2)
    sv = Solver(w, "f32")
    sv.forward(w.window_len)
    with pytest.raises(LbmError, match="full_history"):
        sv.adjoint_full()
    sv.close()
    w.full_history = True
    sv = Solver(w, "f32")
    with pytest.raises(LbmError, match="LBM_E_STATE"):
        sv.adjoint_full()
    sv.forward(3 * w.window_len)
    with pytest.raises(LbmError, match="max_windows"):
        sv.adjoint_full()
    sv.reset()
    sv.forward(2 * w.window_len)
    g, J = sv.adjoint_full()
    assert np.isfinite(J) and np.all(np.isfinite(g.cpu().numpy()))
    sv.close()
