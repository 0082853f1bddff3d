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


@pytest.mark.parametrize("prec,tol_f,tol_g", [("f32", 2e-5, 1e-4), ("f16s", 1e-2, 1e-2)])
def test_small_window_reduced(Solver, prec, tol_f, tol_g):
    name, w = _small_cases()[0]
    prob = oracle_problem(w)
    f0 = random_start_state(prob, seed=5)
    J_o, g_o, _ = ad.window_gradient(prob, w.gamma, f0)
    sv = Solver(w, prec)
    sv.set_state(f0, 0)
    sv.forward(w.window_len)
    g, J = sv.adjoint()
    assert abs(J - J_o) <= tol_f * abs(J_o) + 1e-9
    assert rel_l2(g.cpu().numpy(), g_o) <= tol_g
    sv.close()


# --------------------------------------------------------- cylinder channel

@pytest.fixture(scope="module")
def c1_oracle():
    """Cylinder channel 160 x 64, Re 100, C_s = 0.1: oracle states after 1000
    and 1500 steps, window means of windows 1-4 (|W| = 500, dW = 1) and the
    adjoint over window 4."""
    w = W.cylinder_channel()
    prob = oracle_problem(w)
    res = fw.run(prob, w.gamma, 2000, keep=(1000, 1500))
    J4, g4, _ = ad.window_gradient(prob, w.gamma, res["states"][1500])
    return dict(w=w, f1000=res["states"][1000], J=res["J"], M=res["M"], J4=J4, g4=g4)


def test_c1_fp64(Solver, c1_oracle):
    w = c1_oracle["w"]
    sv = Solver(w, "f64")
    sv.forward(1000)
    f, step = sv.get_state()
    assert step == 1000
    assert rel_l2(f, c1_oracle["f1000"]) <= 1e-12
    rep = sv.forward(1000)
    assert rep["windows_done"] == 4
    J, M, _ = sv.history()
    assert rel_l2(J, c1_oracle["J"]) <= 1e-12
    assert rel_l2(M, c1_oracle["M"]) <= 1e-12
    g, Jw = sv.adjoint()
    assert abs(Jw - c1_oracle["J4"]) <= 1e-12 * abs(c1_oracle["J4"])
    assert rel_l2(g.cpu().numpy(), c1_oracle["g4"]) <= 1e-10
    sv.close()


def test_c1_fp32(Solver, c1_oracle):
    w = c1_oracle["w"]
    sv = Solver(w, "f32")
    sv.forward(1000)
    f, _ = sv.get_state()
    assert rel_l2(f, c1_oracle["f1000"]) <= 1e-5
    sv.forward(1000)
    g, Jw = sv.adjoint()
    assert abs(Jw - c1_oracle["J4"]) <= 1e-3 * abs(c1_oracle["J4"])
    assert rel_l2(g.cpu().numpy(), c1_oracle["g4"]) <= 1e-4
    sv.close()


def test_c1_fp16s(Solver, c1_oracle):
    w = c1_oracle["w"]
    sv = Solver(w, "f16s")
    sv.forward(2000)
    g, Jw = sv.adjoint()
    err_J = abs(Jw - c1_oracle["J4"]) / abs(c1_oracle["J4"])
    err_g = rel_l2(g.cpu().numpy(), c1_oracle["g4"])
    print(f"FP16S cylinder channel: J rel err {err_J:.3e}, dJ/dgamma rel-L2 {err_g:.3e}")
    assert err_g <= 1e-2
    sv.close()
