"""Test-side glue: builds the oracle's problem description from a workload
(the same seeded inputs the HIP path receives) and compares results."""

import numpy as np

from oracle import forward as fw


def oracle_problem(w, window_len=None, sample_every=None, u_ref=None):
    """oracle.forward.Problem for a Workload (same inputs, independent code);
    u_ref: the wake objective's reference mean velocity (None: zero)."""
    d = len(w.shape)
    u_init = np.zeros((d,) + tuple(w.shape))
    if w.u_init_mode == 1:
        sl = (0,) + (slice(None),) * d
        u_init[0] = np.broadcast_to(
            np.asarray(w.u_in).reshape((1, -1) + (1,) * (d - 2)), w.shape)
    per = tuple(w.periodic)[:d]
    return fw.Problem(
        w.shape, w.tau, w.c_smag, periodic=per, west=w.west, east=w.east, u_in=w.u_in,
        rho_out=w.rho_out, s_map=w.s_map, s_q=w.s_q, objective=w.objective, monitor=w.monitor,
        sec_in=w.sec_in, sec_out=w.sec_out,
        window_len=w.window_len if window_len is None else window_len,
        sample_every=w.sample_every if sample_every is None else sample_every,
        eps=w.eps, max_windows=w.max_windows, rho_init=w.rho_init, u_init=u_init,
        force_box=_box3(w.force_box, d), drag_ref=w.drag_ref, meas_box=_box3(w.meas_box, d), u_ref=u_ref)


def _box3(box, d):
    return None if box is None else tuple(tuple(b) for b in box)[:d]


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def random_start_state(prob, seed, amp=0.01, u_amp=0.03):
    """Seeded near-equilibrium start state (test input): f^eq of random
    smooth-ish density and velocity plus small random non-equilibrium parts,
    so that Pi != 0 everywhere."""
    rng = np.random.default_rng(seed)
    lat = prob.lat
    rho = 1.0 + amp * rng.standard_normal(prob.shape)
    u = u_amp * rng.standard_normal((lat.d,) + prob.shape)
    f = fw.equilibrium(lat, rho, u)
    w = lat.w.reshape((-1,) + (1,) * len(prob.shape))
    return f + amp * w * rng.standard_normal(f.shape)
