"""Python front end of the HIP library: a Solver owning its device workspace
(torch memory on the current HIP stream) and forwarding every call to the C
ABI. No solver arithmetic happens here."""

import ctypes

import numpy as np
import torch

from . import binding as B

_PREC = {"f64": B.LBM_F64, "f32": B.LBM_F32, "f16s": B.LBM_F16S}
_OBJ = {"dp": B.LBM_J_PRESSURE_DROP, "diss_dp": B.LBM_J_DISSIPATION_PLUS_DP, "drag": B.LBM_J_DRAG,
        "wake": B.LBM_J_WAKE, "cd": B.LBM_J_DRAG}
_SMAP = {"linear": B.LBM_S_LINEAR, "paper": B.LBM_S_PAPER}


def to_device_order(a):
    """[x, y(, z)] array -> flat x-fastest node order used by the library."""
    a = np.asarray(a)
    return np.ascontiguousarray(a.transpose(tuple(range(a.ndim - 1, -1, -1)))).reshape(-1)


def from_device_order(flat, shape):
    """Inverse of to_device_order for one field."""
    rev = tuple(reversed(shape))
    a = np.asarray(flat).reshape(rev)
    return a.transpose(tuple(range(a.ndim - 1, -1, -1)))


def make_config(w, prec="f32"):
    """lbm_config for a Workload; returns (config, keep-alive buffers)."""
    shape = tuple(w.shape)
    nz = shape[2] if len(shape) == 3 else 1
    ny = shape[1]
    west = np.ascontiguousarray(np.asarray(w.west, dtype=np.int32))
    east = np.ascontiguousarray(np.asarray(w.east, dtype=np.int32))
    u_in = np.ascontiguousarray(np.asarray(w.u_in, dtype=np.float64))
    assert west.shape == (ny,) and east.shape == (ny,) and u_in.shape == (ny,)
    per = tuple(w.periodic) + (False,) * (3 - len(w.periodic))
    c = B.lbm_config()
    c.lattice = B.LBM_D2Q9 if len(shape) == 2 else B.LBM_D3Q19
    c.nx, c.ny, c.nz = shape[0], ny, nz
    c.tau = float(w.tau)
    c.c_smag = float(w.c_smag)
    c.prec = _PREC[prec]
    c.s_map = _SMAP[w.s_map]
    c.s_q = float(w.s_q)
    c.periodic_x, c.periodic_y, c.periodic_z = (int(bool(p)) for p in per)
    c.west = west.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    c.east = east.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    c.u_in = u_in.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    c.rho_out = float(w.rho_out)
    c.rho_init = float(w.rho_init)
    c.u_init_mode = int(w.u_init_mode)
    c.window_len = int(w.window_len)
    c.sample_every = int(w.sample_every)
    c.max_windows = int(w.max_windows)
    c.eps = float(w.eps)
    c.objective = _OBJ[w.objective]
    c.monitor = _OBJ[w.monitor]
    c.sec_in_x, c.sec_in_lo, c.sec_in_hi = (int(v) for v in w.sec_in)
    c.sec_out_x, c.sec_out_lo, c.sec_out_hi = (int(v) for v in w.sec_out)
    c.ckpt_every = int(w.ckpt_every)
    c.full_history = int(bool(getattr(w, "full_history", False)))
    for name in ("force_box", "meas_box"):
        box = getattr(w, name, None)
        flat = [0, 0, 0, 0, 0, 0] if box is None else [int(v) for b in box for v in b]
        flat += [0, 1] if len(flat) == 4 else []
        getattr(c, name)[:] = flat
    c.drag_ref = float(getattr(w, "drag_ref", 1.0))
    return c, (west, east, u_in)


def box_shape(w, name):
    """Node counts per axis of a Workload box (None: the whole grid)."""
    box = getattr(w, name, None)
    return tuple(w.shape) if box is None else tuple(hi - lo for lo, hi in box)


def workspace_bytes(w, prec="f32"):
    cfg, keep = make_config(w, prec)
    n = ctypes.c_size_t(0)
    B.check(B.lib.lbm_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n)))
    return n.value


class Solver:
    """One context of the library on the current HIP device and stream.

    gamma: design field indexed [x, y(, z)] (numpy or torch), 1 = solid.
    """

    def __init__(self, w, prec="f32", gamma=None, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("the solver needs a GPU (no CPU fallback)")
        self.w = w
        self.prec = prec
        self.shape = tuple(w.shape)
        self.N = int(np.prod(self.shape))
        self.Q = 9 if len(self.shape) == 2 else 19
        self.D = len(self.shape)
        self.device = torch.device(device)
        cfg, self._keep = make_config(w, prec)
        self._cfg = cfg
        n = ctypes.c_size_t(0)
        B.check(B.lib.lbm_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n)))
        self.workspace_bytes = n.value
        self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        g = self._gamma_tensor(w.gamma if gamma is None else gamma)
        self._ctx = ctypes.c_void_p()
        B.check(B.lib.lbm_init(ctypes.byref(cfg), ctypes.c_void_p(g.data_ptr()),
                               ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(n.value),
                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._ctx)))
        self.blocking = None      # library default (see lbm_set_blocking)
        # bumped by every call that changes the state, the design or the
        # objective, so that a saved adjoint request can tell it is stale
        self.generation = 0

    # ------------------------------------------------------------ helpers
    def _gamma_tensor(self, gamma):
        if isinstance(gamma, torch.Tensor):
            if tuple(gamma.shape) == self.shape:
                g = gamma.detach().to(self.device, torch.float64)
                g = g.permute(*range(g.ndim - 1, -1, -1)).contiguous().reshape(-1)
            else:
                g = gamma.detach().to(self.device, torch.float64).contiguous().reshape(-1)
        else:
            g = torch.from_numpy(to_device_order(np.asarray(gamma, np.float64))).to(self.device)
        assert g.numel() == self.N
        return g

    def _state_to_host_layout(self, flat):
        """(Q*N,) library order -> [alpha, x, y(, z)]."""
        rev = (self.Q,) + tuple(reversed(self.shape))
        a = flat.reshape(rev)
        return a.transpose((0,) + tuple(range(a.ndim - 1, 0, -1)))

    # -------------------------------------------------------------- calls
    def set_gamma(self, gamma):
        g = self._gamma_tensor(gamma)
        self.generation += 1
        B.check(B.lib.lbm_set_gamma(self._ctx, ctypes.c_void_p(g.data_ptr())))

    def reset(self):
        self.generation += 1
        B.check(B.lib.lbm_reset(self._ctx))

    def forward(self, n_steps, stop_on_converge=False):
        rep = B.lbm_fwd_report()
        self.generation += 1
        B.check(B.lib.lbm_forward(self._ctx, int(n_steps), int(bool(stop_on_converge)), ctypes.byref(rep)))
        return {k: getattr(rep, k) for k, _ in B.lbm_fwd_report._fields_}

    def history(self):
        n = ctypes.c_int(0)
        B.check(B.lib.lbm_window_history(self._ctx, None, None, None, 0, ctypes.byref(n)))
        k = n.value
        J = np.zeros(max(k, 1))
        M = np.zeros(max(k, 1))
        R = np.zeros(max(k, 1))
        P = ctypes.POINTER(ctypes.c_double)
        B.check(B.lib.lbm_window_history(self._ctx, J.ctypes.data_as(P), M.ctypes.data_as(P),
                                         R.ctypes.data_as(P), k, ctypes.byref(n)))
        return J[:k], M[:k], R[:k]

    def adjoint(self, window=0):
        """dJ/dgamma of the last completed window: (torch FP64 [x, y(, z)], J)."""
        out = torch.empty(self.N, dtype=torch.float64, device=self.device)
        J = ctypes.c_double(0.0)
        B.check(B.lib.lbm_adjoint(self._ctx, int(window), ctypes.c_void_p(out.data_ptr()), ctypes.byref(J)))
        rev = tuple(reversed(self.shape))
        g = out.reshape(rev).permute(*range(len(rev) - 1, -1, -1))
        return g, J.value

    def adjoint_full(self):
        """Full-time adjoint (needs the workload's full_history): dJ/dgamma of
        the last window's objective through the whole history, (torch FP64
        [x, y(, z)], J)."""
        out = torch.empty(self.N, dtype=torch.float64, device=self.device)
        J = ctypes.c_double(0.0)
        B.check(B.lib.lbm_adjoint_full(self._ctx, ctypes.c_void_p(out.data_ptr()), ctypes.byref(J)))
        rev = tuple(reversed(self.shape))
        g = out.reshape(rev).permute(*range(len(rev) - 1, -1, -1))
        return g, J.value

    def replay(self, gamma):
        """Objective of the last completed window replayed with gamma."""
        g = self._gamma_tensor(gamma)
        J = ctypes.c_double(0.0)
        B.check(B.lib.lbm_window_replay(self._ctx, ctypes.c_void_p(g.data_ptr()), ctypes.byref(J)))
        return J.value

    def set_wake_reference(self, u_ref):
        """Wake objective: reference mean velocity on the measurement box,
        indexed [component, x, y(, z)] relative to the box corner."""
        shp = (self.D,) + box_shape(self.w, "meas_box")
        u = np.asarray(u_ref.detach().cpu() if isinstance(u_ref, torch.Tensor) else u_ref, np.float64)
        assert u.shape == shp, (u.shape, shp)
        flat = np.concatenate([to_device_order(u[p]) for p in range(self.D)])
        t = torch.from_numpy(flat).to(self.device)
        self.generation += 1
        B.check(B.lib.lbm_set_wake_reference(self._ctx, ctypes.c_void_p(t.data_ptr())))

    def wake_mean_velocity(self):
        """Wake objective: u_bar of the last completed window on the
        measurement box, numpy [component, x, y(, z)]."""
        box = box_shape(self.w, "meas_box")
        nb = int(np.prod(box))
        t = torch.empty(self.D * nb, dtype=torch.float64, device=self.device)
        B.check(B.lib.lbm_wake_mean_velocity(self._ctx, ctypes.c_void_p(t.data_ptr())))
        flat = t.cpu().numpy()
        return np.stack([from_device_order(flat[p * nb:(p + 1) * nb], box) for p in range(self.D)])

    def get_state(self):
        """(f [alpha, x, y(, z)] FP64 numpy, step)."""
        buf = np.empty(self.Q * self.N, np.float64)
        step = ctypes.c_long(0)
        B.check(B.lib.lbm_get_state(self._ctx, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    ctypes.byref(step)))
        return np.ascontiguousarray(self._state_to_host_layout(buf)), step.value

    def set_state(self, f, step):
        f = np.asarray(f, np.float64)
        flat = np.ascontiguousarray(f.transpose((0,) + tuple(range(f.ndim - 1, 0, -1)))).reshape(-1)
        self.generation += 1
        B.check(B.lib.lbm_set_state(self._ctx, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(step)))

    def fields(self):
        """rho and u as a torch FP64 tensor [1 + D, x, y(, z)]."""
        out = torch.empty((1 + self.D) * self.N, dtype=torch.float64, device=self.device)
        B.check(B.lib.lbm_get_fields(self._ctx, ctypes.c_void_p(out.data_ptr())))
        rev = (1 + self.D,) + tuple(reversed(self.shape))
        return out.reshape(rev).permute(0, *range(len(rev) - 1, 0, -1))

    def timing(self, enable):
        out = np.zeros(11)
        B.check(B.lib.lbm_timing(self._ctx, int(bool(enable)), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return {"fwd_launches": out[0], "fwd_ms": out[1], "adj_launches": out[2], "adj_ms": out[3],
                "rec_launches": out[4], "rec_ms": out[5], "tb_launches": out[6], "tb_ms": out[7],
                "tb_steps": out[8], "rec_steps": out[9], "adj_steps": out[10]}

    def set_blocking(self, nsteps, tile_x=32, tile_y=16):
        """Temporal blocking of forward launches (D2Q9): nsteps per launch."""
        B.check(B.lib.lbm_set_blocking(self._ctx, int(nsteps), int(tile_x), int(tile_y)))
        self.blocking = (int(nsteps), int(tile_x), int(tile_y))

    def set_blocking_3d(self, nsteps, tile_x=16, tile_y=8, tile_z=8):
        """Two-step blocking of D3Q19 forward launches (nsteps 1 or 2)."""
        B.check(B.lib.lbm_set_blocking_3d(self._ctx, int(nsteps), int(tile_x), int(tile_y), int(tile_z)))
        self.blocking = (int(nsteps), int(tile_x), int(tile_y), int(tile_z))

    def set_adjoint_blocking_3d(self, nsteps, tile_x=32, tile_y=13, tile_z=64):
        """Two-step blocking of D3Q19 adjoint launches over recomputed segments."""
        B.check(B.lib.lbm_set_adjoint_blocking_3d(self._ctx, int(nsteps), int(tile_x), int(tile_y), int(tile_z)))

    def set_adjoint_blocking(self, nsteps, tile_x=32, tile_y=16):
        """Blocking of the adjoint launches over recomputed segments (D2Q9)."""
        B.check(B.lib.lbm_set_adjoint_blocking(self._ctx, int(nsteps), int(tile_x), int(tile_y)))

    def close(self):
        """Destroys the context and drops the workspace (the caching
        allocator keeps its memory until torch.cuda.empty_cache())."""
        if getattr(self, "_ctx", None):
            B.lib.lbm_destroy(self._ctx)
            self._ctx = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def state_rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


__all__ = ["Solver", "make_config", "workspace_bytes", "to_device_order", "from_device_order",
           "state_rel_l2"]
