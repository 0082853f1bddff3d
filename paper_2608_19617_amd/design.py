"""Python front end of the design update (include/lbm_design.h): a Design
owns its device workspace and forwards every call to the C ABI; fields are
FP64 arrays indexed [x, y(, z)] (torch or numpy). No design arithmetic
happens here."""

import ctypes

import numpy as np
import torch

from . import binding as B


class Design:
    """Filter, projection, volume fraction, chain rule and update step on a
    design domain `mask` (nonzero = design node); `base` is gamma off the
    domain."""

    def __init__(self, shape, mask, base, radius=4.0, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("the design update needs a GPU (no CPU fallback)")
        self.shape = tuple(int(s) for s in shape)
        self.N = int(np.prod(self.shape))
        self.device = torch.device(device)
        nx, ny = self.shape[0], self.shape[1]
        nz = self.shape[2] if len(self.shape) == 3 else 1
        n = ctypes.c_size_t(0)
        B.check(B.lib.lbm_design_workspace_bytes(nx, ny, nz, float(radius), ctypes.byref(n)))
        self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        ws = (self._ws.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        m = self._flat(torch.as_tensor(np.asarray(mask) != 0 if not isinstance(mask, torch.Tensor) else mask != 0),
                       torch.uint8)
        b = self._flat(base)
        self._ctx = ctypes.c_void_p()
        B.check(B.lib.lbm_design_init(nx, ny, nz, float(radius), ctypes.c_void_p(m.data_ptr()),
                                      ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(ws), ctypes.c_size_t(n.value),
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._ctx)))

    def _flat(self, a, dtype=torch.float64):
        t = a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a))
        t = t.detach().to(self.device, dtype)
        if tuple(t.shape) == self.shape:
            t = t.permute(*range(t.ndim - 1, -1, -1))
        return t.contiguous().reshape(-1)

    def _field(self, flat):
        rev = tuple(reversed(self.shape))
        return flat.reshape(rev).permute(*range(len(rev) - 1, -1, -1))

    def map(self, x, beta, eta=0.5):
        """(gamma [x, y(, z)], volume fraction) of the design x."""
        xf = self._flat(x)
        g = torch.empty(self.N, dtype=torch.float64, device=self.device)
        v = ctypes.c_double(0.0)
        B.check(B.lib.lbm_design_map(self._ctx, ctypes.c_void_p(xf.data_ptr()), float(beta), float(eta),
                                     ctypes.c_void_p(g.data_ptr()), ctypes.byref(v)))
        return self._field(g), v.value

    def chain(self, x, beta, eta, dJdgamma):
        """(dJ/dx, dV/dx), [x, y(, z)], for the sensitivity dJ/dgamma."""
        xf, gf = self._flat(x), self._flat(dJdgamma)
        gJ = torch.empty(self.N, dtype=torch.float64, device=self.device)
        gV = torch.empty(self.N, dtype=torch.float64, device=self.device)
        B.check(B.lib.lbm_design_chain(self._ctx, ctypes.c_void_p(xf.data_ptr()), float(beta), float(eta),
                                       ctypes.c_void_p(gf.data_ptr()), ctypes.c_void_p(gJ.data_ptr()),
                                       ctypes.c_void_p(gV.data_ptr())))
        return self._field(gJ), self._field(gV)

    def update(self, x, dJdx, dVdx, beta, eta, move, vmax, vmin=0.0):
        """(x_new [x, y(, z)], volume fraction, multiplier) of one step under
        vmin <= V <= vmax."""
        xf, gJ, gV = self._flat(x), self._flat(dJdx), self._flat(dVdx)
        xn = torch.empty(self.N, dtype=torch.float64, device=self.device)
        v, lam = ctypes.c_double(0.0), ctypes.c_double(0.0)
        B.check(B.lib.lbm_design_update(self._ctx, ctypes.c_void_p(xf.data_ptr()), ctypes.c_void_p(gJ.data_ptr()),
                                        ctypes.c_void_p(gV.data_ptr()), float(beta), float(eta), float(move),
                                        float(vmin), float(vmax), ctypes.c_void_p(xn.data_ptr()), ctypes.byref(v),
                                        ctypes.byref(lam)))
        return self._field(xn), v.value, lam.value

    def close(self):
        if self._ctx:
            B.lib.lbm_design_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def map_noalloc(shape, mask, base, x, radius, beta, eta=0.5, stream=None):
    """lbm_design_map_noalloc: (gamma [x, y(, z)], volume fraction as a
    0-dim device tensor) without a design context or workspace. The result
    tensors are allocated here by torch; the library call allocates nothing."""
    shape = tuple(int(s) for s in shape)
    dev = torch.device("cuda")

    def flat(a, dtype=torch.float64):
        t = a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a))
        t = t.detach().to(dev, dtype)
        if tuple(t.shape) == shape:
            t = t.permute(*range(t.ndim - 1, -1, -1))
        return t.contiguous().reshape(-1)

    nx, ny = shape[0], shape[1]
    nz = shape[2] if len(shape) == 3 else 1
    m = flat(torch.as_tensor(np.asarray(mask) != 0) if not isinstance(mask, torch.Tensor) else mask != 0,
             torch.uint8)
    b, xf = flat(base), flat(x)
    g = torch.empty(m.numel(), dtype=torch.float64, device=dev)
    v = torch.empty((), dtype=torch.float64, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    B.check(B.lib.lbm_design_map_noalloc(nx, ny, nz, float(radius), ctypes.c_void_p(m.data_ptr()),
                                         ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(xf.data_ptr()),
                                         float(beta), float(eta), ctypes.c_void_p(g.data_ptr()),
                                         ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(st.cuda_stream)))
    rev = tuple(reversed(shape))
    return g.reshape(rev).permute(*range(len(rev) - 1, -1, -1)), v

