"""C-ABI contract on the CPU: the library loads, exports every symbol that
include/*.h declares, validates configurations before any HIP call, and
its workspace sizing matches the documented layout. No kernel runs here."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names.update(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def B():
    from paper_2608_19617_amd import binding
    return binding


def test_exports_every_declared_symbol(B):
    declared = _declared_functions()
    assert len(declared) >= 14
    assert sorted(B.EXPORTED) == declared
    for name in declared:
        assert hasattr(B.lib, name), name


def test_header_is_plain_c():
    """The headers compile as C (no HIP, torch or C++ types)."""
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        with open(src, "w") as fh:
            fh.write('#include "lbm.h"\n#include "lbm_design.h"\n'
                     'int main(void){lbm_config c; lbm_design* d = 0; (void)c; (void)d; return 0;}\n')
        r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                            "-c", src, "-o", os.path.join(d, "t.o")], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


def _cfg(B, **over):
    from paper_2608_19617_amd import workloads as W
    from paper_2608_19617_amd.solver import make_config
    w = W.cylinder_channel(nx=40, ny=16, radius=3, center=(10, 8), window_len=20, ckpt_every=5)
    for k, v in over.items():
        setattr(w, k, v)
    return make_config(w)


def _bytes(B, cfg):
    n = ctypes.c_size_t(0)
    st = B.lib.lbm_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n))
    return st, n.value


def test_workspace_layout(B):
    cfg, keep = _cfg(B)
    st, n = _bytes(B, cfg)
    assert st == B.LBM_OK
    N, Q = 40 * 16, 9
    state = -(-Q * N * 4 // 256) * 256
    record = -(-6 * N * 4 // 256) * 256
    # two ping-pong states, two rings of |W|/K = 4 slots, two recompute states
    # and K - 1 = 4 moment records (drho, j, Pi) of the recomputed steps
    fixed = (2 + 2 * 4 + 2) * state + 4 * record
    assert n >= fixed
    assert n < fixed + 2 * 2 * Q * N * 4 + 64 * 1024 + 20 * 3 * 8 * 8


@pytest.mark.parametrize("prec,ss,cs", [(0, 8, 8), (1, 4, 4), (2, 2, 4)])
def test_workspace_layout_3d(B, prec, ss, cs):
    """D3Q19: the records hold 10 values per node (drho, j, Pi) in the
    compute precision, whatever the storage precision."""
    from paper_2608_19617_amd import workloads as W
    from paper_2608_19617_amd.solver import make_config
    w = W.cylinder_3d(nx=24, ny=12, nz=6, radius=3, center=(8, 6), window_len=20, sample_every=5,
                      ckpt_every=5, n_windows=2)
    cfg, keep = make_config(w, ("f64", "f32", "f16s")[prec])
    st, n = _bytes(B, cfg)
    assert st == B.LBM_OK
    N, Q = 24 * 12 * 6, 19
    state = -(-Q * N * ss // 256) * 256
    record = -(-10 * N * cs // 256) * 256
    fixed = (2 + 2 * 4 + 2) * state + 4 * record
    assert n >= fixed
    assert n < fixed + 2 * 2 * Q * N * 8 + 64 * 1024 + 20 * 3 * 8 * 8 + 4 * N * 8


@pytest.mark.parametrize("field,value", [
    ("tau", 0.5), ("tau", float("nan")), ("c_smag", -0.1), ("window_len", 0),
    ("sample_every", 3), ("ckpt_every", 3), ("max_windows", 0), ("eps", float("nan")),
    ("rho_out", 0.0), ("sec_in", (0, 5, 5)), ("sec_out", (40, 1, 15)), ("u_init_mode", 2),
])
def test_invalid_configs_rejected(B, field, value):
    cfg, keep = _cfg(B, **{field: value})
    st, _ = _bytes(B, cfg)
    assert st == B.LBM_E_INVALID
    assert len(B.lib.lbm_last_error()) > 0


def test_invalid_rows_rejected(B):
    from paper_2608_19617_amd import workloads as W
    from paper_2608_19617_amd.solver import make_config
    w = W.cylinder_channel(nx=40, ny=16, radius=3, center=(10, 8), window_len=20, ckpt_every=5)
    w.west = w.west.copy()
    w.west[0] = 1                       # velocity row touching the y wall
    cfg, keep = make_config(w)
    assert _bytes(B, cfg)[0] == B.LBM_E_INVALID
    w = W.cylinder_channel(nx=40, ny=16, radius=3, center=(10, 8), window_len=20, ckpt_every=5)
    w.east = w.east.copy()
    w.east[4] = 1                       # east velocity rows are not modelled
    cfg, keep = make_config(w)
    assert _bytes(B, cfg)[0] == B.LBM_E_INVALID
    w = W.cylinder_channel(nx=40, ny=16, radius=3, center=(10, 8), window_len=20, ckpt_every=5)
    w.u_in = np.full(16, 0.7)           # |u0| must stay below 0.5
    cfg, keep = make_config(w)
    assert _bytes(B, cfg)[0] == B.LBM_E_INVALID


def test_null_arguments(B):
    assert B.lib.lbm_workspace_bytes(None, None) == B.LBM_E_INVALID
    cfg, keep = _cfg(B)
    assert B.lib.lbm_forward(None, 1, 0, None) == B.LBM_E_INVALID
    assert B.lib.lbm_adjoint(None, 0, None, None) == B.LBM_E_INVALID
    out = ctypes.c_void_p()
    # NULL gamma and workspace are rejected before any HIP call
    assert B.lib.lbm_init(ctypes.byref(cfg), None, None, 0, None, ctypes.byref(out)) == B.LBM_E_INVALID
    # misaligned workspace
    assert B.lib.lbm_init(ctypes.byref(cfg), ctypes.c_void_p(256), ctypes.c_void_p(258), 1 << 30,
                          None, ctypes.byref(out)) == B.LBM_E_INVALID
    # too-small workspace
    assert B.lib.lbm_init(ctypes.byref(cfg), ctypes.c_void_p(256), ctypes.c_void_p(512), 16,
                          None, ctypes.byref(out)) == B.LBM_E_NOMEM


def test_product_path_has_no_cpu_fallback():
    """The binding refuses to run without the HIP library and the package never
    imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2608_19617_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            text = open(os.path.join(pkg, fn)).read()
            assert "oracle" not in re.sub(r'""".*?"""', "", text, flags=re.S), fn
    src = open(os.path.join(pkg, "binding.py")).read()
    assert "raise ImportError" in src


def test_design_entry_points_validate_before_any_hip_call(B):
    """lbm_design_* reject bad sizes, radii, NULL pointers and small
    workspaces with LBM_E_INVALID before touching the GPU."""
    n = ctypes.c_size_t(0)
    assert B.lib.lbm_design_workspace_bytes(0, 8, 1, 4.0, ctypes.byref(n)) == B.LBM_E_INVALID
    assert B.lib.lbm_design_workspace_bytes(16, 8, 1, 0.5, ctypes.byref(n)) == B.LBM_E_INVALID
    assert B.lib.lbm_design_workspace_bytes(16, 8, 1, 5.5, ctypes.byref(n)) == B.LBM_E_INVALID
    assert B.lib.lbm_design_workspace_bytes(16, 8, 1, 4.0, None) == B.LBM_E_INVALID
    assert B.lib.lbm_design_workspace_bytes(16, 8, 1, 4.0, ctypes.byref(n)) == B.LBM_OK
    small, big = n.value, ctypes.c_size_t(0)
    assert B.lib.lbm_design_workspace_bytes(64, 32, 16, 4.0, ctypes.byref(big)) == B.LBM_OK
    # fields (mask, base, normalisation, filtered, two scratch) grow with the grid
    assert big.value - small >= 64 * 32 * 16 * 41 - 16 * 8 * 41
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(256)
    assert B.lib.lbm_design_init(16, 8, 1, 4.0, None, fake, fake, small, None, ctypes.byref(out)) == B.LBM_E_INVALID
    assert B.lib.lbm_design_init(16, 8, 1, 4.0, fake, fake, ctypes.c_void_p(257), small, None,
                                 ctypes.byref(out)) == B.LBM_E_INVALID
    assert B.lib.lbm_design_init(16, 8, 1, 4.0, fake, fake, fake, small - 1, None,
                                 ctypes.byref(out)) == B.LBM_E_INVALID
    assert "workspace" in B.lib.lbm_last_error().decode()
    assert B.lib.lbm_design_map(None, fake, 2.0, 0.5, fake, None) == B.LBM_E_INVALID


def test_grid_limits_rejected(B):
    """Degenerate and maximum sizes: fewer than 3 nodes per axis, nz != 1 in
    2D, nz < 3 in 3D, and Q * nodes at 2^31 or beyond are rejected; the
    largest 2D grid below the limit is accepted."""
    for over in ({"nx": 2}, {"ny": 2}, {"nz": 2}):
        cfg, keep = _cfg(B)
        for k, v in over.items():
            setattr(cfg, k, v)
        assert _bytes(B, cfg)[0] == B.LBM_E_INVALID, over
    cfg, keep = _cfg(B)
    cfg.lattice, cfg.nz = B.LBM_D3Q19, 2
    assert _bytes(B, cfg)[0] == B.LBM_E_INVALID
    cfg, keep = _cfg(B)
    cfg.nx = (2 ** 31) // (9 * cfg.ny) + 1        # 9 nx ny >= 2^31
    assert _bytes(B, cfg)[0] == B.LBM_E_INVALID
    cfg.nx = (2 ** 31 - 1) // (9 * cfg.ny)        # just below
    assert _bytes(B, cfg)[0] == B.LBM_OK


def test_objective_configs(B):
    """The paper's objectives: unknown kinds, the wake as a monitor, boxes
    outside the grid or empty, and the C_d monitor without drag_ref are
    rejected; the drag and wake objectives add their window-field
    accumulators (three fields and the reference over the box) to the
    workspace."""
    for obj, mon in ((4, 0), (-1, 0), (0, B.LBM_J_WAKE), (0, 5)):
        cfg, keep = _cfg(B)
        cfg.objective, cfg.monitor = obj, mon
        assert _bytes(B, cfg)[0] == B.LBM_E_INVALID, (obj, mon)
    for box in ((0, 41, 0, 16, 0, 1), (5, 10, 7, 7, 0, 1), (-1, 5, 0, 5, 0, 1), (5, 10, 0, 17, 0, 1)):
        for name in ("force_box", "meas_box"):
            cfg, keep = _cfg(B)
            getattr(cfg, name)[:] = box
            assert _bytes(B, cfg)[0] == B.LBM_E_INVALID, (name, box)
    cfg, keep = _cfg(B)
    cfg.monitor, cfg.drag_ref = B.LBM_J_DRAG, 0.0
    assert _bytes(B, cfg)[0] == B.LBM_E_INVALID
    cfg.drag_ref = 0.5
    assert _bytes(B, cfg)[0] == B.LBM_OK
    cfg, keep = _cfg(B)
    st, base = _bytes(B, cfg)
    cfg.objective = B.LBM_J_DRAG
    cfg.force_box[:] = (5, 15, 2, 12, 0, 1)              # 100 nodes, one component
    st, drag = _bytes(B, cfg)
    assert st == B.LBM_OK and 4 * 100 * 8 + 1024 * 8 <= drag - base <= 4 * (100 * 8 + 256) + 1024 * 8 + 256
    cfg.objective = B.LBM_J_WAKE
    cfg.meas_box[:] = (20, 26, 5, 11, 0, 1)              # 36 nodes, two components
    st, wake = _bytes(B, cfg)
    assert st == B.LBM_OK and 4 * 72 * 8 + 1024 * 8 <= wake - base <= 4 * (72 * 8 + 256) + 1024 * 8 + 256


def test_design_map_noalloc_validates_before_any_hip_call(B):
    """The allocation-free map rejects NULL inputs, bad parameters and grids
    beyond its fixed scratch (more than 65536 tiles) before touching the
    GPU, so these calls run without one."""
    import ctypes
    P = ctypes.c_void_p
    ok = P(256)
    f = B.lib.lbm_design_map_noalloc
    assert f(64, 64, 1, 4.0, None, ok, ok, 2.0, 0.5, ok, ok, None) == B.LBM_E_INVALID
    assert f(64, 64, 1, 4.0, ok, ok, ok, 2.0, 0.5, None, ok, None) == B.LBM_E_INVALID
    assert f(64, 64, 1, 6.0, ok, ok, ok, 2.0, 0.5, ok, ok, None) == B.LBM_E_INVALID
    assert f(64, 64, 1, 4.0, ok, ok, ok, 0.0, 0.5, ok, ok, None) == B.LBM_E_INVALID
    assert f(64, 64, 1, 4.0, ok, ok, ok, 2.0, 1.0, ok, ok, None) == B.LBM_E_INVALID
    # 8224 x 2048 in 2D is 257 x 256 tiles of 32 x 8
    assert f(8224, 2048, 1, 4.0, ok, ok, ok, 2.0, 0.5, ok, ok, None) == B.LBM_E_INVALID
    assert b"65536 tiles" in B.lib.lbm_last_error()
    # 3D tiles are 8 x 8 x 4
    assert f(520, 512, 64, 4.0, ok, ok, ok, 2.0, 0.5, ok, ok, None) == B.LBM_E_INVALID   # 65 x 64 x 16 tiles
