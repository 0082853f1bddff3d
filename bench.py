"""Benchmark of the windowed LBM-LES forward + discrete-adjoint hot path.

Default workload (the largest single-GPU configuration): the D3Q19 cylinder
channel 384 x 128 x 128 (6.29M nodes; cylinder of radius 16 along z at
(96, 64); parabolic inlet u_max = 0.05 between walls in y, pressure outlet,
periodic z; Re = 1000 on the diameter, regularized BGK with Smagorinsky
C_s = 0.1), FP32 population storage. One benchmark step = set the design
field (reset to t = 0) -> 20 000 forward steps in 4 windows of 5000 steps
(samples every 20 steps, the consecutive-window test evaluated at every
window end, checkpoints every 250 steps in HBM) -> the discrete adjoint over
the last window (recompute of each 250-step segment from its checkpoint,
adjoint steps) -> dJ/dgamma. The inputs are resident in HBM before the timed
region. value = lattice updates per second over the timed steps, counting
every forward step and every adjoint step of each node once (recompute steps
are not counted as updates).

Besides the timed FP32 steps the line carries the kernel rates of the step,
the roofline of its dominant kernel, one FP64 and one FP16S step (speed and
the J / dJ/dgamma errors against FP64, from rest and from a shared window
start) and the CPU oracle on a slab of the same workload.

Prints one JSON line. Single GPU only. --suite selects other measurements.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS fwd & adjoint step, % HBM peak; FP32/FP16 vs FP64 at stated dJ/dγ error"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per lattice update of the forward step: read and write
# of the Q populations in storage precision plus the bounce-back fraction
# plane in compute precision (boundary kinds come from coordinates).
FWD_BYTES = {"f64": 9 * 8 * 2 + 8, "f32": 9 * 4 * 2 + 4, "f16s": 9 * 2 * 2 + 4}
# Adjoint step (D2Q9): adjoint populations read + write (FP64 in FP64 mode,
# else FP32), the pre-state's moment record read (6 values of the compute
# type), s, FP64 sensitivity read-modify-write.
ADJ_BYTES = {"f64": 9 * 8 * 2 + 6 * 8 + 8 + 16, "f32": 9 * 4 * 2 + 6 * 4 + 4 + 16,
             "f16s": 9 * 4 * 2 + 6 * 4 + 4 + 16}
# Recompute step (D2Q9): a forward step that also writes the moment record.
REC_BYTES = {p: FWD_BYTES[p] + 6 * (8 if p == "f64" else 4) for p in FWD_BYTES}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="f32", choices=["f64", "f32", "f16s"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 / FP16S comparison")
    ap.add_argument("--max-windows", type=int, default=20)
    ap.add_argument("--case", default="", help="paper suite: run only the workloads whose name contains this")
    ap.add_argument("--counters", action="store_true",
                    help="run one window and its adjoint of the workload plus a 256 MiB device copy "
                         "(for rocprofv3 --pmc byte counters) and exit")
    ap.add_argument("--counters-case", choices=["bfs", "cyl3d", "wake8192"], default="bfs",
                    help="workload of --counters: the backward-facing step (bfs), the D3Q19 "
                         "channel 384x128x128 (cyl3d) or the cylinder wake 8192x2048 (wake8192) in their "
                         "default launches: 40 forward steps and the adjoint of their last 20-step window")
    ap.add_argument("--suite", choices=["bfs", "hbm", "design", "fulltime", "paper", "optimize", "conditioning",
                                        "wake2048", "ubend1024"],
                    default=None,
                    help="bfs: the backward-facing step 800x200 (FP32 vs FP64 window criterion "
                         "workload) benchmarked to its converged window and adjoint; hbm: rooflines of the forward, recompute and adjoint kernels on grids far "
                         "larger than the caches (one JSON line per configuration) instead of the "
                         "benchmark step; design: timings of the design update (filter + projection, "
                         "chain rule, volume-constrained step); fulltime: one optimisation iteration "
                         "with the window adjoint against the full-time adjoint (time and storage); "
                         "paper: the paper's cylinder-drag and wake-recovery examples at their sizes "
                         "with their objectives and the finite-difference check of the adjoint; "
                         "optimize: the paper's cylinder drag minimisation (Re 51.2) for up to 60 "
                         "iterations of forward windows, adjoint and design update; conditioning: "
                         "precision errors and finite differences against window length; wake2048: the "
                         "cylinder wake 2048x512 with 20000-step windows through the autograd entry "
                         "point; ubend1024: the U-bend 1024x1024, FP16S against FP32 over 10000 steps")
    return ap.parse_args()


def counters_run(args, torch):
    """Workload for hardware-counter runs: one window forward and its adjoint
    of the benchmark workload (or 40 forward steps of the D3Q19 channel),
    then a plain 256 MiB device-to-device copy whose byte counters calibrate
    FETCH_SIZE / WRITE_SIZE."""
    from paper_2608_19617_amd import workloads as W
    from paper_2608_19617_amd.solver import Solver
    if args.counters_case in ("cyl3d", "wake8192"):
        if args.counters_case == "cyl3d":
            w = W.cylinder_3d(window_len=20, sample_every=20, ckpt_every=20, n_windows=2)
        else:
            w = W.cylinder_wake(nx=8192, ny=2048, radius=128, window_len=20, sample_every=20, ckpt_every=20,
                                max_windows=2)
        sv = Solver(w, args.prec)
        sv.forward(2 * w.window_len)
        sv.adjoint()
    else:
        w = W.backward_facing_step(max_windows=args.max_windows)
        sv = Solver(w, args.prec)
        sv.forward(w.window_len)
        sv.adjoint()
    sv.close()
    a = torch.ones(256 * 2 ** 20 // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"counters_run": True, "copy_bytes": a.numel() * 4}), flush=True)


def kernel_source_digest():
    """SHA-256 of the kernel sources: counter figures in profiles/ apply only
    to the kernels they were measured on."""
    import hashlib
    h = hashlib.sha256()
    for fn in ("kernels.hip", "device.hpp", "lattice.hpp"):
        with open(os.path.join(ROOT, "paper_2608_19617_amd", "csrc", fn), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_values(stem):
    """key = value lines of profiles/<stem>.txt, or {} when the file is absent
    or the kernel sources changed since its figures were taken (the file
    records their SHA-256)."""
    path = os.path.join(ROOT, "profiles", stem + ".txt")
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_digest():
        return {}
    return vals


def measured_traffic(kernel, prec):
    """HBM bytes per launch of `kernel` on the backward-facing step from the
    committed counter summary (None when absent or stale)."""
    v = profile_values(f"{kernel}_bfs800x200_{prec}_counters").get("hbm_bytes_per_launch")
    return None if v is None else float(v)


def bench_step(sv, w, max_windows):
    rep = sv.forward(max_windows * w.window_len, stop_on_converge=True)
    g, J = sv.adjoint()
    return rep, g, J


def run_timed(sv, w, args, torch):
    gamma = w.gamma
    for _ in range(args.warmup):
        sv.set_gamma(gamma)
        bench_step(sv, w, args.max_windows)
    torch.cuda.synchronize()
    sv.timing(True)
    total_fwd = total_adj = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sv.set_gamma(gamma)
        rep, g, J = bench_step(sv, w, args.max_windows)
        total_fwd += rep["steps_done"]
        total_adj += w.window_len
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = sv.timing(False)
    return dict(rep=rep, g=g, J=J, dt=dt, fwd=total_fwd, adj=total_adj, tm=tm)


def cpu_baseline(w, fwd_per_step, adj_per_step):
    """The oracle as it stands, on this host, on a bounded sample of the same
    workload: 100 forward steps from t = 0 and a 6-step window adjoint."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import oracle_problem
    from oracle import adjoint as ad
    from oracle import forward as fw

    n_f, n_a = 100, 6
    with threadpool_limits(limits=1):
        prob = oracle_problem(w)
        s = fw.design_map(prob, w.gamma)
        f = fw.initial_state(prob)
        t0 = time.perf_counter()
        for _ in range(n_f):
            f = fw.step(prob, f, s)
        t_f = (time.perf_counter() - t0) / n_f
        prob_a = oracle_problem(w, window_len=n_a, sample_every=1)
        t0 = time.perf_counter()
        ad.window_gradient(prob_a, w.gamma, f)
        t_wa = time.perf_counter() - t0
        t_a = max(t_wa / n_a - t_f, 1e-9)      # the window gradient replays the forward too
    N = w.nodes
    secs = fwd_per_step * t_f + adj_per_step * t_a
    value = N * (fwd_per_step + adj_per_step) / secs / 1e6
    return {"value": round(value, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": (f"{n_f} forward steps and a {n_a}-step window adjoint of the same "
                       f"{w.shape[0]}x{w.shape[1]} workload (FP64 numpy, 1 thread); per-step "
                       f"times {t_f*1e3:.1f} ms forward, {t_a*1e3:.1f} ms adjoint, weighted by "
                       f"the GPU step's mix of {fwd_per_step} forward + {adj_per_step} adjoint steps"),
            "fwd_mlups": round(N / t_f / 1e6, 4), "adj_mlups": round(N / t_a / 1e6, 4)}


def precision_compare(w, ref_prec, res_ref, args, torch, Solver):
    """FP64 and FP16S beside the benchmarked precision: time one benchmark
    step of each; the error of J and dJ/dgamma from rest (each precision on
    its own trajectory from t = 0, on its own W_eff) and of the same window
    computed from the FP64 window-start state. On this workload the window
    means of the pressure drop swing about zero from window to window (an
    acoustic oscillation of the mean density), so besides the error relative
    to the window's own J the absolute error is given relative to the RMS of
    the FP64 window means over the run."""
    import numpy as np
    out = {}
    sv64 = Solver(w, "f64")
    sv64.set_gamma(w.gamma)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep64, g64, J64 = bench_step(sv64, w, args.max_windows)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    g64r = g64.cpu().numpy()          # from rest, FP64's own W_eff
    n_upd64 = rep64["steps_done"] + w.window_len
    Jhist, _, _ = sv64.history()
    j_rms = float(np.sqrt(np.mean(np.square(Jhist))))    # scale of the window means over the run
    out["f64"] = {"mlups": round(w.nodes * n_upd64 / t64 / 1e6, 1), "w_eff": rep64["w_eff"],
                  "J": J64, "window_J_rms": j_rms}
    # shared window-start state: FP64 state entering W_eff
    w_eff = rep64["w_eff"]
    sv64.set_gamma(w.gamma)
    start = (w_eff - 1) * w.window_len
    if start > 0:
        sv64.forward(start)
    f_start, step = sv64.get_state()
    sv64.forward(w.window_len)
    g64w, J64w = sv64.adjoint()
    g64w = g64w.cpu().numpy()
    sv64.close()
    for prec in ("f32", "f16s"):
        sv = Solver(w, prec)
        sv.set_gamma(w.gamma)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep, g, J = bench_step(sv, w, args.max_windows)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        gr = g.cpu().numpy()
        n_upd = rep["steps_done"] + w.window_len
        mlups = w.nodes * n_upd / tp / 1e6
        sv.set_state(f_start, step)
        sv.forward(w.window_len)
        gw, Jw = sv.adjoint()
        gw = gw.cpu().numpy()
        out[prec] = {"mlups": round(mlups, 1), "w_eff": rep["w_eff"],
                     "speedup_vs_f64": round(mlups / out["f64"]["mlups"], 3),
                     "J_rel_err_vs_f64_same_start": float(abs(Jw - J64w) / abs(J64w)),
                     "J_abs_err_vs_f64_same_start": float(abs(Jw - J64w)),
                     "J_err_over_window_J_rms": float(abs(Jw - J64w) / j_rms),
                     "dJdgamma_rel_l2_vs_f64_same_start":
                         float(np.linalg.norm(gw - g64w) / np.linalg.norm(g64w)),
                     "J_rel_err_vs_f64_from_rest": float(abs(J - J64) / abs(J64)),
                     "dJdgamma_rel_l2_vs_f64_from_rest":
                         float(np.linalg.norm(gr - g64r) / np.linalg.norm(g64r))}
        sv.close()
    return out


# Algorithmic bytes per update on D3Q19: the forward reads and writes the 19
# populations and reads s; the adjoint reads and writes the 19 adjoint
# populations, reads the moment record (10 values of the compute type) of its
# pre-state and s, and read-modify-writes the FP64 sensitivity; the recompute
# is a forward step that also writes the record.
FWD_BYTES_3D = {"f32": 19 * 4 * 2 + 4, "f64": 19 * 8 * 2 + 8, "f16s": 19 * 2 * 2 + 4}
ADJ_BYTES_3D = {"f32": 19 * 4 * 2 + 10 * 4 + 4 + 16, "f64": 19 * 8 * 2 + 10 * 8 + 8 + 16,
                "f16s": 19 * 4 * 2 + 10 * 4 + 4 + 16}
REC_BYTES_3D = {p: FWD_BYTES_3D[p] + 10 * (8 if p == "f64" else 4) for p in FWD_BYTES_3D}


def hbm_suite(args, torch):
    """Kernel rooflines where the state does not fit in any cache: the
    cylinder wake scaled 4x per axis (8192 x 2048, 16.8M nodes, disk R = 128,
    same Re and inlet speed) in every precision, and the 3D cylinder channel
    384 x 128 x 128 (6.3M nodes, D3Q19, FP32). Each configuration runs a
    spin-up window, a timed window of forward steps, then the adjoint of that
    window (recompute + adjoint steps), all timed per kernel class with HIP
    events; one JSON line per configuration."""
    from paper_2608_19617_amd import workloads as W
    from paper_2608_19617_amd.solver import Solver
    # reference ceiling: a plain device-to-device copy of 2 GiB
    a = torch.ones(2 ** 29, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    copy_gbs = 2 * a.numel() * 4 * 10 / (time.perf_counter() - t0) / 1e9
    print(json.dumps({"suite": "hbm", "device_copy_2GiB_GBs": round(copy_gbs, 1),
                      "frac_of_hbm_peak": round(copy_gbs / HBM_PEAK_GBS, 4)}), flush=True)
    del a, b
    cases = []
    for prec in ("f64", "f32", "f16s"):
        w = W.cylinder_wake(nx=8192, ny=2048, radius=128, window_len=500, sample_every=20, ckpt_every=50,
                            max_windows=2)
        cases.append(("cylinder wake 8192x2048 (the 2048x512 wake x4 per axis)", w, prec, FWD_BYTES[prec], ADJ_BYTES[prec],
                      REC_BYTES[prec]))
    for prec in ("f32", "f16s", "f64"):
        w3 = W.cylinder_3d(window_len=100, sample_every=20, ckpt_every=20, n_windows=2)
        cases.append(("cylinder 3D 384x128x128 D3Q19", w3, prec, FWD_BYTES_3D[prec], ADJ_BYTES_3D[prec],
                      REC_BYTES_3D[prec]))
    for name, w, prec, fb, ab, rb in cases:
        sv = Solver(w, prec)
        sv.set_gamma(w.gamma)
        sv.forward(w.window_len)                  # spin-up window
        torch.cuda.synchronize()
        sv.timing(True)
        sv.forward(w.window_len)
        torch.cuda.synchronize()
        tf = sv.timing(True)
        t0 = time.perf_counter()
        sv.adjoint()
        torch.cuda.synchronize()
        t_sweep = time.perf_counter() - t0
        ta = sv.timing(False)
        N = w.nodes
        fwd_ms = tf["fwd_ms"] + tf["tb_ms"]
        fwd_steps = tf["fwd_launches"] + tf["tb_steps"]
        fwd_s = fwd_ms * 1e-3 / fwd_steps
        adj_s = ta["adj_ms"] * 1e-3 / ta["adj_steps"]
        rec_s = ta["rec_ms"] * 1e-3 / max(ta["rec_steps"], 1)
        line = {"suite": "hbm", "workload": name, "grid": list(w.shape), "nodes": N, "dtype": prec,
                "forward": {"steps": int(fwd_steps), "us_per_step": round(fwd_s * 1e6, 3),
                            "steps_per_launch": round(fwd_steps / max(tf["fwd_launches"] + tf["tb_launches"], 1), 2),
                            "mlups": round(N / fwd_s / 1e6, 1), "bytes_per_lup": fb,
                            "achieved_GBs": round(fb * N / fwd_s / 1e9, 1),
                            "frac_of_hbm_peak": round(fb * N / fwd_s / 1e9 / HBM_PEAK_GBS, 4)},
                "adjoint": {"steps": int(ta["adj_steps"]), "us_per_step": round(adj_s * 1e6, 3),
                            "steps_per_launch": round(ta["adj_steps"] / max(ta["adj_launches"], 1), 2),
                            "mlups": round(N / adj_s / 1e6, 1), "bytes_per_lup": ab,
                            "achieved_GBs": round(ab * N / adj_s / 1e9, 1),
                            "frac_of_hbm_peak": round(ab * N / adj_s / 1e9 / HBM_PEAK_GBS, 4)},
                "recompute": {"steps": int(ta["rec_steps"]), "us_per_step": round(rec_s * 1e6, 3),
                              "bytes_per_lup": rb,
                              "frac_of_hbm_peak": round(rb * N / rec_s / 1e9 / HBM_PEAK_GBS, 4)},
                "reverse_sweep": {"s": round(t_sweep, 4),
                                  "mlups_per_window_lup": round(N * w.window_len / t_sweep / 1e6, 1)}}
        sv.close()
        print(json.dumps(line), flush=True)


def design_suite(args, torch):
    """Design update (lbm_design.h) on the cylinder-wake grid 2048 x 512 and
    the D3Q19 channel 384 x 128 x 128, every node a design node, filter
    radius 4: per-call times of the map (filter + projection + volume), the
    chain rule and one volume-constrained step (which maps the design about
    70 times while it bisects the multiplier), timed with CUDA events on the
    current stream. The stencil reads each of its n_off neighbours from LDS:
    2 n_off flop and n_off 8-byte LDS reads per node (n_off = 45 in 2D, 257 in
    3D); its HBM bytes per node are x, W, base, mask read and x~, gamma
    written (41 B; the chain rule: x~, g, W, mask read, dJ/dx, dV/dx written,
    41 B)."""
    import numpy as np
    from paper_2608_19617_amd.design import Design
    for shape in ((2048, 512), (384, 128, 128)):
        N = int(np.prod(shape))
        rng = np.random.default_rng(0)
        mask = np.ones(shape, dtype=bool)
        x = torch.as_tensor(rng.random(shape), device="cuda")
        g = torch.as_tensor(rng.standard_normal(shape), device="cuda")
        d = Design(shape, mask, np.zeros(shape), radius=4.0)
        n_off = 45 if len(shape) == 2 else 257

        def timed(fn, reps):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) * 1e-3 / reps

        t_map = timed(lambda: d.map(x, 8.0, 0.5), 20)
        t_chain = timed(lambda: d.chain(x, 8.0, 0.5, g), 20)
        gJ, gV = d.chain(x, 8.0, 0.5, g)
        _, v0 = d.map(x, 8.0, 0.5)
        t_upd = timed(lambda: d.update(x, -gV, gV, 8.0, 0.5, 0.2, v0 - 0.05), 3)
        line = {"suite": "design", "grid": list(shape), "nodes": N, "dtype": "f64", "radius": 4.0,
                "neighbours": n_off,
                "map": {"us": round(t_map * 1e6, 1), "mlups": round(N / t_map / 1e6, 1),
                        "hbm_GBs": round(41 * N / t_map / 1e9, 1),
                        "fp64_TFLOPs": round(2 * n_off * N / t_map / 1e12, 2),
                        "lds_TBs": round(8 * n_off * N / t_map / 1e12, 1)},
                "chain": {"us": round(t_chain * 1e6, 1), "mlups": round(N / t_chain / 1e6, 1),
                          "fp64_TFLOPs": round(4 * n_off * N / t_chain / 1e12, 2)},
                "update_ms": round(t_upd * 1e3, 2)}
        d.close()
        print(json.dumps(line), flush=True)


def fulltime_suite(args, torch):
    """The comparison of Sec. "Comparison with full-time adjoint
    optimization" at MI355X scale: the cylinder wake 2048 x 512 (disk D = 64)
    run for 4 windows of 5000 steps (dW = 50, K = 250), then dJ/dgamma of the
    last window with the window-restricted adjoint and with the full-time
    adjoint (the sweep chained back to t = 0; earlier windows replayed once
    from their start states), at the paper's Re = 51.2 of that comparison and
    in the LES regime (Re = 1000). Reports the time of each part, the
    workspace of both methods, the bytes of the stored trajectory that the
    full-time method needs without replays (every state of the run, as in the
    paper), and the norms and cosine of the two gradients."""
    import numpy as np
    from paper_2608_19617_amd import workloads as W
    from paper_2608_19617_amd.solver import Solver
    for re in (51.2, 1000.0):
        w = W.cylinder_wake(nx=2048, ny=512, radius=32, re=re, window_len=5000, sample_every=50,
                            ckpt_every=250, max_windows=4, eps=-1.0)
        w.full_history = True
        n_win = 4
        sv = Solver(w, args.prec)
        sv.set_gamma(w.gamma)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sv.forward(n_win * w.window_len)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        t0 = time.perf_counter()
        g_w, J = sv.adjoint()
        torch.cuda.synchronize()
        t_win = time.perf_counter() - t0
        t0 = time.perf_counter()
        g_f, _ = sv.adjoint_full()
        torch.cuda.synchronize()
        t_full = time.perf_counter() - t0
        gw, gf = g_w.cpu().numpy().ravel(), g_f.cpu().numpy().ravel()
        ws_full = sv.workspace_bytes
        sv.close()
        w.full_history = False
        sv = Solver(w, args.prec)
        ws_win = sv.workspace_bytes
        sv.close()
        state_bytes = 9 * w.nodes * {"f64": 8, "f32": 4, "f16s": 2}[args.prec]
        nw, nf = float(np.linalg.norm(gw)), float(np.linalg.norm(gf))
        line = {"suite": "fulltime", "workload": f"cylinder wake 2048x512 Re {re}, 4 windows of 5000 steps",
                "dtype": args.prec, "steps": n_win * w.window_len, "J": J,
                "forward_s": round(t_fwd, 3), "window_adjoint_s": round(t_win, 3),
                "full_time_adjoint_s": round(t_full, 3),
                "iteration_s": {"window": round(t_fwd + t_win, 3), "full_time": round(t_fwd + t_full, 3)},
                "workspace_GB": {"window": round(ws_win / 1e9, 3),
                                 "full_time_two_level": round(ws_full / 1e9, 3),
                                 "full_trajectory": round(n_win * w.window_len * state_bytes / 1e9, 1)},
                "gradient_norm": {"window": nw, "full_time": nf},
                "gradient_cosine": float(gw @ gf / (nw * nf)) if nw > 0 and nf > 0 else None}
        print(json.dumps(line), flush=True)


def _timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def _fd_check(torch, sv, gamma, g_adj, points, J, steps=(1e-3, 1e-4)):
    """Forward-difference sensitivities of the representative window (each
    perturbed design replayed from the window's start state) at the given
    nodes, for each perturbation in `steps`, against the adjoint."""
    import numpy as np
    out = {}
    adj = np.array([g_adj[p] for p in points])
    for h in steps:
        fd = []
        t0 = time.perf_counter()
        for p in points:
            gp = gamma.copy()
            hs = h if gp[p] + h <= 1.0 else -h      # stay inside [0, 1]
            gp[p] += hs
            fd.append((sv.replay(gp) - J) / hs)
        torch.cuda.synchronize()
        fd = np.array(fd)
        top = float(np.max(np.abs(fd)))
        out[f"h={h:g}"] = {"max_err_over_max_fd": float(np.max(np.abs(adj - fd)) / top) if top > 0 else None,
                           "rel_l2": float(np.linalg.norm(adj - fd) / np.linalg.norm(fd)) if top > 0 else None,
                           "replay_s": round(time.perf_counter() - t0, 3)}
    return out


def paper_suite(args, torch):
    """The paper's own examples at their sizes and with their objectives:
    the flow around a cylinder (200 x 100, radius 8, Re 3.2 / 12.8 / 51.2;
    drag objective over the domain, C_d monitor, |W| = 5000, dW = 50,
    eps = 1e-3, at most 20 windows) with the 60-point finite-difference check
    of the adjoint (gamma + 1e-3 and + 1e-4 at the 60 nodes downstream of the
    cylinder centre on its axis, the representative window replayed for
    each), and the wake-flow recovery (200 x 50; Re 60 with d = 10 and Re 72
    with d = 12): a reference run with the cylinder gives u_ref on M, then
    the wake objective from the constant initial design, with a 20-point
    check inside the design domain; and the U-bend (240 x 192 at Re 400,
    300 x 240 at Re 750; pressure-drop objective, |W| = 20000, dW = 20,
    eps = 0.05) with a 20-point check on design nodes next to the channel.
    Perturbations that would leave [0, 1] are taken downward. FP64 for the checks (skipped with
    --no-compare); the forward run and the adjoint are also timed in the
    requested precision."""
    import numpy as np
    from paper_2608_19617_amd import workloads as W
    from paper_2608_19617_amd.solver import Solver
    cases = [("cylinder_drag", re, W.cylinder_drag(re)) for re in (3.2, 12.8, 51.2)]
    for re, d, lmeas in ((60.0, 10, 33), (72.0, 12, 39)):
        cases.append(("wake_recovery", re, W.wake_recovery(re, d, lmeas)))
    for re in (400.0, 750.0):
        cases.append(("u_bend", re, W.u_bend_paper(re)))
    for kind, re, w in cases:
        if args.case not in w.name:
            continue
        u_ref, ref_line = None, None
        if kind == "wake_recovery":
            wr = W.wake_recovery(re, w.notes["d"], w.notes["l_measure"], reference=True)
            sv = Solver(wr, "f64")
            rep, t = _timed(torch, lambda: sv.forward(wr.n_steps, stop_on_converge=True))
            u_ref = sv.wake_mean_velocity()
            ref_line = {"windows": rep["windows_done"], "converged": rep["converged"], "monitor_mean": rep["monitor"],
                        "forward_s": round(t, 3)}
            sv.close()
        line = {"suite": "paper", "workload": w.name, "grid": list(w.shape), "re": re, "tau": w.tau,
                "objective": w.objective, "window_len": w.window_len, "sample_every": w.sample_every,
                "eps": w.eps}
        if ref_line:
            line["reference_run"] = ref_line
        for prec in ("f64", args.prec) if args.prec != "f64" else ("f64",):
            sv = Solver(w, prec)
            if u_ref is not None:
                sv.set_wake_reference(u_ref)
            rep, t_fwd = _timed(torch, lambda: sv.forward(w.n_steps, stop_on_converge=True))
            (g, J), t_adj = _timed(torch, lambda: sv.adjoint())
            steps = rep["steps_done"]
            res = {"windows": rep["windows_done"], "converged": rep["converged"], "monitor_mean": rep["monitor"],
                   "J": J, "forward_s": round(t_fwd, 4),
                   "forward_MLUPS": round(steps * w.nodes / t_fwd / 1e6, 1),
                   "adjoint_s": round(t_adj, 4),
                   "adjoint_MLUPS": round(w.window_len * w.nodes / t_adj / 1e6, 1)}
            if prec == "f64" and not args.no_compare:
                gh = g.cpu().numpy()
                if kind == "cylinder_drag":
                    cx, cy = w.notes["center"]
                    pts = [(cx + 1 + k, cy) for k in range(60)]
                elif kind == "u_bend":
                    # design nodes within 3 nodes of the channel (where the sensitivity lives)
                    from scipy.ndimage import binary_dilation
                    near = binary_dilation(w.gamma == 0.0, iterations=3) & w.notes["design_mask"]
                    cand = np.argwhere(near)
                    pick = np.random.default_rng(0).choice(len(cand), 20, replace=False)
                    pts = [tuple(int(v) for v in cand[i]) for i in pick]
                else:
                    (x0, x1), (y0, y1) = w.force_box
                    rng = np.random.default_rng(0)
                    pts = [(int(x), int(y)) for x, y in zip(rng.integers(x0, x1, 20), rng.integers(y0, y1, 20))]
                # the U-bend's long unsteady window responds linearly only to
                # small perturbations: a ladder of steps down to 1e-6
                steps = (1e-4, 1e-5, 1e-6) if kind == "u_bend" else (1e-3, 1e-4)
                res["fd_check"] = dict(points=len(pts), **_fd_check(torch, sv, w.gamma, gh, pts, J, steps))
            line[prec] = res
            sv.close()
        print(json.dumps(line), flush=True)


def optimize_suite(args, torch):
    """The optimisation loop on the paper's cylinder example (Re 51.2,
    200 x 100, |W| = 5000, dW = 50, eps = 1e-3): minimise the drag under
    0.014 <= V <= 0.016 over the design domain 10 <= x < 190, 5 <= y < 95
    (the initial design x = 0.5 inside the cylinder of radius 8, 0
    elsewhere; filter radius 4, beta from 2 doubling every 10 iterations to
    16, move limit 0.2, eps_o = 0.005, at most 60 iterations). Each iteration
    runs the forward windows from t = 0 to the criterion, the adjoint over
    the representative window and the volume-constrained design update, all
    on the GPU. Reports the time per iteration and the objective and volume
    history; then the paper's comparison with prescribed windows.""" 
    import numpy as np
    from paper_2608_19617_amd import workloads as W
    from paper_2608_19617_amd.optimize import optimize
    w = W.cylinder_drag(51.2)
    cx, cy = w.notes["center"]
    mask = np.zeros(w.shape, dtype=bool)
    mask[10:190, 5:95] = True
    X, Y = np.meshgrid(np.arange(w.shape[0]), np.arange(w.shape[1]), indexing="ij")
    x0 = np.where(np.hypot(X - cx, Y - cy) <= w.notes["radius"], 0.5, 0.0)
    base = np.zeros(w.shape)
    for prec in ("f32", "f64") if args.prec != "f64" else ("f64",):
        times = []
        last = [time.perf_counter()]

        def tick(rec):
            torch.cuda.synchronize()
            now = time.perf_counter()
            times.append(now - last[0])
            last[0] = now

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last[0] = t0
        x, hist = optimize(w, mask, x0, prec=prec, radius=4.0, eta=0.5, beta=2.0, beta_max=16.0, beta_every=10,
                           move=0.2, vmin=0.014, vmax=0.016, n_max=60, eps_o=0.005, base=base, callback=tick)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        J = [h["J"] for h in hist]
        V = [h["V"] for h in hist]
        line = {"suite": "optimize", "workload": "cylinder drag 200x100 Re 51.2, 0.014 <= V <= 0.016",
                "dtype": prec, "iterations": len(hist), "total_s": round(total, 3),
                "s_per_iteration": round(total / max(len(hist), 1), 4),
                "median_iteration_s": round(float(np.median(times)), 4) if times else None,
                "J_first": J[0], "J_last": J[-1], "J_min": min(J), "V_first": V[0], "V_last": V[-1],
                "windows_last": hist[-1]["w_eff"], "J_history": [round(j, 6) for j in J],
                "V_history": [round(v, 5) for v in V]}
        print(json.dumps(line), flush=True)
    # Sec. "Comparison between representative and prescribed time windows":
    # the same optimisation with the window prescribed as t in [20000, 25000]
    # and t in [5000, 6000]; every final design re-evaluated with the
    # representative-window criterion
    from paper_2608_19617_amd.design import Design
    from paper_2608_19617_amd.solver import Solver
    runs = {}
    for name, wl, steps in (("representative", 5000, None), ("prescribed_20000_25000", 5000, 25000),
                            ("prescribed_5000_6000", 1000, 6000)):
        wp = W.cylinder_drag(51.2, window_len=wl, sample_every=50, ckpt_every=250 if wl == 5000 else 100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, hist = optimize(wp, mask, x0, prec=args.prec, radius=4.0, eta=0.5, beta=2.0, beta_max=16.0,
                           beta_every=10, move=0.2, vmin=0.014, vmax=0.016, n_max=60, eps_o=0.005, base=base,
                           steps=steps)
        torch.cuda.synchronize()
        dz = Design(w.shape, mask, base, 4.0)
        gamma, V = dz.map(x, hist[-1]["beta"], 0.5)
        dz.close()
        sv = Solver(w, args.prec)
        sv.set_gamma(gamma)
        rep = sv.forward(w.max_windows * w.window_len, stop_on_converge=True)
        sv.close()
        runs[name] = {"iterations": len(hist), "s": round(time.perf_counter() - t0, 3), "J_last": hist[-1]["J"],
                      "V": V, "J_reevaluated": rep["J_eff"], "reevaluation_windows": rep["windows_done"]}
    ref = runs["representative"]["J_reevaluated"]
    for r in runs.values():
        r["reevaluated_vs_representative"] = r["J_reevaluated"] / ref - 1.0
    print(json.dumps({"suite": "optimize", "comparison": "representative vs prescribed windows, Re 51.2",
                      "dtype": args.prec, "runs": runs}), flush=True)
    # the paper's other two examples: wake recovery (Re 60; u_ref from the
    # cylinder's converged mean flow; 0.1 <= V <= 0.9; eps_o = 5e-3, at most
    # 200 iterations) and the U-bend (Re 400; 0.52 <= V <= 0.65; eps_o = 1e-5,
    # at most 90 iterations)
    from paper_2608_19617_amd.solver import Solver as _S
    wr = W.wake_recovery(60.0, 10, 33, reference=True)
    sv = _S(wr, args.prec)
    sv.forward(wr.n_steps, stop_on_converge=True)
    u_ref = sv.wake_mean_velocity()
    sv.close()
    ww = W.wake_recovery(60.0, 10, 33)
    (bx0, bx1), (by0, by1) = ww.force_box
    wmask = np.zeros(ww.shape, dtype=bool)
    wmask[bx0:bx1, by0:by1] = True
    ub = W.u_bend_paper(400.0)
    for name, wk, m, xi, bs, vmn, vmx, eps_o, nmax, ur in (
            ("wake recovery 200x50 Re 60, 0.1 <= V <= 0.9", ww, wmask, np.where(wmask, 0.5, 0.0), np.zeros(ww.shape),
             0.1, 0.9, 5e-3, 200, u_ref),
            ("U-bend 240x192 Re 400, 0.52 <= V <= 0.65", ub, ub.notes["design_mask"], ub.gamma, ub.gamma,
             0.52, 0.65, 1e-5, 90, None)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, hist = optimize(wk, m, xi, prec=args.prec, radius=4.0, eta=0.5, beta=2.0, beta_max=16.0, beta_every=10,
                           move=0.2, vmin=vmn, vmax=vmx, n_max=nmax, eps_o=eps_o, base=bs, u_ref=ur)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        J = [h["J"] for h in hist]
        print(json.dumps({"suite": "optimize", "workload": name, "dtype": args.prec, "iterations": len(hist),
                          "total_s": round(total, 3), "s_per_iteration": round(total / len(hist), 4),
                          "J_first": J[0], "J_last": J[-1], "J_min": min(J), "V_first": hist[0]["V"],
                          "V_last": hist[-1]["V"], "J_history": [float("%.6g" % j) for j in J]}), flush=True)


def bfs_bench(args, torch):
    """The backward-facing step 800 x 200 (FP32 vs FP64 window-criterion
    workload): one step = set gamma -> forward windows of 2000 steps until the
    criterion passes (at most 20) -> adjoint over W_eff (K = 100); the line
    layout of the default benchmark, on this cache-resident grid."""
    from paper_2608_19617_amd import workloads as W
    from paper_2608_19617_amd.solver import Solver

    w = W.backward_facing_step(max_windows=args.max_windows)
    sv = Solver(w, args.prec)
    res = run_timed(sv, w, args, torch)
    N = w.nodes
    upd = N * (res["fwd"] + res["adj"])
    value = upd / res["dt"] / 1e6
    tm = res["tm"]
    # forward time per step over all forward launches (blocked and single)
    fwd_steps = tm["tb_steps"] + tm["fwd_launches"]
    fwd_step_s = (tm["tb_ms"] + tm["fwd_ms"]) * 1e-3 / fwd_steps
    adj_step_s = tm["adj_ms"] / tm["adj_steps"] * 1e-3
    # dominant kernel: the temporally blocked forward kernel when it is used
    if tm["tb_launches"] > 0 and tm["tb_ms"] >= tm["fwd_ms"]:
        kname = "k_step_tb (forward, temporally blocked)"
        kfile = "k_step_tb"
        steps_per_launch = tm["tb_steps"] / tm["tb_launches"]
        launch_s = tm["tb_ms"] / tm["tb_launches"] * 1e-3
    else:
        kname = "k_step (forward)"
        kfile = "k_step"
        steps_per_launch = 1.0
        launch_s = tm["fwd_ms"] / tm["fwd_launches"] * 1e-3
    bytes_per_launch = steps_per_launch * FWD_BYTES[args.prec] * N
    achieved = bytes_per_launch / launch_s / 1e9
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res["dt"] / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.prec, "data": "synthetic",
        "config": {"workload": "backward-facing step 800x200 D2Q9, Re 800, C_s 0.1, windows 2000 / "
                               "dW 100 / eps 1e-3 / max 20, adjoint over W_eff with K = 100",
                   "grid": list(w.shape), "window_len": w.window_len, "sample_every": w.sample_every,
                   "ckpt_every": w.ckpt_every, "tau": w.tau,
                   "fwd_steps_per_step": res["fwd"] // args.steps,
                   "adj_steps_per_step": res["adj"] // args.steps,
                   "w_eff": res["rep"]["w_eff"], "converged": res["rep"]["converged"]},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(kfile, args.prec), "bytes_per_lup": FWD_BYTES[args.prec],
                     "steps_per_launch": round(steps_per_launch, 3),
                     "avg_launch_us": round(launch_s * 1e6, 3)},
        "fwd_mlups": round(N / fwd_step_s / 1e6, 1),
        "adj_kernel_mlups": round(N / adj_step_s / 1e6, 1),
        "adj_kernel": {"avg_launch_us": round(tm["adj_ms"] / tm["adj_launches"] * 1e3, 3),
                       "steps_per_launch": round(tm["adj_steps"] / tm["adj_launches"], 3),
                       "us_per_step": round(adj_step_s * 1e6, 3), "bytes_per_lup": ADJ_BYTES[args.prec],
                       "achieved_GBs": round(ADJ_BYTES[args.prec] * N / adj_step_s / 1e9, 1)},
        "recompute": {"avg_launch_us": round(tm["rec_ms"] / max(tm["rec_launches"], 1) * 1e3, 3),
                      "us_per_step": round(tm["rec_ms"] / max(tm["rec_steps"], 1) * 1e3, 3),
                      "steps_per_launch": round(tm["rec_steps"] / max(tm["rec_launches"], 1), 3)},
        "J": res["J"],
    }
    sv.close()
    if not args.no_compare:
        line["precision"] = precision_compare(w, args.prec, res, args, torch, Solver)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, res["fwd"] // args.steps, res["adj"] // args.steps)
    print(json.dumps(line), flush=True)



# ------------------------------- default: the D3Q19 channel 384x128x128

C5_SLAB_NZ, C5_SLAB_FWD, C5_SLAB_WIN = 2, 4, 2


def channel3d_workload():
    """The D3Q19 cylinder channel 384 x 128 x 128: 4 windows of 5000 steps
    (dW = 20, K = 250), pressure-drop objective and monitor; the window test
    (eps = 1e-3) is evaluated at every window end, and the run is the fixed
    20 000 steps with the adjoint over the last window."""
    from paper_2608_19617_amd import workloads as W
    w = W.cylinder_3d()
    w.eps = 1e-3
    return w


def _device_gamma(w, torch):
    """The design field in the library's node order, resident on the GPU."""
    from paper_2608_19617_amd.solver import to_device_order
    return torch.from_numpy(to_device_order(w.gamma.astype("float64"))).to("cuda")


def _free(torch, *solvers):
    for sv in solvers:
        sv.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def channel3d_step(sv, w, gamma_dev):
    sv.set_gamma(gamma_dev)
    rep = sv.forward(w.max_windows * w.window_len)
    g, J = sv.adjoint()
    return rep, g, J


def channel3d_timed(w, gamma_dev, args, torch):
    from paper_2608_19617_amd.solver import Solver
    sv = Solver(w, args.prec)
    for _ in range(args.warmup):
        channel3d_step(sv, w, gamma_dev)
    torch.cuda.synchronize()
    sv.timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rep, g, J = channel3d_step(sv, w, gamma_dev)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = sv.timing(False)
    Jh, Mh, Rh = sv.history()
    out = dict(rep=rep, J=J, g=g.cpu().numpy(), dt=dt, tm=tm, J_hist=Jh, M_hist=Mh, rel_hist=Rh,
               workspace=sv.workspace_bytes)
    _free(torch, sv)
    return out


def _rel(a, b):
    import numpy as np
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


def channel3d_precisions(w, gamma_dev, res, args, torch):
    """FP64 and FP16S beside the timed FP32 run: one step of each from rest
    (timed; the FP64 state entering the last window is exported on the way,
    outside the timed parts), then the last window of FP32 and FP16S rerun
    from that FP64 state. Errors of J and dJ/dgamma against FP64, from rest
    (each precision on its own trajectory from t = 0) and from the shared
    window start."""
    from paper_2608_19617_amd.solver import Solver
    W_ = w.window_len
    n_before = (w.max_windows - 1) * W_
    upd = (w.max_windows * W_ + W_) * w.nodes
    sv = Solver(w, "f64")
    sv.set_gamma(gamma_dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv.forward(n_before)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    f_start, step = sv.get_state()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sv.forward(W_)
    g64, J64 = sv.adjoint()
    torch.cuda.synchronize()
    t64 = (t1 - t0) + (time.perf_counter() - t2)
    g64 = g64.cpu().numpy()
    J64_hist = sv.history()[0]
    _free(torch, sv)
    mlups = {"f64": upd / t64 / 1e6, args.prec: upd / (res["dt"] / args.steps) / 1e6}
    from_rest = {args.prec: (res["J"], res["g"])}
    for prec in ("f16s", "f32"):
        if prec in from_rest:
            continue
        sv = Solver(w, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep, g, J = channel3d_step(sv, w, gamma_dev)
        torch.cuda.synchronize()
        mlups[prec] = upd / (time.perf_counter() - t0) / 1e6
        from_rest[prec] = (J, g.cpu().numpy())
        _free(torch, sv)
    out = {"f64": {"mlups": round(mlups["f64"], 1), "J": J64, "window_J": [float(j) for j in J64_hist]}}
    for prec in ("f32", "f16s"):
        sv = Solver(w, prec)
        sv.set_gamma(gamma_dev)
        sv.set_state(f_start, step)
        sv.forward(W_)
        g, J = sv.adjoint()
        g = g.cpu().numpy()
        _free(torch, sv)
        Jr, gr = from_rest[prec]
        out[prec] = {"mlups": round(mlups[prec], 1), "speedup_vs_f64": round(mlups[prec] / mlups["f64"], 3),
                     "same_start": {"J_rel_err": abs(J - J64) / abs(J64), "dJdgamma_rel_l2": _rel(g, g64)},
                     "from_rest": {"J": Jr, "J_rel_err": abs(Jr - J64) / abs(J64),
                                   "dJdgamma_rel_l2": _rel(gr, g64)}}
    bars = {"f32": (1e-3, 1e-4), "f16s": (None, 1e-2)}
    for prec, (bj, bg) in bars.items():
        ss = out[prec]["same_start"]
        out[prec]["bars"] = {"J_window_1e-3": None if bj is None else ss["J_rel_err"] <= bj,
                             "dJdgamma_" + ("1e-4" if prec == "f32" else "1e-2"): ss["dJdgamma_rel_l2"] <= bg}
    # the configured 5000-step window amplifies state perturbations about
    # 2e6-fold (bench.py --suite conditioning): its gradient is
    # ill-conditioned, and FP64's own J moves by about 1% when its start
    # state changes by rounding. A 200-step window from the same FP64 state,
    # over which a perturbation decays, shows the storage errors where the
    # gradient is well conditioned.
    out["window_gradient_conditioning"] = "profiles/precision_conditioning.md"
    from paper_2608_19617_amd import workloads as W
    ws = W.cylinder_3d(window_len=200, sample_every=20, ckpt_every=100, n_windows=1)
    short = {}
    for prec in ("f64", "f32", "f16s"):
        sv = Solver(ws, prec)
        sv.set_gamma(gamma_dev)
        sv.set_state(f_start, step)
        sv.forward(ws.window_len)
        g, J = sv.adjoint()
        short[prec] = (J, g.cpu().numpy())
        _free(torch, sv)
    J64s, g64s = short["f64"]
    out["window_200_same_start"] = {
        prec: {"J_rel_err": abs(short[prec][0] - J64s) / abs(J64s), "dJdgamma_rel_l2": _rel(short[prec][1], g64s),
               "meets_" + ("1e-4" if prec == "f32" else "1e-2"): _rel(short[prec][1], g64s) <= (1e-4 if prec == "f32" else 1e-2)}
        for prec in ("f32", "f16s")}
    return out


def _oracle_slab_worker(nz, n_fwd, n_win):
    """The oracle as it stands, single-threaded, on a slab of the channel
    (nz planes of 384 x 128, periodic z): seconds per forward step and per
    adjoint step (a window gradient over n_win steps minus its forward
    steps). Runs in a fresh process."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from threadpoolctl import threadpool_limits
    from helpers import oracle_problem
    from oracle import adjoint as ad
    from oracle import forward as fw
    from paper_2608_19617_amd import workloads as W
    w = W.cylinder_3d(nz=nz, window_len=n_win, sample_every=n_win, ckpt_every=n_win, n_windows=1)
    with threadpool_limits(limits=1):
        prob = oracle_problem(w)
        s = fw.design_map(prob, w.gamma)
        f = fw.initial_state(prob)
        t0 = time.perf_counter()
        for _ in range(n_fwd):
            f = fw.step(prob, f, s)
        t_f = (time.perf_counter() - t0) / n_fwd
        t0 = time.perf_counter()
        ad.window_gradient(prob, w.gamma, f)
        t_a = max((time.perf_counter() - t0) / n_win - t_f, 1e-9)
    return t_f, t_a, w.nodes


def channel3d_cpu_baseline(fwd_per_step, adj_per_step):
    """The oracle on the host's cores, on slabs of the same workload: one
    process alone (single thread), then one process per core of the host's
    share (at most 16) running the same slab at once. Rates are node updates
    per second in the benchmark step's mix of forward and adjoint steps."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    job = (C5_SLAB_NZ, C5_SLAB_FWD, C5_SLAB_WIN)
    with ctx.Pool(1) as pool:
        single = pool.apply(_oracle_slab_worker, job)
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    with ctx.Pool(cores) as pool:
        every = pool.starmap(_oracle_slab_worker, [job] * cores)

    def rate(t_f, t_a, nodes):
        return nodes * (fwd_per_step + adj_per_step) / (fwd_per_step * t_f + adj_per_step * t_a) / 1e6

    value = sum(rate(*r) for r in every)
    t_f, t_a, nodes = single
    return {"value": round(value, 4), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": (f"FP64 numpy oracle on a {C5_SLAB_NZ}-plane slab (384x128x{C5_SLAB_NZ}, periodic z) of the "
                       f"same channel: {C5_SLAB_FWD} forward steps and a {C5_SLAB_WIN}-step window gradient per "
                       f"process, {cores} single-threaded processes at once, rates weighted by the GPU step's mix "
                       f"of {fwd_per_step} forward + {adj_per_step} adjoint steps"),
            "single_thread": {"value": round(rate(*single), 4), "fwd_mlups": round(nodes / t_f / 1e6, 4),
                              "adj_mlups": round(nodes / t_a / 1e6, 4)},
            "per_core_all_cores": {"fwd_mlups": round(sum(r[2] / r[0] for r in every) / cores / 1e6, 4),
                                   "adj_mlups": round(sum(r[2] / r[1] for r in every) / cores / 1e6, 4)}}


def channel3d_roofline(tm, N, prec):
    """Roofline of the dominant kernel of the step (the forward: 20 000 of the
    step's 25 000 updates), from the HIP-event launch averages of the timed
    steps; the counter bytes and SQ figures come from the committed profile
    summary of the same kernel (null when stale)."""
    fb = FWD_BYTES_3D[prec]
    if tm["tb_launches"] > 0 and tm["tb_ms"] >= tm["fwd_ms"]:
        kname = "k_step_tbz (forward, two steps per launch, z-marching)"
        spl = tm["tb_steps"] / tm["tb_launches"]
        launch_s = tm["tb_ms"] / tm["tb_launches"] * 1e-3
        stem = f"k_step_tbz_cyl3d384x128x128_{prec}_counters"
    else:
        kname = "k_step (forward, single step)"
        spl = 1.0
        launch_s = tm["fwd_ms"] / tm["fwd_launches"] * 1e-3
        stem = f"k_step_cyl3d384x128x128_{prec}_counters"
    alg = spl * fb * N
    achieved = alg / launch_s / 1e9
    pv = profile_values(stem)
    traffic = float(pv["hbm_bytes_per_launch"]) if "hbm_bytes_per_launch" in pv else None
    line = {"bound": pv.get("bound", "hbm"), "kernel": kname, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "bytes_per_lup": fb, "algorithmic_bytes_per_launch": alg,
            "steps_per_launch": round(spl, 3), "avg_launch_us": round(launch_s * 1e6, 3)}
    if traffic is not None:
        line["traffic_GBs"] = round(traffic / launch_s / 1e9, 1)
        line["traffic_frac_of_peak"] = round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4)
    for k in ("valu_busy", "waves_per_simd", "binding"):
        if k in pv:
            line[k] = pv[k]
    return line


def channel3d_bench(args, torch):
    import numpy as np
    w = channel3d_workload()
    N = w.nodes
    gamma_dev = _device_gamma(w, torch)
    res = channel3d_timed(w, gamma_dev, args, torch)
    tm = res["tm"]
    fwd_per_step = w.max_windows * w.window_len
    adj_per_step = w.window_len
    value = N * (fwd_per_step + adj_per_step) * args.steps / res["dt"] / 1e6
    fwd_steps = tm["tb_steps"] + tm["fwd_launches"]
    fwd_s = (tm["tb_ms"] + tm["fwd_ms"]) * 1e-3 / fwd_steps
    adj_s = tm["adj_ms"] * 1e-3 / tm["adj_steps"]
    rec_s = tm["rec_ms"] * 1e-3 / max(tm["rec_steps"], 1)
    p = args.prec
    kern = {"forward": {"us_per_step": round(fwd_s * 1e6, 2), "mlups": round(N / fwd_s / 1e6, 1),
                        "bytes_per_lup": FWD_BYTES_3D[p],
                        "frac_of_hbm_peak": round(FWD_BYTES_3D[p] * N / fwd_s / 1e9 / HBM_PEAK_GBS, 4)},
            "recompute": {"us_per_step": round(rec_s * 1e6, 2), "bytes_per_lup": REC_BYTES_3D[p],
                          "frac_of_hbm_peak": round(REC_BYTES_3D[p] * N / rec_s / 1e9 / HBM_PEAK_GBS, 4)},
            "adjoint": {"us_per_step": round(adj_s * 1e6, 2), "mlups": round(N / adj_s / 1e6, 1),
                        "bytes_per_lup": ADJ_BYTES_3D[p],
                        "frac_of_hbm_peak": round(ADJ_BYTES_3D[p] * N / adj_s / 1e9 / HBM_PEAK_GBS, 4)},
            "step_s": round(res["dt"] / args.steps, 3),
            "forward_s_per_step": round(fwd_s * fwd_per_step, 3),
            "reverse_sweep_s_per_step": round((adj_s + rec_s) * adj_per_step, 3)}
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res["dt"] / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": p, "data": "synthetic",
        "config": {"workload": "D3Q19 cylinder channel 384x128x128 (R 16 along z), Re 1000, C_s 0.1, FP32 "
                               "storage, periodic z: 20000 forward steps in 4 windows of 5000 (dW 20, window "
                               "test eps 1e-3 at each window end), adjoint over the last 5000-step window with "
                               "checkpoints every 250 steps in HBM",
                   "grid": list(w.shape), "nodes": N, "tau": w.tau, "window_len": w.window_len,
                   "sample_every": w.sample_every, "ckpt_every": w.ckpt_every,
                   "fwd_steps_per_step": fwd_per_step, "adj_steps_per_step": adj_per_step,
                   "workspace_GB": round(res["workspace"] / 1e9, 1)},
        "roofline": channel3d_roofline(tm, N, p),
        "kernels": kern,
        "J": res["J"],
        "windows": {"J": [float(j) for j in res["J_hist"]],
                    "rel_change": [None if not np.isfinite(r) else float(r) for r in res["rel_hist"]],
                    "criterion_passed_at_last_window": bool(res["rep"]["converged"])},
    }
    if not args.no_compare:
        line["precision"] = channel3d_precisions(w, gamma_dev, res, args, torch)
    if not args.no_cpu:
        line["cpu_baseline"] = channel3d_cpu_baseline(fwd_per_step, adj_per_step)
    print(json.dumps(line), flush=True)


# ------------------- the cylinder wake 2048x512 and the U-bend 1024x1024

def wake2048_suite(args, torch):
    """The cylinder wake 2048 x 512 (disk R = 32, Re 1000, u_max = 0.04,
    C_s = 0.1) in FP32 through WindowedJ: windows of 20 000 steps (dW = 20,
    K = 500) from rest until the criterion (eps = 1e-3) passes or 5 windows
    ran, backward = the adjoint over W_eff; then central differences
    (h = 1e-4) of the window objective through WindowedJ's fixed-start form
    on 16 seed-chosen entries (the disk ramp and the near wake, numpy
    default_rng(0)), in FP32 and in FP64 from the same window-start state."""
    import numpy as np
    from paper_2608_19617_amd import workloads as W
    from paper_2608_19617_amd.autograd import windowed_objective
    from paper_2608_19617_amd.solver import Solver
    w = W.cylinder_wake(window_len=20000, sample_every=20, ckpt_every=500, max_windows=5, eps=1e-3)
    line = {"suite": "wake2048", "workload": "cylinder wake 2048x512 Re 1000, windows of 20000, K 500", "dtype": "f32"}
    sv = Solver(w, "f32")
    gamma = torch.tensor(w.gamma, dtype=torch.float64, device="cuda", requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = windowed_objective(gamma, sv, w.max_windows * w.window_len)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g = gamma.grad.cpu().numpy()
    Jh, Mh, Rh = sv.history()
    w_eff = len(Jh)
    line.update({"w_eff": w_eff, "J": float(J), "window_J": [float(v) for v in Jh],
                 "rel_change": [None if not np.isfinite(r) else float(r) for r in Rh],
                 "forward_s": round(t1 - t0, 3), "adjoint_s": round(t2 - t1, 3),
                 "forward_mlups": round(w_eff * w.window_len * w.nodes / (t1 - t0) / 1e6, 1),
                 "reverse_sweep_mlups": round(w.window_len * w.nodes / (t2 - t1) / 1e6, 1),
                 "workspace_GB": round(sv.workspace_bytes / 1e9, 2)})
    sv.set_gamma(w.gamma)
    sv.forward((w_eff - 1) * w.window_len)
    start = sv.get_state()
    rng = np.random.default_rng(0)
    X, Y = np.meshgrid(np.arange(2048), np.arange(512), indexing="ij")
    cand = np.argwhere(((w.gamma > 0) & (w.gamma < 1)) | ((X >= 544) & (X < 704) & (np.abs(Y - 256) <= 64)))
    pick = [tuple(int(v) for v in cand[i]) for i in rng.choice(len(cand), 16, replace=False)]
    h = 1e-4
    fd = {}
    sv64 = Solver(w, "f64")
    g64_t = torch.tensor(w.gamma, dtype=torch.float64, device="cuda", requires_grad=True)
    J64 = windowed_objective(g64_t, sv64, 0, start=start)
    J64.backward()
    g64 = g64_t.grad.cpu().numpy()
    for name, s_, gref in (("f32", sv, g), ("f64", sv64, g64)):
        errs, errs_top = [], []
        top = float(np.max(np.abs(gref)))
        for p in pick:
            gp = torch.tensor(w.gamma, dtype=torch.float64, device="cuda")
            gm = gp.clone()
            gp[p] += h
            gm[p] -= h
            d = (float(windowed_objective(gp, s_, 0, start=start)) -
                 float(windowed_objective(gm, s_, 0, start=start))) / (2 * h)
            errs.append(abs(d - gref[p]) / max(abs(gref[p]), 1e-300))
            errs_top.append(abs(d - gref[p]) / top)
        fd[name] = {"max_rel_err": float(max(errs)), "median_rel_err": float(np.median(errs)),
                    "max_err_over_max_dJdgamma": float(max(errs_top))}
    _free(torch, sv, sv64)
    line["fd_h=1e-4_16_entries"] = fd
    line["dJdgamma_f32_vs_f64_same_start"] = _rel(g, g64)
    line["fd_entries"] = [list(p) for p in pick]
    print(json.dumps(line), flush=True)


def ubend1024_suite(args, torch):
    """The U-bend 1024 x 1024 (legs of width 128 on the west face, Re 2000,
    uniform inlet 0.03, C_s = 0.1; J = window mean of dissipation plus the
    pressure drop, dW = 20, K = 500): a spin-up window of 10 000 steps, then
    the adjoint over the second 10 000-step window, in FP64, FP32 and FP16S
    from rest (timed) and in FP32 and FP16S from the FP64 state entering the
    second window. J and dJ/dgamma errors against FP64 and FP16S against
    FP32."""
    from paper_2608_19617_amd import workloads as W
    from paper_2608_19617_amd.solver import Solver
    w = W.u_bend(window_len=10000, sample_every=20, ckpt_every=500, max_windows=2)
    w.eps = -1.0
    gamma_dev = _device_gamma(w, torch)
    res = {}
    f_start = None
    for prec in ("f64", "f32", "f16s"):
        sv = Solver(w, prec)
        sv.set_gamma(gamma_dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sv.forward(w.window_len)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if prec == "f64":
            f_start = sv.get_state()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sv.forward(w.window_len)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        g, J = sv.adjoint()
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        res[prec] = {"J": J, "g": g.cpu().numpy(), "forward_s": (t1 - t0) + (t3 - t2), "adjoint_s": t4 - t3}
        _free(torch, sv)
    same = {}
    for prec in ("f32", "f16s"):
        sv = Solver(w, prec)
        sv.set_gamma(gamma_dev)
        sv.set_state(*f_start)
        sv.forward(w.window_len)
        g, J = sv.adjoint()
        same[prec] = (J, g.cpu().numpy())
        _free(torch, sv)
    N = w.nodes
    line = {"suite": "ubend1024", "workload": "U-bend 1024x1024 Re 2000, spin-up window + 10000-step window", "precisions": {}}
    for prec, r in res.items():
        e = {"J": r["J"], "forward_mlups": round(2 * w.window_len * N / r["forward_s"] / 1e6, 1),
             "reverse_sweep_mlups": round(w.window_len * N / r["adjoint_s"] / 1e6, 1),
             "step_s": round(r["forward_s"] + r["adjoint_s"], 3)}
        if prec != "f64":
            J64, g64 = res["f64"]["J"], res["f64"]["g"]
            Js, gs = same[prec]
            e["speedup_vs_f64"] = round((res["f64"]["forward_s"] + res["f64"]["adjoint_s"]) / e["step_s"], 3)
            e["vs_f64_from_rest"] = {"J_rel_err": abs(r["J"] - J64) / abs(J64), "dJdgamma_rel_l2": _rel(r["g"], g64)}
            e["vs_f64_same_start"] = {"J_rel_err": abs(Js - J64) / abs(J64), "dJdgamma_rel_l2": _rel(gs, g64)}
        line["precisions"][prec] = e
    J32, g32 = same["f32"]
    J16, g16 = same["f16s"]
    line["f16s_vs_f32_same_start"] = {"J_rel_err": abs(J16 - J32) / abs(J32), "dJdgamma_rel_l2": _rel(g16, g32)}
    line["f16s_vs_f32_from_rest"] = {"J_rel_err": abs(res["f16s"]["J"] - res["f32"]["J"]) / abs(res["f32"]["J"]),
                                     "dJdgamma_rel_l2": _rel(res["f16s"]["g"], res["f32"]["g"])}
    print(json.dumps(line), flush=True)


# ------------------------------------------------------ conditioning suite

def _conditioning_cases():
    """(name, workload factory for a window of L steps, spin-up steps S,
    window lengths, the window of the configuration, finite-difference
    entries, finite-difference steps h)."""
    from paper_2608_19617_amd import workloads as W

    def channel3d(L):
        return W.cylinder_3d(window_len=L, sample_every=20, ckpt_every=min(250, L // 2), n_windows=1)

    def wake(L):
        return W.cylinder_wake(window_len=L, sample_every=20, ckpt_every=min(500, L // 2), max_windows=1, eps=-1.0)

    def bfs(L):
        w = W.backward_facing_step(window_len=L, sample_every=100, ckpt_every=min(100, L), max_windows=1, eps=-1.0)
        return w

    def ubend(L):
        return W.u_bend_paper(400.0, window_len=L, sample_every=20, ckpt_every=min(500, L // 2), max_windows=1,
                              eps=-1.0)

    hs = (1e-3, 1e-4, 1e-5, 1e-6)
    return [("cylinder_3d_384x128x128", channel3d, 15000, (40, 200, 1000, 5000), 5000, 4, hs),
            ("cylinder_wake_2048x512", wake, 20000, (100, 1000, 5000, 20000), 20000, 8, hs),
            ("backward_facing_step_800x200", bfs, 38000, (100, 500, 2000), 2000, 8, hs),
            ("u_bend_paper_240x192_re400", ubend, 40000, (2000, 5000, 10000, 20000), 20000, 12,
             (1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8))]


def _fd_entries(g, n, seed):
    """n seeded entries among the nodes whose |dJ/dgamma| is in the top 5%."""
    import numpy as np
    a = np.abs(g).ravel()
    thr = np.quantile(a, 0.95)
    cand = np.flatnonzero(a >= thr) if thr > 0 else np.flatnonzero(a > 0)
    pick = np.random.default_rng(seed).choice(cand, min(n, len(cand)), replace=False)
    return [np.unravel_index(int(i), g.shape) for i in pick]


def conditioning_suite(args, torch):
    import numpy as np
    from paper_2608_19617_amd.solver import Solver

    def window(w, prec, f, step, keep_state=False):
        sv = Solver(w, prec)
        sv.set_state(f, step)
        rep = sv.forward(w.window_len)
        fe = sv.get_state()[0] if keep_state else None
        g, J = sv.adjoint()
        return sv, rep, J, g.cpu().numpy(), fe

    for name, make, S, lengths, w_cfg, n_fd, hs in _conditioning_cases():
        if args.case not in name:
            continue
        w0 = make(lengths[0])
        sv = Solver(w0, "f64")
        sv.forward(S)
        f64_S, step = sv.get_state()
        _free(torch, sv)
        rng = np.random.default_rng(1)
        delta = 1e-8 * rng.standard_normal(f64_S.shape) * np.abs(f64_S).mean()
        for L in lengths:
            w = make(L)
            t0 = time.perf_counter()
            sv64, rep, J64, g64, fe64 = window(w, "f64", f64_S, S, keep_state=True)
            pts = _fd_entries(g64, n_fd, 0)
            top = float(np.max(np.abs(g64)))
            fd = {}
            for h in hs:
                errs = []
                for p in pts:
                    gp = w.gamma.copy()
                    gm = w.gamma.copy()
                    hp = min(h, 1.0 - gp[p]) if gp[p] + h > 1.0 else h
                    hm = min(h, gm[p]) if gm[p] - h < 0.0 else h
                    gp[p] += hp
                    gm[p] -= hm
                    d = (sv64.replay(gp) - sv64.replay(gm)) / (hp + hm)
                    errs.append(abs(d - g64[p]) / top)
                fd[f"h={h:g}"] = float(max(errs))
            _free(torch, sv64)
            # growth of a small state perturbation over the window (FP64)
            svp = Solver(w, "f64")
            svp.set_state(f64_S + delta, S)
            svp.forward(L)
            fe_p = svp.get_state()[0]
            _free(torch, svp)
            growth = float(np.linalg.norm(fe_p - fe64) / np.linalg.norm(delta))
            line = {"suite": "conditioning", "workload": name, "grid": list(w.shape), "window_len": L,
                    "spin_up_steps": S, "J_f64": J64, "dJdgamma_norm_f64": float(np.linalg.norm(g64)),
                    "dJdgamma_max_f64": top, "fd_f64_max_err_over_max_dJdgamma": fd,
                    "fd_entries": len(pts), "perturbation_growth": growth}
            for prec in ("f32", "f16s"):
                svr, _, J, g, _ = window(w, prec, f64_S, S)
                _free(torch, svr)
                line[prec] = {"J_rel_err": abs(J - J64) / abs(J64), "dJdgamma_rel_l2": _rel(g, g64),
                              "dJdgamma_norm": float(np.linalg.norm(g))}
            line["s"] = round(time.perf_counter() - t0, 2)
            print(json.dumps(line), flush=True)
        # from rest: how much of each precision's error comes from its own
        # window-start state (the FP64 adjoint run from that state) and how
        # much from rounding inside the window (the same-start error)
        w = make(w_cfg)
        sv64, _, J64, g64, _ = window(w, "f64", f64_S, S)
        _free(torch, sv64)
        out = {"suite": "conditioning", "workload": name, "window_len": w_cfg, "from_rest_decomposition": {}}
        for prec in ("f32", "f16s"):
            sv = Solver(w0, prec)
            sv.forward(S)
            fp_S, _ = sv.get_state()
            _free(torch, sv)
            sva, _, Jp, gp, _ = window(w, prec, fp_S, S)
            _free(torch, sva)
            svb, _, Jb, gb, _ = window(w, "f64", fp_S, S)
            _free(torch, svb)
            svc, _, Jc, gc, _ = window(w, prec, f64_S, S)
            _free(torch, svc)
            out["from_rest_decomposition"][prec] = {
                "start_state_rel_l2_vs_f64": float(np.linalg.norm(fp_S - f64_S) / np.linalg.norm(f64_S)),
                "from_rest": {"J_rel_err": abs(Jp - J64) / abs(J64), "dJdgamma_rel_l2": _rel(gp, g64)},
                "f64_from_this_start": {"J_rel_err": abs(Jb - J64) / abs(J64), "dJdgamma_rel_l2": _rel(gb, g64)},
                "same_start": {"J_rel_err": abs(Jc - J64) / abs(J64), "dJdgamma_rel_l2": _rel(gc, g64)}}
        print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is designed but not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.counters:
        counters_run(args, torch)
        return
    suites = {"bfs": bfs_bench, "hbm": hbm_suite, "design": design_suite, "fulltime": fulltime_suite,
              "paper": paper_suite, "optimize": optimize_suite, "conditioning": conditioning_suite,
              "wake2048": wake2048_suite, "ubend1024": ubend1024_suite}
    if args.suite:
        suites[args.suite](args, torch)
        return
    channel3d_bench(args, torch)


if __name__ == "__main__":
    main()
