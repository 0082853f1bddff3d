/*
 * lbm.h - C ABI of the windowed regularized LBM-LES solver and its discrete
 * adjoint for AMD Instinct MI355X (gfx950).
 *
 * The library computes, on one GPU, the data-parallel hot path of the
 * representative-time-window adjoint method ("Adaptive Time Windows for
 * Discrete Adjoint Topology Optimization of Unsteady Flows"):
 *   - the regularized D2Q9 (or D3Q19) BGK step with Smagorinsky eddy
 *     viscosity (Sec. 2.1.1-2.1.2, Eqs. feq, Pi, tau_eff,
 *     modified_collision), partial bounce-back driven by a per-node design
 *     field gamma (Sec. 2.2, Eq. external_force), streaming with halfway
 *     bounce-back walls and Zou-He inlet / outlet rows (Sec. 2.1.3,
 *     Eqs. wall, inlet, outlet);
 *   - window-averaged objective and monitor samples and the
 *     consecutive-window convergence test (Sec. 3.1, Eqs. statistical_force,
 *     statistical_criterion, weighted_temporal_sampling, Algorithm
 *     "LES solver");
 *   - the discrete adjoint over the last completed window, which returns
 *     dJ/dgamma (Sec. 3.2, Eqs. adjoint_collision, adjoint_streaming,
 *     adjoint_inlet_bc, adjoint_outlet_bc, sensitivity).
 *
 * Conventions
 *   - gamma is the per-node design field, 1 = solid, 0 = fluid (the paper's
 *     phi is 1 - gamma). The bounce-back fraction is s = gamma
 *     (LBM_S_LINEAR) or s = g(1 - gamma) with the paper's convex
 *     interpolation g(phi) = 0.5 (1 - phi (1+q)/(phi+q)) (LBM_S_PAPER).
 *   - Node order is x fastest: node = (z * ny + y) * nx + x (nz = 1 in 2D).
 *     Population arrays are structure-of-arrays: f[alpha * N + node],
 *     N = nx * ny * nz. D2Q9 directions are ordered as printed in the
 *     paper (rest, E, N, W, S, NE, NW, SW, SE); D3Q19 as rest, +x, -x, +y,
 *     -y, +z, -z, then the 12 edge directions (+-x+-y, +-x+-z, +-y+-z with
 *     the first sign slowest).
 *   - Time: f^k is the post-streaming, post-boundary state after k steps
 *     (f^0 = f^eq(rho_init, u_init)). Window i (1-based) is the |W|
 *     transitions ending at step i*|W|; its samples are taken on f^k at
 *     the end-aligned instants k = (i-1)|W| + m*dW, m = 1..|W|/dW, each
 *     weighted dW/|W|.
 *   - The adjoint differentiates the window-restricted subproblem: the
 *     state entering the window is held fixed.
 *
 * Memory and streams
 *   - The caller owns all device memory: the workspace (sized by
 *     lbm_workspace_bytes), the gamma array and the dJ/dgamma array. The
 *     library never allocates device memory. All work is enqueued on the
 *     caller's HIP stream (passed as void*, a hipStream_t). The library
 *     synchronises that stream only at window ends inside lbm_forward and
 *     before lbm_forward, lbm_adjoint, lbm_window_replay, lbm_get_state
 *     and lbm_set_state return.
 *   - A context is bound to one stream and is not thread-safe.
 *
 * Errors
 *   - Every call returns an lbm_status; lbm_last_error() gives a
 *     thread-local message for the last failure. Arguments are validated
 *     before any HIP call (LBM_E_INVALID). HIP failures return LBM_E_HIP.
 *     A sampled state with a non-finite value or |u| >= 0.4 returns
 *     LBM_E_UNSTABLE at the end of that window; the context then needs
 *     lbm_reset, lbm_set_gamma or lbm_set_state. LBM_E_STATE reports a call
 *     made in the wrong state (e.g. lbm_adjoint before any window ended).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_E_INVALID = 1,
    LBM_E_NOMEM = 2,      /* workspace smaller than lbm_workspace_bytes */
    LBM_E_HIP = 3,
    LBM_E_UNSTABLE = 4,
    LBM_E_STATE = 5
} lbm_status;

enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };                 /* lattice */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2 };      /* population storage */
enum { LBM_WALL = 0, LBM_VELOCITY = 1, LBM_PRESSURE = 2 }; /* x-face row kinds */
enum { LBM_S_LINEAR = 0, LBM_S_PAPER = 1 };           /* s(gamma) */
/* Objective / monitor kinds (Sec. 3.1 and the examples of Sec. 4):
 *   LBM_J_PRESSURE_DROP        c_s^2 (mean rho over sec_in - mean over sec_out)
 *   LBM_J_DISSIPATION_PLUS_DP  sum of the node dissipation 2 rho nu_eff S:S plus
 *                              the pressure drop
 *   LBM_J_DRAG                 objective: the drag D = sum over force_box of
 *                              2 s rho u_x, the x force the flow exerts on the
 *                              porous solid (minus the x part of the force of
 *                              Eq. external_force summed over the directions);
 *                              monitor: the drag coefficient C_d = D / drag_ref
 *                              (Eq. C_d)
 *   LBM_J_WAKE                 objective only (wake recovery): the window value
 *                              J = sum over meas_box of |u_bar - u_ref|^2, u_bar
 *                              the dW/|W|-weighted sum of the sampled u = j / rho
 *                              over the window, u_ref set by
 *                              lbm_set_wake_reference (zero until then) */
enum { LBM_J_PRESSURE_DROP = 0, LBM_J_DISSIPATION_PLUS_DP = 1, LBM_J_DRAG = 2, LBM_J_WAKE = 3 };

/*
 * Problem description. Storage precisions: LBM_F64 stores and computes in
 * FP64; LBM_F32 stores f - w_alpha in FP32 and computes in FP32; LBM_F16S
 * stores f - w_alpha in IEEE binary16 (round to nearest even) and computes
 * in FP32. The adjoint populations are FP64 in LBM_F64, FP32 otherwise.
 * Objective, monitor, window means and dJ/dgamma are always accumulated in
 * FP64.
 */
typedef struct {
    int lattice;                 /* LBM_D2Q9 or LBM_D3Q19 */
    int nx, ny, nz;              /* nodes per axis; nz = 1 for D2Q9 */
    double tau;                  /* molecular relaxation time, > 0.5 */
    double c_smag;               /* Smagorinsky constant C_s >= 0 (filter width = 1) */
    int prec;                    /* LBM_F64 / LBM_F32 / LBM_F16S */
    int s_map;                   /* LBM_S_LINEAR or LBM_S_PAPER */
    double s_q;                  /* interpolation parameter q of LBM_S_PAPER, > 0 */
    int periodic_x, periodic_y, periodic_z; /* 1 = periodic axis; else walls / open rows */
    const int* west;             /* host, ny entries, x = 0 face row kinds (NULL = all wall) */
    const int* east;             /* host, ny entries, x = nx-1 face (LBM_WALL or LBM_PRESSURE) */
    const double* u_in;          /* host, ny entries: inlet x-velocity u0 of each velocity row */
    double rho_out;              /* prescribed outlet density rho_0 of pressure rows */
    double rho_init;             /* initial density */
    int u_init_mode;             /* 0: u(x,0) = 0; 1: u(x,0) = (u_in(y), 0[, 0]) */
    int window_len;              /* |W| in steps */
    int sample_every;            /* dW, must divide window_len */
    int max_windows;             /* W_max of the window loop (stop_on_converge runs) */
    double eps;                  /* criterion tolerance; < 0 disables the test */
    int objective;               /* LBM_J_* : sampled objective j(t) */
    int monitor;                 /* LBM_J_* : monitored quantity of the criterion */
    int sec_in_x, sec_in_lo, sec_in_hi;    /* inlet pressure section: x, rows [lo, hi), all z */
    int sec_out_x, sec_out_lo, sec_out_hi; /* outlet pressure section */
    int ckpt_every;              /* K: checkpoint interval, must divide window_len */
    int full_history;            /* 1: also keep the start state of every window (for
                                    lbm_adjoint_full); 0: the two newest windows only */
    int force_box[6];            /* x0, x1, y0, y1, z0, z1: half-open node box of the drag
                                    sum; x1 <= x0 means the whole grid; z ignored in 2D */
    double drag_ref;             /* rho_0 u_0^2 L_ref / 2, the denominator of C_d; must be
                                    > 0 when the monitor is LBM_J_DRAG */
    int meas_box[6];             /* measurement region M of LBM_J_WAKE, as force_box */
} lbm_config;

/* Result of lbm_forward. w_eff is the 1-based index of the last completed
 * window (0 if none); converged tells whether that window passed the
 * criterion; J_eff and monitor are its objective and monitor means. */
typedef struct {
    long steps_done;             /* total steps since t = 0 */
    int windows_done;
    int converged;
    int w_eff;
    double J_eff;
    double monitor;
    double rel_change;           /* |(M_i - M_{i-1}) / M_i| of the last window (NaN for window 1) */
    int unstable;
} lbm_fwd_report;

typedef struct lbm_ctx lbm_ctx;

/* Bytes of device workspace that lbm_init needs for this configuration
 * (state ping-pong, two checkpoint rings of |W|/K slots, the recompute
 * slots of a segment: two states and K - 1 moment records of 6 (D2Q9) or
 * 10 (D3Q19) values per node in the compute precision (FP64 for LBM_F64,
 * else FP32); adjoint buffers, sample partials;
 * with full_history also max_windows window-start states and a third
 * ring). Validates the configuration. */
lbm_status lbm_workspace_bytes(const lbm_config* cfg, size_t* bytes);

/* Creates a context: the setup of the problem statement (Sec. 2.1.3 initial
 * and boundary conditions; Sec. 2.2 bounce-back fraction s(gamma), Eq.
 * external_force): builds s from gamma, the per-row boundary tables and
 * inlet speeds, and f^0 = f^eq(rho_init, u_init) (Eq. feq). gamma_dev:
 * device FP64 array of N design values in [0, 1] (copied; the caller may
 * reuse it). workspace_dev: device memory of at least lbm_workspace_bytes
 * bytes, 256-byte aligned, owned by the caller and used exclusively by this
 * context until lbm_destroy. stream: the hipStream_t every launch goes to.
 * Errors: LBM_E_INVALID for a bad configuration (checked before any HIP
 * call) or a gamma entry that is not finite (or, with LBM_S_PAPER, outside
 * the map's range), LBM_E_NOMEM for a short workspace, LBM_E_HIP if a HIP
 * call fails; *out is set only on LBM_OK. */
lbm_status lbm_init(const lbm_config* cfg, const double* gamma_dev, void* workspace_dev,
                    size_t bytes, void* stream, lbm_ctx** out);

/* Copies a new design field (device FP64, N values) and resets to t = 0. */
lbm_status lbm_set_gamma(lbm_ctx* ctx, const double* gamma_dev);

/* Resets the state to f^0 and clears the window history. */
lbm_status lbm_reset(lbm_ctx* ctx);

/* Advances at most n_steps steps (Algorithm "LES solver"). Samples the
 * objective and monitor, checkpoints the current window every K steps, and
 * applies the criterion at each window end. With stop_on_converge it stops
 * at the first window that passes the criterion or when max_windows windows
 * have completed (not an error: rep->converged = 0). rep may be NULL. */
lbm_status lbm_forward(lbm_ctx* ctx, long n_steps, int stop_on_converge, lbm_fwd_report* rep);

/* Copies the per-window objective means, monitor means and relative changes
 * (NaN for the first window) of the windows completed so far, oldest first,
 * into host arrays of capacity cap (any may be NULL). *n = windows done. */
lbm_status lbm_window_history(lbm_ctx* ctx, double* J, double* M, double* rel, int cap, int* n);

/* Discrete adjoint over window `window` (1-based), which must be the last
 * completed window (or pass 0 for it): the reverse sweep of Sec. 3.2 over
 * the window-restricted subproblem (adjoint boundary rules, Eqs.
 * adjoint_inlet_bc and adjoint_outlet_bc; adjoint streaming, Eq.
 * adjoint_streaming; adjoint collision, Eq. adjoint_collision; objective
 * sources at the sampling instants, Eq. weighted_temporal_sampling), then
 * the design gradient of Eq. sensitivity with ds/dgamma. Writes dJ/dgamma
 * (device FP64, N values, caller-owned) and, if J_out is not NULL, the
 * window objective. The forward state is not changed. Recomputes each
 * K-step segment from its HBM checkpoint. Errors: LBM_E_STATE without a
 * completed window, for another window or after LBM_E_UNSTABLE. The drag's samples depend on s directly: their explicit
 * derivative, dW/|W| times 2 j_x summed over the window's samples, is kept
 * by the forward on the force box and added here. */
lbm_status lbm_adjoint(lbm_ctx* ctx, int window, double* dJdgamma_dev, double* J_out);

/* Full-time adjoint (the comparison case of Sec. "Comparison with full-time
 * adjoint optimization"): dJ/dgamma of the same objective J (the last
 * completed window) with the adjoint carried back through every earlier
 * window to the start of the history (t = 0 after lbm_init, lbm_reset or
 * lbm_set_gamma; the lbm_set_state step otherwise), so that the state
 * entering the window is not held fixed. Needs cfg.full_history = 1: the
 * start state of every window is kept, each earlier window is replayed from
 * it once to rebuild its K-step checkpoints, and its reverse sweep takes no
 * objective source. Errors: LBM_E_STATE without full history, without a
 * completed window, or when more than max_windows windows have run since
 * the start of the history. Writes dJ/dgamma (device FP64, N) and J. */
lbm_status lbm_adjoint_full(lbm_ctx* ctx, double* dJdgamma_dev, double* J_out);

/* Replays the last completed window from its (fixed) start state with the
 * design field gamma_dev (device FP64, N values) and returns its objective:
 * the function lbm_adjoint differentiates, for finite-difference checks on
 * the same window and sampling instants (the validation protocol of Sec.
 * 4.2.1). The forward state, checkpoints and the context's own gamma are
 * unchanged. Errors: LBM_E_STATE without a completed window, LBM_E_INVALID
 * for a gamma entry that is not finite (or outside the LBM_S_PAPER map's
 * range). */
lbm_status lbm_window_replay(lbm_ctx* ctx, const double* gamma_dev, double* J_out);

/* Wake recovery (objective LBM_J_WAKE): sets the reference mean velocity
 * u_ref on the measurement box M from device FP64 memory, D planes of |M|
 * values (component p of box node (i, j, k) at p |M| + (k nyM + j) nxM + i,
 * box coordinates relative to its low corner). Window values of later
 * windows and replays, and the adjoint, use it. LBM_E_STATE if the
 * objective is not LBM_J_WAKE. */
lbm_status lbm_set_wake_reference(lbm_ctx* ctx, const double* u_ref_dev);

/* Wake recovery: the window-mean velocity u_bar of the last completed
 * window on M (layout of lbm_set_wake_reference) to device FP64 memory.
 * With the flow of a reference design, this is the u_ref of the problem.
 * LBM_E_STATE if the objective is not LBM_J_WAKE or no window completed. */
lbm_status lbm_wake_mean_velocity(lbm_ctx* ctx, double* u_bar_dev);

/* Exports the current state f^k (unshifted populations, FP64, Q*N values in
 * SoA order) to host memory, and its step k. */
lbm_status lbm_get_state(lbm_ctx* ctx, double* host_f, long* step);

/* Replaces the state by f^k given in host memory (layout of lbm_get_state).
 * step must be a multiple of window_len; the window history is cleared and
 * windows continue from step. */
lbm_status lbm_set_state(lbm_ctx* ctx, const double* host_f, long step);

/* Writes rho, u_x, u_y[, u_z] of the current state to device FP64 memory
 * (planes of N values). */
lbm_status lbm_get_fields(lbm_ctx* ctx, double* rho_u_dev);

/* HIP-event timing of the hot kernels: one event pair brackets each run of
 * back-to-back launches of the forward step kernel, of the adjoint step
 * kernel and of the recompute step launches. enable = 1 starts it (and
 * clears the counters), 0 stops it. If out is not NULL it receives
 * launches and total milliseconds of each class,
 * so ms / launches is the average launch duration including the dispatch
 * gaps between consecutive launches. A fourth pair counts the temporally
 * blocked forward launches; the ninth double is the steps they advanced and
 * the tenth the steps advanced by the recompute launches, which are also
 * blocked where the forward is, the eleventh the steps advanced by the
 * adjoint launches (11 doubles in all). */
lbm_status lbm_timing(lbm_ctx* ctx, int enable, double* out);

/* Temporal blocking of forward launches (D2Q9 only): each launch advances
 * nsteps steps on output tiles of tile_x x tile_y nodes, keeping the
 * intermediate populations of each tile and its halo in LDS. nsteps = 1
 * turns it off. Samples, checkpoints and window ends always fall on the last
 * step of a launch, so results are those of single steps up to the
 * contraction of multiply-adds. With R = (tile_x + 2(nsteps-1)) *
 * (tile_y + 2(nsteps-1)) region nodes, requires tile_x * tile_y >= 256 and
 * 18 R state values (FP16 for FP16S, else the compute type), R compute-type
 * values of s and a row cache of (tile_y + 2(nsteps-1)) * (value + 2 bytes)
 * within 159 KB (R may be rounded up to a fixed plane stride). FP16S
 * intermediate states are rounded to FP16 as a single step stores them.
 * A launch never runs past the next sample,
 * checkpoint or window end, so shorter blocked launches occur. Defaults
 * after lbm_init (measured on MI355X): grids of at most 400k nodes use
 * square tiles of about N / 256 nodes (16 to 25 per side) and 10 steps
 * (FP32, FP16S) or 4 steps (FP64); larger grids 6 steps on 64 x 16 tiles
 * (FP32), 2 steps on 32 x 8 (FP64), and for FP16S (whose LDS holds FP16
 * states) 6 steps on 48 x 48 below 4M nodes, 5 steps on 64 x 40 above. The
 * recompute of the adjoint sweep uses the same blocking, storing the moment
 * record of every recomputed step. The adjoint steps that read their
 * pre-state's record from a recomputed segment run blocked too (see lbm_set_adjoint_blocking); this
 * call sets their default: on grids of more than 400k nodes 4 steps on
 * 25 x 25 tiles (FP64) or 5 steps on 48 x 24 (FP32, FP16S), else the
 * forward's steps and tiles, falling back to the first of 48 x 24, 64 x 16,
 * 32 x 32, 32 x 16, 16 x 16 whose LDS allows two or more steps; nsteps = 1
 * turns both off. */
lbm_status lbm_set_blocking(lbm_ctx* ctx, int nsteps, int tile_x, int tile_y);

/* Temporal blocking of D3Q19 forward launches: nsteps = 2 advances two
 * steps per launch (the recompute of the adjoint sweep too, storing the
 * moment records of both steps). A workgroup owns tile_x x tile_y nodes in
 * x and y and tile_z consecutive z planes; it takes the first step plane by
 * plane over the tile grown by one node in x and y, keeping that state in
 * an LDS ring (walls on x and y faces as ghost cells, as for D2Q9), and the
 * second step of each plane as soon as the plane above is ready. The ring
 * keeps each direction of a plane only as long as the second step reads it
 * (43 plane slots in all). nsteps = 1 turns it off. Requires
 * at least 256 nodes per block, (tile_x + 2) * (tile_y + 2) <= 1024 and
 * (tile_x + 2)(tile_y + 2) x (43 state values in the storage-rounded LDS
 * type + two compute-type values) within 159 KB, and a state (19 x nodes x
 * storage bytes) and a moment record (10 x nodes x compute bytes) below
 * 4 GB each. Samples, checkpoints and window ends fall on a launch's last
 * step as in 2D. This call sets the tiles of the recompute's launches to
 * the same. Default (set by lbm_init) on grids of more than 2M nodes:
 * FP32 takes 2 steps on 48 x 16 tiles (1024 threads per workgroup; 32 x 19
 * with 768 threads where nx < 48 or ny < 16) and its recompute 2 steps on
 * 32 x 19 tiles (768 threads), FP64 2 steps on 48 x 7 tiles
 * (512 threads; 32 x 10 where nx < 48), each with the z run that lets the
 * blocks fill the compute units in nearly whole rounds with the fewest halo
 * planes; FP16S and smaller grids take single steps.
 * Errors: LBM_E_INVALID for a D2Q9 context or out-of-range arguments,
 * LBM_E_HIP if the LDS opt-in fails. */
lbm_status lbm_set_blocking_3d(lbm_ctx* ctx, int nsteps, int tile_x, int tile_y, int tile_z);

/* Blocking of the adjoint launches that read their pre-states' moment
 * records from a recomputed segment (D2Q9 only): up to nsteps reverse
 * steps per launch on tile_x x tile_y output tiles, the adjoint populations (FP32, or FP64 for
 * LBM_F64) of the tile and its halo and an FP64 sensitivity plane of the
 * tile in LDS. nsteps = 1 turns it off. Requires tile_x * tile_y >= 256 and
 * tile_x * tile_y * 8 bytes plus 19 R values of the adjoint type plus the
 * row cache within 159 KB (R as for lbm_set_blocking). lbm_set_blocking
 * resets it to its default (described there). Errors: LBM_E_INVALID for
 * out-of-range arguments, LBM_E_HIP if the LDS opt-in fails. */
lbm_status lbm_set_adjoint_blocking(lbm_ctx* ctx, int nsteps, int tile_x, int tile_y);

/* Blocking of the D3Q19 adjoint launches that read their pre-states'
 * moment records from a recomputed segment: nsteps = 2 takes two reverse
 * steps per launch. A workgroup owns tile_x x tile_y nodes in x and y and
 * tile_z consecutive z planes; the first step runs plane by plane over the
 * tile grown by one node in x and y, keeping its adjoint populations in an
 * LDS ring that holds each direction only as long as the second step
 * gathers it (43 plane slots; walls on x and y faces as ghost cells, 0
 * behind open faces), and the second gathers from it; each step reads its
 * own pre-state's record from the segment, and the tile's sensitivity
 * takes one FP64 read-modify-write per launch. nsteps = 1 turns it off.
 * Requires at least 256 nodes per block, (tile_x + 2) * (tile_y + 2) <= 768
 * (one thread per region cell), (tile_x + 2) x (tile_y + 2) x (16 + two
 * compute-type values + 43 adjoint values) bytes within 159 KB (in FP64
 * about 430 region cells), and a moment record and the adjoint populations
 * below 4 GB each. Default (set by lbm_init) on grids of more than 2M
 * nodes: 2 steps on 48 x 13 tiles with 768 threads for FP32 and FP16S
 * storage (32 x 19 where nx < 48), on 40 x 8 tiles with 512 threads for
 * FP64 (32 x 10 where nx < 40), with the z run chosen as for the forward;
 * smaller grids take single steps. Errors: LBM_E_INVALID for a D2Q9 context
 * or out-of-range arguments, LBM_E_HIP if the LDS opt-in fails. */
lbm_status lbm_set_adjoint_blocking_3d(lbm_ctx* ctx, int nsteps, int tile_x, int tile_y, int tile_z);

/* Thread-local message of the last failing call on this thread. */
const char* lbm_last_error(void);

/* Frees the host-side context. The workspace stays with the caller. */
void lbm_destroy(lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
