// Host driver and C ABI (include/lbm.h): workspace layout, window loop
// with the consecutive-window test, HBM checkpoint rings, the checkpointed
// reverse sweep, replays for finite differences, state import / export.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "lbm.h"
#include "launch.hpp"

using namespace lbm;

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(LBM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
    int nstart;                // window-start states kept (full history)
    size_t off_starts, off_ringrep;
    int Q, D;
    long N;
    size_t ss, cs, as;         // bytes per stored / compute / adjoint value
    size_t SB;                 // bytes of one population state
    int R;                     // checkpoint slots per window
    int nseg;                  // recompute state slots
    int nrec;                  // recompute record slots (D2Q9: K - 1, at least 1; D3Q19: 0)
    size_t RB;                 // bytes of one moment record of all nodes
    long nblocks;
    long pstride;
    int nsamp;                 // samples per window
    size_t off_G, off_ring, off_seg, off_rec, off_s, off_srep, off_gamma, off_nu, off_sens, off_part, off_samples,
        off_acc, off_roww, off_rowe, off_uin, total;
    int fbox[6], mbox[6];      // force and measurement boxes, resolved
    int ncomp;                 // window-field components: 1 (drag), D (wake), 0
    long nb, nf;               // nodes of the accumulator box; nb * ncomp
    size_t off_facc;           // three accumulators, the wake reference, reduction scratch
};

constexpr int FACC_PARTS = 1024;   // block partials of the wake window value

// A half-open box x0, x1, y0, y1, z0, z1; x1 <= x0 selects the whole grid;
// z is [0, 1) in 2D.
bool resolve_box(const lbm_config* c, const int* b, int out[6]) {
    const int n[3] = {c->nx, c->ny, c->nz};
    const bool whole = b[1] <= b[0];
    for (int a = 0; a < 3; ++a) {
        const bool take_all = whole || (a == 2 && c->lattice == LBM_D2Q9);
        out[2 * a] = take_all ? 0 : b[2 * a];
        out[2 * a + 1] = take_all ? n[a] : b[2 * a + 1];
        if (out[2 * a] < 0 || out[2 * a] >= out[2 * a + 1] || out[2 * a + 1] > n[a]) return false;
    }
    return true;
}

lbm_status validate(const lbm_config* c) {
    if (!c) return fail(LBM_E_INVALID, "config is NULL");
    if (c->lattice != LBM_D2Q9 && c->lattice != LBM_D3Q19) return fail(LBM_E_INVALID, "unknown lattice");
    if (c->nx < 3 || c->ny < 3 || c->nz < 1) return fail(LBM_E_INVALID, "grid must be at least 3 x 3");
    if (c->lattice == LBM_D2Q9 && c->nz != 1) return fail(LBM_E_INVALID, "D2Q9 needs nz = 1");
    if (c->lattice == LBM_D3Q19 && c->nz < 3) return fail(LBM_E_INVALID, "D3Q19 needs nz >= 3");
    const double nodes = (double)c->nx * c->ny * c->nz;
    if (nodes * (c->lattice == LBM_D2Q9 ? 9 : 19) > 2147483647.0)
        return fail(LBM_E_INVALID, "grid too large (Q * nodes must stay below 2^31)");
    if (!(c->tau > 0.5) || !std::isfinite(c->tau)) return fail(LBM_E_INVALID, "tau must be > 0.5");
    if (!(c->c_smag >= 0.0) || !std::isfinite(c->c_smag)) return fail(LBM_E_INVALID, "c_smag must be >= 0");
    if (c->prec < LBM_F64 || c->prec > LBM_F16S) return fail(LBM_E_INVALID, "unknown precision");
    if (c->s_map != LBM_S_LINEAR && c->s_map != LBM_S_PAPER) return fail(LBM_E_INVALID, "unknown s_map");
    if (c->s_map == LBM_S_PAPER && !(c->s_q > 0.0)) return fail(LBM_E_INVALID, "s_q must be > 0");
    if (c->window_len < 1 || c->sample_every < 1 || c->window_len % c->sample_every != 0)
        return fail(LBM_E_INVALID, "sample_every must divide window_len");
    if (c->ckpt_every < 1 || c->window_len % c->ckpt_every != 0)
        return fail(LBM_E_INVALID, "ckpt_every must divide window_len");
    if (c->max_windows < 1) return fail(LBM_E_INVALID, "max_windows must be >= 1");
    if (c->full_history != 0 && c->full_history != 1) return fail(LBM_E_INVALID, "full_history must be 0 or 1");
    if (std::isnan(c->eps)) return fail(LBM_E_INVALID, "eps is NaN");
    if (c->objective < LBM_J_PRESSURE_DROP || c->objective > LBM_J_WAKE || c->monitor < LBM_J_PRESSURE_DROP ||
        c->monitor > LBM_J_DRAG)
        return fail(LBM_E_INVALID, "unknown objective or monitor");
    int box[6];
    if (!resolve_box(c, c->force_box, box)) return fail(LBM_E_INVALID, "bad force_box");
    if (!resolve_box(c, c->meas_box, box)) return fail(LBM_E_INVALID, "bad meas_box");
    if (c->monitor == LBM_J_DRAG && !(c->drag_ref > 0.0 && std::isfinite(c->drag_ref)))
        return fail(LBM_E_INVALID, "drag_ref must be > 0 for the C_d monitor");
    if (c->sec_in_x < 0 || c->sec_in_x >= c->nx || c->sec_out_x < 0 || c->sec_out_x >= c->nx ||
        c->sec_in_lo < 0 || c->sec_in_hi > c->ny || c->sec_in_lo >= c->sec_in_hi || c->sec_out_lo < 0 ||
        c->sec_out_hi > c->ny || c->sec_out_lo >= c->sec_out_hi)
        return fail(LBM_E_INVALID, "bad pressure section");
    if (!(c->rho_out > 0.0) || !(c->rho_init > 0.0)) return fail(LBM_E_INVALID, "densities must be > 0");
    if (c->u_init_mode != 0 && c->u_init_mode != 1) return fail(LBM_E_INVALID, "u_init_mode must be 0 or 1");
    bool need_u = c->u_init_mode == 1;
    if (!c->periodic_x) {
        for (int face = 0; face < 2; ++face) {
            const int* k = face == 0 ? c->west : c->east;
            if (!k) continue;
            for (int y = 0; y < c->ny; ++y) {
                if (k[y] < LBM_WALL || k[y] > LBM_PRESSURE) return fail(LBM_E_INVALID, "bad row kind");
                if (face == 1 && k[y] == LBM_VELOCITY)
                    return fail(LBM_E_INVALID, "velocity rows are supported on the west face only");
                if (!c->periodic_y && (y == 0 || y == c->ny - 1) && k[y] != LBM_WALL)
                    return fail(LBM_E_INVALID, "rows touching a y wall must be WALL");
                if (k[y] == LBM_VELOCITY) need_u = true;
            }
        }
    }
    if (need_u) {
        if (!c->u_in) return fail(LBM_E_INVALID, "u_in is required");
        for (int y = 0; y < c->ny; ++y)
            if (!std::isfinite(c->u_in[y]) || std::fabs(c->u_in[y]) >= 0.5)
                return fail(LBM_E_INVALID, "u_in must be finite with |u0| < 0.5");
    }
    return LBM_OK;
}

void layout(const lbm_config* c, Layout& L) {
    L.Q = c->lattice == LBM_D2Q9 ? 9 : 19;
    L.D = c->lattice == LBM_D2Q9 ? 2 : 3;
    L.N = (long)c->nx * c->ny * c->nz;
    L.ss = c->prec == LBM_F64 ? 8 : (c->prec == LBM_F32 ? 4 : 2);
    L.cs = c->prec == LBM_F64 ? 8 : 4;
    L.as = L.cs;
    L.SB = align_up((size_t)L.Q * L.N * L.ss);
    L.R = c->window_len / c->ckpt_every;
    // a segment keeps the moment record (drho, j, Pi: 1 + D + D(D+1)/2
    // values per node) of every recomputed step and two states for the
    // recompute's ping-pong
    L.nseg = 2;
    L.nrec = c->ckpt_every < 2 ? 1 : c->ckpt_every - 1;
    L.RB = align_up((size_t)(c->lattice == LBM_D2Q9 ? 6 : 10) * L.N * L.cs);
    L.nblocks = blocks_for(L.N);
    L.pstride = 2 * L.nblocks + 64;      // partial slots per sample, for any launch grid
    L.nsamp = c->window_len / c->sample_every;
    size_t o = 0;
    L.off_G = o;       o += 2 * L.SB;
    L.off_ring = o;    o += 2 * (size_t)L.R * L.SB;
    L.off_seg = o;     o += (size_t)L.nseg * L.SB;
    L.off_rec = o;     o += (size_t)L.nrec * L.RB;
    L.off_s = o;       o += align_up(L.N * L.cs);
    L.off_srep = o;    o += align_up(L.N * L.cs);
    L.off_gamma = o;   o += align_up(L.N * 8);
    L.off_nu = o;      o += 2 * align_up((size_t)L.Q * L.N * L.as);   // >= Q N 8: FP64 staging
    L.off_sens = o;    o += align_up(L.N * 8);
    L.off_part = o;    o += 2 * align_up((size_t)L.nsamp * L.pstride * 3 * 8);
    L.off_samples = o; o += align_up((size_t)L.nsamp * 3 * 8);
    L.off_acc = o;     o += align_up(8 * 8);
    L.off_roww = o;    o += align_up(c->ny);
    L.off_rowe = o;    o += align_up(c->ny);
    L.off_uin = o;     o += align_up(c->ny * 8);
    // full history: the start state of every window and a ring for replays
    L.nstart = c->full_history ? c->max_windows : 0;
    L.off_starts = o;  o += (size_t)L.nstart * L.SB;
    L.off_ringrep = o; o += c->full_history ? (size_t)L.R * L.SB : 0;
    // window field of the drag (explicit dD/ds) or of the wake (u_bar)
    resolve_box(c, c->force_box, L.fbox);
    resolve_box(c, c->meas_box, L.mbox);
    const int* ab = c->objective == LBM_J_WAKE ? L.mbox : L.fbox;
    L.nb = (long)(ab[1] - ab[0]) * (ab[3] - ab[2]) * (ab[5] - ab[4]);
    L.ncomp = c->objective == LBM_J_DRAG ? 1 : (c->objective == LBM_J_WAKE ? L.D : 0);
    L.nf = L.ncomp * L.nb;
    L.off_facc = o;    o += L.ncomp ? 4 * align_up((size_t)L.nf * 8) + align_up(FACC_PARTS * 8) : 0;
    L.total = o;
}

// Timing of the hot kernels: one HIP event pair brackets each run of
// consecutive launches of one kernel class (forward step, adjoint step,
// recompute step), so the per-launch average includes the back-to-back
// dispatch gaps but no event overhead inside a run.
struct Timer {
    bool on = false;
    std::vector<hipEvent_t> ev;      // pool of start/stop pairs
    std::vector<int> cls;            // class of each closed or open run
    std::vector<long> cnt;           // launches in each run
    std::vector<long> steps;         // steps in each run
    int used = 0;                    // runs in the pool
    int open = -1;                   // class of the open run, -1 if none
    double n[4] = {0, 0, 0, 0}, ms[4] = {0, 0, 0, 0}, st[4] = {0, 0, 0, 0};
};

}  // namespace

struct lbm_ctx {
    lbm_config cfg;
    std::vector<int> west, east;
    std::vector<double> u_in;
    std::vector<signed char> roww, rowe;
    hipStream_t stream;
    Layout L;
    char* ws;
    void* G[2];
    std::vector<void*> ring[2];
    std::vector<void*> seg;
    std::vector<void*> recs;                // moment records of a recomputed D2Q9 segment
    std::vector<void*> starts, ring_rep;   // full history: window-start states, replay ring
    double* facc[3];                 // window-field accumulators (two forward, one replay)
    double *uref, *fparts;           // wake reference; wake-value block partials
    int fa, fw;                      // forward accumulator in use; last completed window's (-1: none)
    void *s, *s_rep, *nu[2];
    double *gamma, *sens, *partials[2], *samples, *acc;
    Geo geo;
    Phys ph;
    Obj ob;
    long step, base;
    int cur;
    std::vector<double> J, M, rel;
    std::vector<int> conv;
    bool unstable;
    int tb_steps, tile_x, tile_y;    // temporal blocking of forward launches (1 = off)
    int tile_z;                      // D3Q19 tiles are tile_x x tile_y x tile_z
    int rec_tile_x, rec_tile_y, rec_tile_z;  // D3Q19 tiles of the recompute's blocked launches
    int adj_steps, adj_tile_x, adj_tile_y;   // blocked adjoint launches (adj_steps 1 = off)
    int adj_tile_z;                          // D3Q19: z planes per workgroup
    Timer tm;
};

namespace {

void* at(lbm_ctx* c, size_t off) { return c->ws + off; }

lbm_status t_close(lbm_ctx* c) {
    if (!c->tm.on || c->tm.open < 0) return LBM_OK;
    HIPCHK(hipEventRecord(c->tm.ev[2 * (c->tm.used - 1) + 1], c->stream));
    c->tm.open = -1;
    return LBM_OK;
}

lbm_status t_drain(lbm_ctx* c) {
    if (!c->tm.on) return LBM_OK;
    lbm_status st = t_close(c);
    if (st != LBM_OK) return st;
    if (c->tm.used == 0) return LBM_OK;
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = 0; i < c->tm.used; ++i) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->tm.ev[2 * i], c->tm.ev[2 * i + 1]));
        c->tm.n[c->tm.cls[i]] += (double)c->tm.cnt[i];
        c->tm.st[c->tm.cls[i]] += (double)c->tm.steps[i];
        c->tm.ms[c->tm.cls[i]] += ms;
    }
    c->tm.used = 0;
    return LBM_OK;
}

// Called before each hot launch of class cls (advancing nsteps steps):
// extends the open run or starts a new one.
lbm_status t_launch(lbm_ctx* c, int cls, long nsteps = 1) {
    if (!c->tm.on) return LBM_OK;
    if (c->tm.open == cls) {
        c->tm.cnt[c->tm.used - 1] += 1;
        c->tm.steps[c->tm.used - 1] += nsteps;
        return LBM_OK;
    }
    lbm_status st = t_close(c);
    if (st != LBM_OK) return st;
    if (2 * c->tm.used + 2 > (int)c->tm.ev.size()) {
        if ((st = t_drain(c)) != LBM_OK) return st;
    }
    const int r = c->tm.used++;
    c->tm.cls[r] = cls;
    c->tm.cnt[r] = 1;
    c->tm.steps[r] = nsteps;
    c->tm.open = cls;
    HIPCHK(hipEventRecord(c->tm.ev[2 * r], c->stream));
    return LBM_OK;
}

StepLaunch step_args(lbm_ctx* c) {
    StepLaunch a;
    a.lattice = c->cfg.lattice;
    a.prec = c->cfg.prec;
    a.geo = c->geo;
    a.ph = c->ph;
    a.ob = c->ob;
    a.stream = c->stream;
    a.pre = nullptr;
    a.sample = 0;
    a.partials = nullptr;
    a.part_stride = (int)c->L.pstride;
    a.nsteps = 1;
    a.tile_x = c->tile_x;
    a.tile_y = c->tile_y;
    a.tile_z = c->tile_z;
    a.rec = nullptr;
    a.rec_slot = 0;
    return a;
}

AuxLaunch aux_args(lbm_ctx* c, int op) {
    AuxLaunch a;
    a.lattice = c->cfg.lattice;
    a.prec = c->cfg.prec;
    a.op = op;
    a.src = nullptr;
    a.dst = nullptr;
    a.s = c->s;
    a.rho0 = c->cfg.rho_init;
    a.umode = c->cfg.u_init_mode;
    a.map = c->cfg.s_map;
    a.q = c->cfg.s_q;
    a.geo = c->geo;
    a.ph = c->ph;
    a.stream = c->stream;
    return a;
}

// Ring slot holding the checkpoint written by step m (m % K == 0).
void* ring_slot_for_step(lbm_ctx* c, long m) {
    const long W = c->cfg.window_len;
    const int p = (int)(((m / W) + 1) % 2);
    const int slot = (int)((m % W) / c->cfg.ckpt_every);
    return c->ring[p][slot];
}

lbm_status apply_design(lbm_ctx* c, const double* gamma_src, void* s_dst) {
    AuxLaunch a = aux_args(c, AUX_DESIGN);
    a.src = gamma_src;
    a.dst = s_dst;
    HIPCHK(launch_aux(a));
    return LBM_OK;
}

lbm_status check_gamma(lbm_ctx* c, const double* gamma_dev) {
    std::vector<double> h(c->L.N);
    HIPCHK(hipMemcpyAsync(h.data(), gamma_dev, c->L.N * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (long i = 0; i < c->L.N; ++i)
        if (!std::isfinite(h[i])) return fail(LBM_E_INVALID, "gamma has a non-finite entry");
    if (c->cfg.s_map == LBM_S_PAPER)
        for (long i = 0; i < c->L.N; ++i)
            if (!(1.0 - h[i] + c->cfg.s_q > 0.0)) return fail(LBM_E_INVALID, "gamma out of range of the paper map");
    return LBM_OK;
}

// Loads a pre-collision state (already in the checkpoint slot of step k)
// and makes G^k from it.
lbm_status start_from_slot(lbm_ctx* c, long k) {
    AuxLaunch a = aux_args(c, AUX_COLLIDE);
    a.src = ring_slot_for_step(c, k);
    a.dst = c->G[0];
    HIPCHK(launch_aux(a));
    if (!c->starts.empty()) HIPCHK(launch_copy(a.src, c->starts[0], c->L.SB, c->stream));
    if (c->L.ncomp) HIPCHK(launch_fill(c->facc[0], c->L.nf, 0.0, c->stream));
    c->fa = 0;
    c->fw = -1;
    c->cur = 0;
    c->step = k;
    c->base = k;
    c->J.clear();
    c->M.clear();
    c->rel.clear();
    c->conv.clear();
    c->unstable = false;
    return LBM_OK;
}

lbm_status do_reset(lbm_ctx* c) {
    AuxLaunch a = aux_args(c, AUX_INIT_EQ);
    a.dst = ring_slot_for_step(c, 0);
    HIPCHK(launch_aux(a));
    return start_from_slot(c, 0);
}

// Window sums of the samples into accbuf[0..2] and to the host; for the
// wake objective the window value comes from the accumulated u_bar (wake).
lbm_status window_end(lbm_ctx* c, double* accbuf, double* part, double out[3], const double* wake = nullptr) {
    const Layout& L = c->L;
    const double wgt = (double)c->cfg.sample_every / c->cfg.window_len;
    HIPCHK(launch_reduce(part, L.pstride, L.nsamp, c->samples, wgt, accbuf, c->stream));
    if (wake) HIPCHK(launch_sq_diff_sum(wake, c->uref, L.nf, c->fparts, FACC_PARTS, accbuf, c->stream));
    HIPCHK(hipMemcpyAsync(out, accbuf, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// Consecutive-window test (Eq. statistical_criterion), strict inequality;
// a zero current mean passes only if the previous one is zero too.
void criterion(double prev, double cur, double eps, double& rel, int& conv) {
    if (cur == 0.0) {
        rel = prev == 0.0 ? 0.0 : INFINITY;
        conv = (prev == 0.0 && eps >= 0.0) ? 1 : 0;
        return;
    }
    rel = std::fabs((cur - prev) / cur);
    conv = (eps >= 0.0 && rel < eps) ? 1 : 0;
}

long gcd_l(long a, long b) {
    while (b) {
        const long t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Steps of the next forward launch from `step`: a temporally blocked launch
// of up to tb_steps steps that ends no later than the next event step (a
// multiple of gev: sample, checkpoint or window end), else one step. Events
// therefore only fall on the last step of a launch. With `reserve`, the
// step that ends a window (a multiple of W) or the budget is always a
// single-step launch, so that the buffer not holding G^k holds G^{k-1},
// from which the post-boundary state f^k is exported.
long plan_launch(lbm_ctx* c, long step, long gev, long W, long budget, bool reserve) {
    const long nt = c->tb_steps;
    if (nt <= 1 || budget <= 1) return 1;
    long lim = gev - (step % gev);
    if (lim > budget) lim = budget;
    if (reserve && (lim == budget || (step + lim) % W == 0)) lim -= 1;
    const long n = lim < nt ? lim : nt;
    return n >= 2 ? n : 1;
}

long last_window(lbm_ctx* c) {
    const long W = c->cfg.window_len;
    const long g = c->step / W;
    return g > c->base / W ? g : 0;
}

// The blocked adjoint keeps FP32/FP64 populations and an FP64 sensitivity
// plane in LDS. Measured on MI355X: on grids of more than 400k nodes 4 steps
// on 25 x 25 tiles (FP64) or 5 steps on 48 x 24 (FP32 populations) are the
// fastest; on smaller grids the forward's tiles. If the first choice does
// not fit, the first of a few tiles that allows two or more steps, with as
// many steps (up to the first choice's) as the LDS allows.
lbm_status default_adj_blocking(lbm_ctx* c, int nsteps, int tile_x, int tile_y) {
    c->adj_steps = 1;
    c->adj_tile_x = tile_x;
    c->adj_tile_y = tile_y;
    if (nsteps > 1 && c->cfg.lattice == LBM_D2Q9) {
        int nfirst = nsteps;
        if (c->L.N > 400000) {
            nfirst = c->cfg.prec == LBM_F64 ? 4 : 5;
            tile_x = c->cfg.prec == LBM_F64 ? 25 : 48;
            tile_y = c->cfg.prec == LBM_F64 ? 25 : 24;
        }
        const int cand[6][2] = {{tile_x, tile_y}, {48, 24}, {64, 16}, {32, 32}, {32, 16}, {16, 16}};
        for (const auto& t : cand) {
            int na = nfirst;
            while (na > 1 && adj_tb_lds_bytes(na, t[0], t[1], c->L.cs) > TB_LDS_MAX) --na;
            if (na >= 2 && tb_blocks(c->cfg.nx, c->cfg.ny, t[0], t[1]) <= c->L.pstride) {
                c->adj_steps = na;
                c->adj_tile_x = t[0];
                c->adj_tile_y = t[1];
                break;
            }
        }
    }
    return LBM_OK;
}

lbm_status set_blocking(lbm_ctx* c, int nsteps, int tile_x, int tile_y) {
    if (nsteps < 1 || nsteps > 16) return fail(LBM_E_INVALID, "nsteps must be in [1, 16]");
    if (nsteps > 1 && c->cfg.lattice != LBM_D2Q9) return fail(LBM_E_INVALID, "temporal blocking is D2Q9 only");
    if (nsteps > 1) {
        if (tile_x < 1 || tile_y < 1 || (long)tile_x * tile_y < 256)
            return fail(LBM_E_INVALID, "tile must hold at least 256 nodes");
        const size_t lds = tb_lds_bytes_prec(nsteps, tile_x, tile_y, c->cfg.prec);
        if (lds > TB_LDS_MAX) return fail(LBM_E_INVALID, "tile and nsteps need more than 159 KB of LDS");
        if (tb_blocks(c->cfg.nx, c->cfg.ny, tile_x, tile_y) > c->L.pstride)
            return fail(LBM_E_INVALID, "too many tiles");
        HIPCHK(tb_prepare(c->cfg.prec));
        c->tile_x = tile_x;
        c->tile_y = tile_y;
    }
    c->tb_steps = nsteps;
    return default_adj_blocking(c, nsteps, tile_x, tile_y);
}

lbm_status set_blocking_3d(lbm_ctx* c, int nsteps, int tile_x, int tile_y, int tile_z) {
    if (c->cfg.lattice != LBM_D3Q19) return fail(LBM_E_INVALID, "3D blocking needs the D3Q19 lattice");
    if (nsteps != 1 && nsteps != 2) return fail(LBM_E_INVALID, "D3Q19 blocking takes 1 or 2 steps");
    if (nsteps == 2) {
        if (tile_x < 1 || tile_y < 1 || tile_z < 1 || (long)tile_x * tile_y * tile_z < 256)
            return fail(LBM_E_INVALID, "tile must hold at least 256 nodes");
        if ((long)(tile_x + 2) * (tile_y + 2) > 1024)
            return fail(LBM_E_INVALID, "(tile_x + 2) * (tile_y + 2) must be at most 1024");
        if (tbz_lds_bytes_prec(tile_x, tile_y, c->cfg.prec) > TB_LDS_MAX)
            return fail(LBM_E_INVALID, "tile needs more than 159 KB of LDS");
        // the blocked kernel addresses a state and a moment record with
        // 32-bit byte offsets
        if ((size_t)c->L.Q * c->L.N * c->L.ss > TBZ_STATE_MAX || (size_t)10 * c->L.N * c->L.cs > TBZ_STATE_MAX)
            return fail(LBM_E_INVALID, "state too large for D3Q19 blocking (limit 4 GB)");
        const long tiles = (long)((c->cfg.nx + tile_x - 1) / tile_x) * ((c->cfg.ny + tile_y - 1) / tile_y) *
                           ((c->cfg.nz + tile_z - 1) / tile_z);
        if (tiles > c->L.pstride) return fail(LBM_E_INVALID, "too many tiles");
        HIPCHK(tb_prepare(c->cfg.prec));
        c->tile_x = c->rec_tile_x = tile_x;
        c->tile_y = c->rec_tile_y = tile_y;
        c->tile_z = c->rec_tile_z = tile_z;
    }
    c->tb_steps = nsteps;
    return LBM_OK;
}

lbm_status set_adj_blocking_3d(lbm_ctx* c, int nsteps, int tile_x, int tile_y, int tile_z) {
    if (c->cfg.lattice != LBM_D3Q19) return fail(LBM_E_INVALID, "3D blocking needs the D3Q19 lattice");
    if (nsteps != 1 && nsteps != 2) return fail(LBM_E_INVALID, "D3Q19 adjoint blocking takes 1 or 2 steps");
    if (nsteps == 2) {
        if (tile_x < 1 || tile_y < 1 || tile_z < 1 || (long)tile_x * tile_y * tile_z < 256)
            return fail(LBM_E_INVALID, "tile must hold at least 256 nodes");
        // one cell per thread, at most 768 threads (registers); FP64 regions
        // are further bounded by the LDS (about 430 cells)
        if ((long)(tile_x + 2) * (tile_y + 2) > 768)
            return fail(LBM_E_INVALID, "(tile_x + 2) * (tile_y + 2) must be at most 768");
        if (adj_tbz_lds_bytes(tile_x, tile_y, c->L.as, c->L.cs) > TB_LDS_MAX)
            return fail(LBM_E_INVALID, "tile needs more than 159 KB of LDS");
        if ((size_t)10 * c->L.N * c->L.cs > TBZ_STATE_MAX || (size_t)c->L.Q * c->L.N * c->L.as > TBZ_STATE_MAX)
            return fail(LBM_E_INVALID, "state too large for D3Q19 blocking (limit 4 GB)");
        HIPCHK(tb_prepare(c->cfg.prec));
        c->adj_tile_x = tile_x;
        c->adj_tile_y = tile_y;
        c->adj_tile_z = tile_z;
    }
    c->adj_steps = nsteps;
    return LBM_OK;
}

// z-run length of a D3Q19 blocked launch on tile_x x tile_y tiles: the run
// count c maximises E * oz / (oz + 2), where E is the fraction of the
// compute units' rounds that the tiles x c blocks fill (one block per
// compute unit) and (oz + 2) / oz the cost of the halo planes of a run of
// oz planes (step 1 computes oz + 2 planes, the loads span oz + 4). Measured
// on MI355X on the 384 x 128 x 128 channel this picks the fastest run of the
// FP32 and FP64 forward and adjoint defaults.
static int compute_units() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    return cus;
}

static int default_z_run(lbm_ctx* c, int tile_x, int tile_y) {
    const int cus = compute_units();
    const long tiles = (long)((c->cfg.nx + tile_x - 1) / tile_x) * ((c->cfg.ny + tile_y - 1) / tile_y);
    const int nz = c->cfg.nz;
    int best = nz;
    double best_score = -1.0;
    for (int runs = 1; runs <= nz; ++runs) {
        const int oz = (nz + runs - 1) / runs;
        if ((long)tile_x * tile_y * oz < 256) break;
        const long blocks = tiles * ((nz + oz - 1) / oz);
        if (blocks > c->L.pstride) continue;
        const long rounds = (blocks + cus - 1) / cus;
        const double score = (double)blocks / ((double)rounds * cus) * oz / (oz + 2.0);
        if (score > best_score + 1e-9) {
            best_score = score;
            best = oz;
        }
    }
    return best;
}

lbm_status set_adj_blocking(lbm_ctx* c, int nsteps, int tile_x, int tile_y) {
    if (nsteps < 1 || nsteps > 16) return fail(LBM_E_INVALID, "nsteps must be in [1, 16]");
    if (nsteps > 1) {
        if (c->cfg.lattice != LBM_D2Q9) return fail(LBM_E_INVALID, "temporal blocking is D2Q9 only");
        if (tile_x < 1 || tile_y < 1 || (long)tile_x * tile_y < 256)
            return fail(LBM_E_INVALID, "tile must hold at least 256 nodes");
        if (adj_tb_lds_bytes(nsteps, tile_x, tile_y, c->L.cs) > TB_LDS_MAX)
            return fail(LBM_E_INVALID, "tile and nsteps need more than 159 KB of LDS");
        if (tb_blocks(c->cfg.nx, c->cfg.ny, tile_x, tile_y) > c->L.pstride)
            return fail(LBM_E_INVALID, "too many tiles");
        HIPCHK(tb_prepare(c->cfg.prec));
        c->adj_tile_x = tile_x;
        c->adj_tile_y = tile_y;
    }
    c->adj_steps = nsteps;
    return LBM_OK;
}

// Reverse sweep over one window whose first step is ns: transitions n_e down
// to n_s, each K-step segment restarted from ring[seg] (its pre-collision
// checkpoint) and recomputed into the seg slots. objective_window: the
// window of the objective, which starts from the terminal condition and adds the sampled
// objective source; otherwise the sweep continues from c->nu[cur] (the
// adjoint of the next window's start state) with no source.
lbm_status adjoint_window(lbm_ctx* c, const std::vector<void*>& ring, long ns, bool objective_window, int& cur) {
    const long W = c->cfg.window_len, dW = c->cfg.sample_every, K = c->cfg.ckpt_every;
    const Layout& L = c->L;
    const double wgt = objective_window ? (double)dW / W : 0.0;
    lbm_status st;
    StepLaunch sa = step_args(c);
    sa.s = c->s;
    if (c->cfg.lattice == LBM_D3Q19) {
        sa.tile_x = c->rec_tile_x;
        sa.tile_y = c->rec_tile_y;
        sa.tile_z = c->rec_tile_z;
    }
    AdjLaunch aa;
    aa.lattice = c->cfg.lattice;
    aa.prec = c->cfg.prec;
    aa.s = c->s;
    aa.sens = c->sens;
    aa.geo = c->geo;
    aa.ph = c->ph;
    aa.ob = c->ob;
    aa.ob.fwin = c->fw >= 0 ? c->facc[c->fw] : nullptr;
    aa.stream = c->stream;
    aa.nsteps = 1;
    aa.tile_x = c->adj_tile_x;
    aa.tile_y = c->adj_tile_y;
    aa.tile_z = c->adj_tile_z;
    aa.gseg = c->seg[0];
    aa.slot = L.SB;
    aa.ns = ns;
    aa.dW = dW;
    aa.wgt = wgt;
    aa.rec = 0;
    for (int seg = L.R - 1; seg >= 0; --seg) {
        const long c0 = ns - 1 + (long)seg * K;       // checkpoint step
        aa.kseg = c0;
        const bool last = seg == L.R - 1;
        const bool seed = last && objective_window;
        // recompute G^{c0+1} .. G^{c0+K-1} through two state slots, keeping
        // the moment record R^m of every pre-collision state f^m,
        // m = c0+1 .. c0+K-1, in recs[m - c0 - 1]: the pre-states of
        // transitions c0+2 .. c0+K
        int gc = 0;
        if (seed || K >= 2) {
            AuxLaunch ca = aux_args(c, AUX_COLLIDE);
            ca.src = ring[seg];
            ca.dst = c->seg[0];
            HIPCHK(launch_aux(ca));
            const long nrec = K - 1;
            for (long j = 1; j <= nrec;) {
                long n = nrec - j + 1;
                if (n > c->tb_steps) n = c->tb_steps;
                sa.nsteps = (int)n;
                sa.gin = c->seg[gc];
                sa.gout = c->seg[gc ^ 1];
                sa.rec = c->recs[j - 1];
                sa.rec_slot = L.RB;
                if ((st = t_launch(c, 2, n)) != LBM_OK) return st;
                HIPCHK(launch_step(sa));
                gc ^= 1;
                j += n;
            }
            sa.rec = nullptr;
            sa.nsteps = 1;
            if ((st = t_close(c)) != LBM_OK) return st;
        }
        if (seed) {
            // terminal condition: nu_hat^{n_e} = BC^T (dJ/df^{n_e}), f^{n_e} = BC(S(G^{n_e - 1}))
            aa.nu_in = nullptr;
            aa.nu_out = c->nu[cur];
            aa.state = c->seg[gc];
            aa.direct = 0;
            aa.rec = 0;
            aa.seed = 1;
            aa.src_w = wgt;
            HIPCHK(launch_adjoint(aa));
        }
        for (long k = c0 + K; k >= c0 + 1;) {
            aa.nu_in = c->nu[cur];
            aa.nu_out = c->nu[cur ^ 1];
            aa.seed = 0;
            aa.nsteps = 1;
            long n = 1;
            if (k - 1 == c0) {
                aa.direct = 1;
                aa.rec = 0;
                aa.state = ring[seg];
            } else {
                // transitions k .. c0 + 2 read the records of their pre-states
                aa.direct = 0;
                aa.rec = 1;
                aa.state = c->recs[k - 2 - c0];
                aa.gseg = c->recs[0];
                aa.slot = L.RB;
                n = k - (c0 + 1);
                if (n > c->adj_steps) n = c->adj_steps;
                if (n > 1) {
                    aa.nsteps = (int)n;
                    aa.k_hi = k;
                }
            }
            aa.src_w = (k > ns && (k - ns) % dW == 0) ? wgt : 0.0;
            if ((st = t_launch(c, 1, n)) != LBM_OK) return st;
            HIPCHK(launch_adjoint(aa));
            cur ^= 1;
            k -= n;
        }
        aa.rec = 0;
        if ((st = t_close(c)) != LBM_OK) return st;
    }
    return LBM_OK;
}

}  // namespace

// Error recording shared with the design-update entry points.
lbm_status lbm::record_error(lbm_status st, const char* msg) { return fail(st, msg); }

extern "C" {

lbm_status lbm_set_blocking(lbm_ctx* c, int nsteps, int tile_x, int tile_y) {
    if (!c) return fail(LBM_E_INVALID, "NULL context");
    return set_blocking(c, nsteps, tile_x, tile_y);
}

lbm_status lbm_set_blocking_3d(lbm_ctx* c, int nsteps, int tile_x, int tile_y, int tile_z) {
    if (!c) return fail(LBM_E_INVALID, "NULL context");
    return set_blocking_3d(c, nsteps, tile_x, tile_y, tile_z);
}

lbm_status lbm_set_adjoint_blocking(lbm_ctx* c, int nsteps, int tile_x, int tile_y) {
    if (!c) return fail(LBM_E_INVALID, "NULL context");
    return set_adj_blocking(c, nsteps, tile_x, tile_y);
}

lbm_status lbm_set_adjoint_blocking_3d(lbm_ctx* c, int nsteps, int tile_x, int tile_y, int tile_z) {
    if (!c) return fail(LBM_E_INVALID, "NULL context");
    return set_adj_blocking_3d(c, nsteps, tile_x, tile_y, tile_z);
}


lbm_status lbm_workspace_bytes(const lbm_config* cfg, size_t* bytes) {
    lbm_status st = validate(cfg);
    if (st != LBM_OK) return st;
    if (!bytes) return fail(LBM_E_INVALID, "bytes is NULL");
    Layout L;
    layout(cfg, L);
    *bytes = L.total;
    return LBM_OK;
}

lbm_status lbm_init(const lbm_config* cfg, const double* gamma_dev, void* workspace_dev, size_t bytes,
                    void* stream, lbm_ctx** out) {
    lbm_status st = validate(cfg);
    if (st != LBM_OK) return st;
    if (!out || !gamma_dev || !workspace_dev) return fail(LBM_E_INVALID, "NULL argument");
    if ((uintptr_t)workspace_dev % ALIGN != 0) return fail(LBM_E_INVALID, "workspace must be 256-byte aligned");
    Layout L;
    layout(cfg, L);
    if (bytes < L.total) return fail(LBM_E_NOMEM, "workspace smaller than lbm_workspace_bytes");
    lbm_ctx* c = new lbm_ctx();
    c->cfg = *cfg;
    c->L = L;
    c->stream = (hipStream_t)stream;
    const int ny = cfg->ny;
    c->west.assign(ny, LBM_WALL);
    c->east.assign(ny, LBM_WALL);
    c->u_in.assign(ny, 0.0);
    if (!cfg->periodic_x) {
        if (cfg->west) c->west.assign(cfg->west, cfg->west + ny);
        if (cfg->east) c->east.assign(cfg->east, cfg->east + ny);
    }
    if (cfg->u_in) c->u_in.assign(cfg->u_in, cfg->u_in + ny);
    c->cfg.west = c->cfg.east = nullptr;
    c->cfg.u_in = nullptr;
    c->roww.resize(ny);
    c->rowe.resize(ny);
    for (int y = 0; y < ny; ++y) {
        c->roww[y] = (signed char)c->west[y];
        c->rowe[y] = (signed char)c->east[y];
    }
    c->ws = (char*)workspace_dev;
    c->G[0] = at(c, L.off_G);
    c->G[1] = at(c, L.off_G + L.SB);
    for (int p = 0; p < 2; ++p)
        for (int r = 0; r < L.R; ++r) c->ring[p].push_back(at(c, L.off_ring + ((size_t)p * L.R + r) * L.SB));
    for (int k = 0; k < L.nseg; ++k) c->seg.push_back(at(c, L.off_seg + (size_t)k * L.SB));
    for (int k = 0; k < L.nrec; ++k) c->recs.push_back(at(c, L.off_rec + (size_t)k * L.RB));
    for (int k = 0; k < L.nstart; ++k) c->starts.push_back(at(c, L.off_starts + (size_t)k * L.SB));
    if (cfg->full_history)
        for (int r = 0; r < L.R; ++r) c->ring_rep.push_back(at(c, L.off_ringrep + (size_t)r * L.SB));
    c->s = at(c, L.off_s);
    c->s_rep = at(c, L.off_srep);
    c->gamma = (double*)at(c, L.off_gamma);
    const size_t nub = align_up((size_t)L.Q * L.N * L.as);
    c->nu[0] = at(c, L.off_nu);
    c->nu[1] = at(c, L.off_nu + nub);
    c->sens = (double*)at(c, L.off_sens);
    const size_t pb = align_up((size_t)L.nsamp * L.pstride * 3 * 8);
    c->partials[0] = (double*)at(c, L.off_part);
    c->partials[1] = (double*)at(c, L.off_part + pb);
    c->samples = (double*)at(c, L.off_samples);
    c->acc = (double*)at(c, L.off_acc);
    signed char* dw = (signed char*)at(c, L.off_roww);
    signed char* de = (signed char*)at(c, L.off_rowe);
    double* du = (double*)at(c, L.off_uin);

    c->geo.nx = cfg->nx;
    c->geo.ny = cfg->ny;
    c->geo.nz = cfg->nz;
    c->geo.N = (int)L.N;
    c->geo.inv_nx = 1.0 / cfg->nx;
    c->geo.inv_ny = 1.0 / cfg->ny;
    c->geo.per_x = cfg->periodic_x ? 1 : 0;
    c->geo.per_y = cfg->periodic_y ? 1 : 0;
    c->geo.per_z = cfg->periodic_z ? 1 : 0;
    c->geo.west = dw;
    c->geo.east = de;
    c->geo.u_in = du;
    c->geo.drho_out = cfg->rho_out - 1.0;
    c->ph.tau = cfg->tau;
    c->ph.c2 = cfg->c_smag * cfg->c_smag;
    c->ob.obj = cfg->objective;
    c->ob.mon = cfg->monitor;
    c->ob.in_x = cfg->sec_in_x;
    c->ob.in_lo = cfg->sec_in_lo;
    c->ob.in_hi = cfg->sec_in_hi;
    c->ob.out_x = cfg->sec_out_x;
    c->ob.out_lo = cfg->sec_out_lo;
    c->ob.out_hi = cfg->sec_out_hi;
    c->ob.inv_nin = 1.0 / ((double)(cfg->sec_in_hi - cfg->sec_in_lo) * cfg->nz);
    c->ob.inv_nout = 1.0 / ((double)(cfg->sec_out_hi - cfg->sec_out_lo) * cfg->nz);
    c->ob.fx0 = L.fbox[0];
    c->ob.fx1 = L.fbox[1];
    c->ob.fy0 = L.fbox[2];
    c->ob.fy1 = L.fbox[3];
    c->ob.fz0 = L.fbox[4];
    c->ob.fz1 = L.fbox[5];
    c->ob.inv_dref = cfg->monitor == LBM_J_DRAG ? 1.0 / cfg->drag_ref : 0.0;
    {
        const int* ab = cfg->objective == LBM_J_WAKE ? L.mbox : L.fbox;
        c->ob.ax0 = ab[0];
        c->ob.ay0 = ab[2];
        c->ob.az0 = ab[4];
        c->ob.anx = ab[1] - ab[0];
        c->ob.any = ab[3] - ab[2];
        c->ob.anz = ab[5] - ab[4];
        c->ob.nb = (int)L.nb;
    }
    c->ob.wgt = (double)cfg->sample_every / cfg->window_len;
    c->ob.facc = nullptr;
    c->ob.fwin = nullptr;
    c->ob.uref = nullptr;
    c->facc[0] = c->facc[1] = c->facc[2] = nullptr;
    c->uref = c->fparts = nullptr;
    c->fa = 0;
    c->fw = -1;
    if (L.ncomp) {
        const size_t fb = align_up((size_t)L.nf * 8);
        for (int k = 0; k < 3; ++k) c->facc[k] = (double*)at(c, L.off_facc + k * fb);
        c->uref = (double*)at(c, L.off_facc + 3 * fb);
        c->fparts = (double*)at(c, L.off_facc + 4 * fb);
        c->ob.uref = c->uref;
    }
    c->step = c->base = 0;
    c->cur = 0;
    c->unstable = false;
    c->tb_steps = 1;
    c->adj_steps = 1;
    c->adj_tile_x = 32;
    c->adj_tile_y = 16;
    c->adj_tile_z = 8;
    c->tile_x = c->rec_tile_x = 32;
    c->tile_y = c->rec_tile_y = 16;
    c->tile_z = c->rec_tile_z = 8;

    auto bail = [&](lbm_status s2) {
        std::string keep = g_err;
        delete c;
        g_err = keep;
        return s2;
    };
#define INITCHK(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            fail(LBM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));               \
            return bail(LBM_E_HIP);                                                            \
        }                                                                                      \
    } while (0)
    INITCHK(hipMemcpyAsync(dw, c->roww.data(), ny, hipMemcpyHostToDevice, c->stream));
    INITCHK(hipMemcpyAsync(de, c->rowe.data(), ny, hipMemcpyHostToDevice, c->stream));
    INITCHK(hipMemcpyAsync(du, c->u_in.data(), ny * 8, hipMemcpyHostToDevice, c->stream));
    INITCHK(hipMemcpyAsync(c->gamma, gamma_dev, L.N * 8, hipMemcpyDeviceToDevice, c->stream));
    if (L.ncomp) INITCHK(launch_fill(c->uref, L.nf, 0.0, c->stream));
    INITCHK(hipStreamSynchronize(c->stream));
#undef INITCHK
    if ((st = check_gamma(c, c->gamma)) != LBM_OK) return bail(st);
    if ((st = apply_design(c, c->gamma, c->s)) != LBM_OK) return bail(st);
    if ((st = do_reset(c)) != LBM_OK) return bail(st);
    if (cfg->lattice == LBM_D2Q9) {
        // default temporal blocking of forward launches, from measurements on
        // MI355X. Small grids are latency-bound: one tile per compute unit
        // (about N / 256 nodes, at least 16 x 16) and long blocks amortise
        // the fixed cost of a launch. On large grids the halo recomputation
        // makes the blocked kernel ALU-bound and wide, shorter blocks win.
        int nt, tx, ty;
        if (L.N <= 400000) {
            int t = (int)std::lround(std::sqrt((double)L.N / 256.0));
            t = t < 16 ? 16 : (t > 25 ? 25 : t);
            tx = ty = t;
            // FP64 on the smallest tiles: 8 steps (measured 23-26% faster
            // than 4 on the 200 x 100 and 160 x 64 cylinders)
            nt = cfg->prec == LBM_F64 ? (t == 16 ? 8 : 4) : 10;
            while (nt > 2 && tb_lds_bytes_prec(nt, tx, ty, cfg->prec) > TB_LDS_MAX) --nt;
        } else if (cfg->prec == LBM_F32) {
            nt = 6;
            tx = 64;
            ty = 16;
        } else if (cfg->prec == LBM_F64) {
            nt = 2;
            tx = 32;
            ty = 8;
        } else if (L.N < 4000000) {
            // FP16 LDS state: larger tiles
            nt = 6;
            tx = ty = 48;
        } else {
            nt = 5;
            tx = 64;
            ty = 40;
        }
        if ((st = set_blocking(c, nt, tx, ty)) != LBM_OK) return bail(st);
    } else if (cfg->prec == LBM_F32 && L.N > 2000000 && cfg->nx >= 32 && cfg->ny >= 13 &&
               (size_t)L.Q * L.N * L.ss <= TBZ_STATE_MAX) {
        // D3Q19 FP32 on large grids: two steps per launch on 48 x 16 tiles
        // (a 900-cell region in one compute unit's LDS, 1024 threads; 32 x 19
        // with 768 threads on grids narrower than 48 or lower than 16), z runs
        // as long as possible while the blocks still fill the compute units in
        // nearly whole rounds (measured on MI355X on the 384 x 128 x 128
        // channel: 124.9 us per step on 48 x 16 in runs of 32 planes, 131.8 on
        // 48 x 13 and 140.1 on 32 x 19 with 768 threads). FP16S stays single
        // steps: its blocked launches measured no faster (113.9 against 109.6
        // us per step on that channel).
        const int ftx = (cfg->nx >= 48 && cfg->ny >= 16) ? 48 : 32, fty = ftx == 48 ? 16 : 19;
        if ((st = set_blocking_3d(c, 2, ftx, fty, default_z_run(c, ftx, fty))) != LBM_OK) return bail(st);
        // the recompute (the same kernel storing the moment records of both
        // steps) runs faster on 32 x 19 tiles with 768 threads: 196.8 against
        // 206.2 us per step on that channel
        c->rec_tile_x = 32;
        c->rec_tile_y = 19;
        c->rec_tile_z = default_z_run(c, 32, 19);
    } else if (cfg->prec == LBM_F64 && L.N > 2000000 && cfg->nx >= 32 && cfg->ny >= 7 &&
               (size_t)L.Q * L.N * L.ss <= TBZ_STATE_MAX) {
        // D3Q19 FP64 on large grids: two steps per launch on 48 x 7 tiles (a
        // 450-cell region, the most the LDS holds in FP64; 512 threads; 32 x 10
        // on grids narrower than 48). Measured on MI355X on the 384 x 128 x
        // 128 channel: 271 us per step in runs of 26 planes against 379 for
        // single steps (40 x 8: 284, 32 x 10: 291, 24 x 14: 306).
        const int ftx = cfg->nx >= 48 ? 48 : 32, fty = ftx == 48 ? 7 : 10;
        if ((st = set_blocking_3d(c, 2, ftx, fty, default_z_run(c, ftx, fty))) != LBM_OK) return bail(st);
    }
    if (cfg->lattice == LBM_D3Q19 && L.N > 2000000 && cfg->nx >= 32 && cfg->ny >= (cfg->prec == LBM_F64 ? 8 : 13) &&
        (size_t)10 * L.N * L.cs <= TBZ_STATE_MAX && (size_t)L.Q * L.N * L.as <= TBZ_STATE_MAX) {
        // D3Q19 adjoint on large grids: two reverse steps per launch, z runs
        // chosen as for the forward. FP32 adjoint populations (FP32 and FP16S
        // storage): 768 threads on 48 x 13 tiles (32 x 19 on grids narrower
        // than 48); measured on MI355X on the 384 x 128 x 128
        // channel, FP32: 212 us per reverse step on 48 x 13, 219 on 32 x 19,
        // 230 on the 512-thread 48 x 8 tiles and 238 on 32 x 13. FP64: 512
        // threads on 40 x 8 tiles (a 420-cell region; 32 x 10 on grids
        // narrower than 40): 416 us per reverse step against 484 for single
        // steps (32 x 10: 426, 24 x 14: 447, 256-thread 14 x 14: 603).
        int atx, aty;
        if (cfg->prec == LBM_F64) {
            atx = cfg->nx >= 40 ? 40 : 32;
            aty = atx == 40 ? 8 : 10;
        } else {
            atx = cfg->nx >= 48 ? 48 : 32;
            aty = atx == 48 ? 13 : 19;
        }
        const int aoz = default_z_run(c, atx, aty);
        if ((st = set_adj_blocking_3d(c, 2, atx, aty, aoz)) != LBM_OK) return bail(st);
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        fail(LBM_E_HIP, std::string("init: ") + hipGetErrorString(e));
        return bail(LBM_E_HIP);
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_set_gamma(lbm_ctx* c, const double* gamma_dev) {
    if (!c || !gamma_dev) return fail(LBM_E_INVALID, "NULL argument");
    lbm_status st = check_gamma(c, gamma_dev);
    if (st != LBM_OK) return st;
    HIPCHK(hipMemcpyAsync(c->gamma, gamma_dev, c->L.N * 8, hipMemcpyDeviceToDevice, c->stream));
    if ((st = apply_design(c, c->gamma, c->s)) != LBM_OK) return st;
    if ((st = do_reset(c)) != LBM_OK) return st;
    HIPCHK(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_reset(lbm_ctx* c) {
    if (!c) return fail(LBM_E_INVALID, "NULL context");
    lbm_status st = do_reset(c);
    if (st != LBM_OK) return st;
    HIPCHK(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_forward(lbm_ctx* c, long n_steps, int stop_on_converge, lbm_fwd_report* rep) {
    if (!c) return fail(LBM_E_INVALID, "NULL context");
    if (n_steps < 0) return fail(LBM_E_INVALID, "n_steps < 0");
    if (c->unstable) return fail(LBM_E_STATE, "state is unstable; reset, set_gamma or set_state first");
    const long W = c->cfg.window_len, dW = c->cfg.sample_every, K = c->cfg.ckpt_every;
    const Layout& L = c->L;
    lbm_status st;
    StepLaunch a = step_args(c);
    a.s = c->s;
    const long gev = gcd_l(dW, K);             // samples, checkpoints and window ends fall on multiples
    long done = 0;
    while (done < n_steps) {
        const long n = plan_launch(c, c->step, gev, W, n_steps - done, true);
        const long m = c->step + n;            // last step of this launch
        const long mw = m % W;
        a.nsteps = (int)n;
        a.gin = c->G[c->cur];
        a.gout = c->G[c->cur ^ 1];
        a.pre = (m % K == 0) ? ring_slot_for_step(c, m) : nullptr;
        a.sample = (m % dW == 0) ? 1 : 0;
        if (a.sample) {
            const long js = (mw == 0 ? W : mw) / dW - 1;
            a.partials = c->partials[0] + js * L.pstride * 3;
        }
        a.ob.facc = L.ncomp ? c->facc[c->fa] : nullptr;
        if ((st = t_launch(c, n > 1 ? 3 : 0, n)) != LBM_OK) return st;
        HIPCHK(launch_step(a));
        if (mw == 0 && !c->starts.empty()) {
            // full history: the start state of the next window
            const long r = (m - c->base) / W;
            if (r < (long)c->starts.size()) HIPCHK(launch_copy(a.pre, c->starts[r], L.SB, c->stream));
        }
        c->cur ^= 1;
        c->step = m;
        done += n;
        if (mw == 0) {
            if ((st = t_close(c)) != LBM_OK) return st;
            double r[3];
            const bool wake = c->cfg.objective == LBM_J_WAKE;
            if ((st = window_end(c, c->acc, c->partials[0], r, wake ? c->facc[c->fa] : nullptr)) != LBM_OK)
                return st;
            if (L.ncomp) {
                // this window's field is the adjoint's; the next one starts at zero
                c->fw = c->fa;
                c->fa = c->fa == 0 ? 1 : 0;
                HIPCHK(launch_fill(c->facc[c->fa], L.nf, 0.0, c->stream));
            }
            double rel = NAN;
            int conv = 0;
            if (!c->M.empty()) criterion(c->M.back(), r[1], c->cfg.eps, rel, conv);
            c->J.push_back(r[0]);
            c->M.push_back(r[1]);
            c->rel.push_back(rel);
            c->conv.push_back(conv);
            if (r[2] > 0.0) {
                c->unstable = true;
                t_drain(c);
                if (rep) {
                    rep->unstable = 1;
                    rep->steps_done = c->step;
                }
                return fail(LBM_E_UNSTABLE, "non-finite or |u| >= 0.4 in window " + std::to_string(m / W));
            }
            if (stop_on_converge && (conv || (int)c->M.size() >= c->cfg.max_windows)) break;
        }
    }
    if ((st = t_close(c)) != LBM_OK) return st;
    HIPCHK(hipStreamSynchronize(c->stream));
    if ((st = t_drain(c)) != LBM_OK) return st;
    if (rep) {
        rep->steps_done = c->step;
        rep->windows_done = (int)c->M.size();
        rep->w_eff = (int)last_window(c);
        rep->converged = c->conv.empty() ? 0 : c->conv.back();
        rep->J_eff = c->J.empty() ? NAN : c->J.back();
        rep->monitor = c->M.empty() ? NAN : c->M.back();
        rep->rel_change = c->rel.empty() ? NAN : c->rel.back();
        rep->unstable = 0;
    }
    return LBM_OK;
}

lbm_status lbm_window_history(lbm_ctx* c, double* J, double* M, double* rel, int cap, int* n) {
    if (!c) return fail(LBM_E_INVALID, "NULL context");
    const int k = (int)c->M.size();
    for (int i = 0; i < k && i < cap; ++i) {
        if (J) J[i] = c->J[i];
        if (M) M[i] = c->M[i];
        if (rel) rel[i] = c->rel[i];
    }
    if (n) *n = k;
    return LBM_OK;
}

lbm_status lbm_adjoint(lbm_ctx* c, int window, double* dJdgamma_dev, double* J_out) {
    if (!c || !dJdgamma_dev) return fail(LBM_E_INVALID, "NULL argument");
    const long g = last_window(c);
    if (g == 0) return fail(LBM_E_STATE, "no completed window");
    if (window != 0 && window != g) return fail(LBM_E_STATE, "only the last completed window can be differentiated");
    if (c->unstable) return fail(LBM_E_STATE, "state is unstable");
    const long W = c->cfg.window_len;
    const Layout& L = c->L;
    lbm_status st;
    HIPCHK(launch_fill(c->sens, L.N, 0.0, c->stream));
    int cur = 0;
    if ((st = adjoint_window(c, c->ring[g % 2], (g - 1) * W + 1, true, cur)) != LBM_OK) return st;
    if (c->cfg.objective == LBM_J_DRAG) HIPCHK(launch_box_add(c->sens, c->facc[c->fw], c->geo, c->ob, c->stream));
    HIPCHK(launch_finalize(c->gamma, c->sens, dJdgamma_dev, L.N, c->cfg.s_map, c->cfg.s_q, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if ((st = t_drain(c)) != LBM_OK) return st;
    if (J_out) *J_out = c->J.back();
    return LBM_OK;
}

lbm_status lbm_adjoint_full(lbm_ctx* c, double* dJdgamma_dev, double* J_out) {
    if (!c || !dJdgamma_dev) return fail(LBM_E_INVALID, "NULL argument");
    if (c->starts.empty()) return fail(LBM_E_STATE, "the full-time adjoint needs cfg.full_history = 1");
    const long g = last_window(c);
    if (g == 0) return fail(LBM_E_STATE, "no completed window");
    if (c->unstable) return fail(LBM_E_STATE, "state is unstable");
    const long W = c->cfg.window_len, K = c->cfg.ckpt_every;
    const long g0 = c->base / W + 1;                  // first window of the history
    if (g - g0 + 1 > (long)c->starts.size())
        return fail(LBM_E_STATE, "more windows than max_windows since the start of the history");
    const Layout& L = c->L;
    lbm_status st;
    HIPCHK(launch_fill(c->sens, L.N, 0.0, c->stream));
    int cur = 0;
    if ((st = adjoint_window(c, c->ring[g % 2], (g - 1) * W + 1, true, cur)) != LBM_OK) return st;
    StepLaunch a = step_args(c);
    a.s = c->s;
    for (long gw = g - 1; gw >= g0; --gw) {
        // rebuild window gw's checkpoints by replaying it from its start state
        HIPCHK(launch_copy(c->starts[gw - g0], c->ring_rep[0], L.SB, c->stream));
        AuxLaunch ca = aux_args(c, AUX_COLLIDE);
        ca.src = c->ring_rep[0];
        ca.dst = c->seg[0];
        HIPCHK(launch_aux(ca));
        int sc = 0;
        for (long m0 = 0; m0 < W - K;) {
            const long n = plan_launch(c, m0, K, W, W - K - m0, false);
            const long m = m0 + n;
            a.nsteps = (int)n;
            a.gin = c->seg[sc];
            a.gout = c->seg[sc ^ 1];
            a.pre = (m % K == 0) ? c->ring_rep[m / K] : nullptr;
            a.sample = 0;
            if ((st = t_launch(c, 2, n)) != LBM_OK) return st;
            HIPCHK(launch_step(a));
            sc ^= 1;
            m0 = m;
        }
        if ((st = t_close(c)) != LBM_OK) return st;
        // its reverse sweep from the adjoint of the next window's start state
        if ((st = adjoint_window(c, c->ring_rep, (gw - 1) * W + 1, false, cur)) != LBM_OK) return st;
    }
    if (c->cfg.objective == LBM_J_DRAG) HIPCHK(launch_box_add(c->sens, c->facc[c->fw], c->geo, c->ob, c->stream));
    HIPCHK(launch_finalize(c->gamma, c->sens, dJdgamma_dev, L.N, c->cfg.s_map, c->cfg.s_q, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if ((st = t_drain(c)) != LBM_OK) return st;
    if (J_out) *J_out = c->J.back();
    return LBM_OK;
}

lbm_status lbm_window_replay(lbm_ctx* c, const double* gamma_dev, double* J_out) {
    if (!c || !gamma_dev) return fail(LBM_E_INVALID, "NULL argument");
    const long g = last_window(c);
    if (g == 0) return fail(LBM_E_STATE, "no completed window");
    lbm_status st = check_gamma(c, gamma_dev);
    if (st != LBM_OK) return st;
    const long W = c->cfg.window_len, dW = c->cfg.sample_every;
    const Layout& L = c->L;
    if ((st = apply_design(c, gamma_dev, c->s_rep)) != LBM_OK) return st;
    AuxLaunch ca = aux_args(c, AUX_COLLIDE);
    ca.src = c->ring[g % 2][0];
    ca.dst = c->seg[0];
    ca.s = c->s_rep;
    HIPCHK(launch_aux(ca));
    StepLaunch a = step_args(c);
    a.s = c->s_rep;
    if (L.ncomp) {
        HIPCHK(launch_fill(c->facc[2], L.nf, 0.0, c->stream));
        a.ob.facc = c->facc[2];
    }
    int cur = 0;
    for (long m0 = 0; m0 < W;) {
        const long n = plan_launch(c, m0, dW, W, W - m0, false);
        const long m = m0 + n;
        a.nsteps = (int)n;
        a.gin = c->seg[cur];
        a.gout = c->seg[cur ^ 1];
        a.sample = (m % dW == 0) ? 1 : 0;
        if (a.sample) a.partials = c->partials[1] + (m / dW - 1) * L.pstride * 3;
        HIPCHK(launch_step(a));
        cur ^= 1;
        m0 = m;
    }
    double r[3];
    if ((st = window_end(c, c->acc + 4, c->partials[1], r,
                         c->cfg.objective == LBM_J_WAKE ? c->facc[2] : nullptr)) != LBM_OK)
        return st;
    if (r[2] > 0.0) return fail(LBM_E_UNSTABLE, "replay became unstable");
    if (J_out) *J_out = r[0];
    return LBM_OK;
}

lbm_status lbm_set_wake_reference(lbm_ctx* c, const double* u_ref_dev) {
    if (!c || !u_ref_dev) return fail(LBM_E_INVALID, "NULL argument");
    if (c->cfg.objective != LBM_J_WAKE) return fail(LBM_E_STATE, "the objective is not LBM_J_WAKE");
    HIPCHK(hipMemcpyAsync(c->uref, u_ref_dev, (size_t)c->L.nf * 8, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_wake_mean_velocity(lbm_ctx* c, double* u_bar_dev) {
    if (!c || !u_bar_dev) return fail(LBM_E_INVALID, "NULL argument");
    if (c->cfg.objective != LBM_J_WAKE) return fail(LBM_E_STATE, "the objective is not LBM_J_WAKE");
    if (last_window(c) == 0 || c->fw < 0) return fail(LBM_E_STATE, "no completed window");
    HIPCHK(hipMemcpyAsync(u_bar_dev, c->facc[c->fw], (size_t)c->L.nf * 8, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_get_state(lbm_ctx* c, double* host_f, long* step) {
    if (!c || !host_f) return fail(LBM_E_INVALID, "NULL argument");
    const Layout& L = c->L;
    AuxLaunch a = aux_args(c, c->step == c->base ? AUX_EXPORT_DIRECT : AUX_EXPORT_PULL);
    a.src = c->step == c->base ? ring_slot_for_step(c, c->base) : c->G[c->cur ^ 1];
    a.dst = c->nu[0];
    HIPCHK(launch_aux(a));
    HIPCHK(hipMemcpyAsync(host_f, c->nu[0], (size_t)L.Q * L.N * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (step) *step = c->step;
    return LBM_OK;
}

lbm_status lbm_set_state(lbm_ctx* c, const double* host_f, long step) {
    if (!c || !host_f) return fail(LBM_E_INVALID, "NULL argument");
    if (step < 0 || step % c->cfg.window_len != 0) return fail(LBM_E_INVALID, "step must be a multiple of window_len");
    const Layout& L = c->L;
    for (long i = 0; i < (long)L.Q * L.N; ++i)
        if (!std::isfinite(host_f[i])) return fail(LBM_E_INVALID, "state has a non-finite entry");
    HIPCHK(hipMemcpyAsync(c->nu[0], host_f, (size_t)L.Q * L.N * 8, hipMemcpyHostToDevice, c->stream));
    AuxLaunch a = aux_args(c, AUX_IMPORT);
    a.src = c->nu[0];
    a.dst = ring_slot_for_step(c, step);
    HIPCHK(launch_aux(a));
    lbm_status st = start_from_slot(c, step);
    if (st != LBM_OK) return st;
    HIPCHK(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_get_fields(lbm_ctx* c, double* rho_u_dev) {
    if (!c || !rho_u_dev) return fail(LBM_E_INVALID, "NULL argument");
    AuxLaunch a = aux_args(c, c->step == c->base ? AUX_FIELDS_DIRECT : AUX_FIELDS_PULL);
    a.src = c->step == c->base ? ring_slot_for_step(c, c->base) : c->G[c->cur ^ 1];
    a.dst = rho_u_dev;
    HIPCHK(launch_aux(a));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_timing(lbm_ctx* c, int enable, double* out) {
    if (!c) return fail(LBM_E_INVALID, "NULL context");
    lbm_status st = t_drain(c);
    if (st != LBM_OK) return st;
    if (out) {
        for (int i = 0; i < 4; ++i) {
            out[2 * i] = c->tm.n[i];
            out[2 * i + 1] = c->tm.ms[i];
        }
        out[8] = c->tm.st[3];
        out[9] = c->tm.st[2];
        out[10] = c->tm.st[1];
    }
    if (enable) {
        if (c->tm.ev.empty()) {
            c->tm.ev.resize(512);
            c->tm.cls.resize(256);
            c->tm.cnt.resize(256);
            c->tm.steps.resize(256);
            for (auto& e : c->tm.ev) HIPCHK(hipEventCreate(&e));
        }
        for (int i = 0; i < 4; ++i) c->tm.n[i] = c->tm.ms[i] = c->tm.st[i] = 0.0;
        c->tm.used = 0;
        c->tm.open = -1;
    }
    c->tm.on = enable != 0;
    return LBM_OK;
}

const char* lbm_last_error(void) { return g_err.c_str(); }

void lbm_destroy(lbm_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& e : c->tm.ev) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
