// gfx950 kernels of the windowed LBM-LES solver and its discrete adjoint.
//
// Structure-of-arrays populations, so that every load and store of a wave
// covers a contiguous run of one population plane. The step is a fused
// pull (stream) -> boundary rules -> sample -> collide -> partial
// bounce-back -> store: the state in HBM is the post-collision one
// (G^k = C(f^k)), and the post-boundary state f^k of the paper only lives
// in registers or LDS. The adjoint step is the mirror pull of the adjoint
// populations fused with the transposed collision in moment space. At
// about 3 flop per algorithmic byte there is no MFMA.
//
// Three launch forms per step kind:
//   * single steps (k_step, k_adjoint): one thread per node, 256 threads
//     per workgroup, each population read and written once per step, no
//     LDS;
//   * temporally blocked D2Q9 launches (k_step_tb, k_adjoint_tb): a
//     workgroup advances its tile and a shrinking halo several steps in
//     LDS, so HBM is touched once per launch;
//   * D3Q19 two-step launches marching along z (k_step_tbz,
//     k_adjoint_tbz): the first step's planes pass through a three-plane
//     LDS ring and the second step reads them there.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "launch.hpp"

namespace lbm {

constexpr int BLOCK = 256;

// Block-wide FP64 sum of NC channels over NT threads; thread 0 writes them
// to out[0..NC).
template <int NC, int NT>
__device__ __forceinline__ void block_sum_n(double v[NC], double* out) {
    __shared__ double red[NC][NT / 64];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double x = v[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        v[c] = x;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) red[c][wid] = v[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double acc = 0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) acc += red[c][w];
            out[c] = acc;
        }
    }
}

template <int NC>
__device__ __forceinline__ void block_sum(double v[NC], double* out) {
    block_sum_n<NC, BLOCK>(v, out);
}

// Per-node objective and monitor contributions on the post-boundary state
// f^k with bounce-back fraction s: the pressure drop c_s^2 (mean_in rho -
// mean_out rho) written with drho (the constant cancels), the node
// dissipation, and the drag 2 s j_x (the collision keeps j, the fluid-solid
// term removes 2 s j from the fluid) over the force box. The window field
// accumulator receives dW/|W| times 2 j_x (drag: the explicit dD/ds) or u
// (wake) on its box.
// Raw buffer access (the range check of a buffer resource): a byte offset
// of BUF_OOB lies beyond every array, so a store there is dropped and a load
// returns 0. The z-marching kernel issues all of its global loads and stores
// this way and unconditionally, so that every plane issues the same sequence
// of vector memory operations whatever the lane, plane or face; the
// compiler's count of the loads still in flight is then exact across its
// branches, and the loads of two planes stay in flight behind the current
// one. The arrays must be smaller than BUF_OOB bytes (checked by the host).
constexpr unsigned BUF_OOB = 0xFFFFFFF0u;
using BufRsrc = __amdgpu_buffer_rsrc_t;
using BufU2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(BufRsrc(), 0, 0, 0));

// The offset passes through an empty asm statement, so that the compiler
// cannot see its out-of-range value and split one access into branches.
__device__ __forceinline__ unsigned buf_off(unsigned off) {
    asm("" : "+v"(off));
    return off;
}

__device__ __forceinline__ BufRsrc buf_rsrc(const void* p, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)(unsigned)bytes, 0x00020000);
}
__device__ __forceinline__ void buf_ld(BufRsrc r, unsigned off, float& v) {
    v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)buf_off(off), 0, 0));
}
__device__ __forceinline__ void buf_ld(BufRsrc r, unsigned off, double& v) {
    v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)buf_off(off), 0, 0));
}
__device__ __forceinline__ void buf_ld(BufRsrc r, unsigned off, _Float16& v) {
    v = __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, (int)buf_off(off), 0, 0));
}
// FP16 storage is loaded into a full 32-bit register (zero-extended), so
// that two values in flight never share one register.
__device__ __forceinline__ void buf_ld(BufRsrc r, unsigned off, unsigned& v) {
    v = (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, (int)buf_off(off), 0, 0);
}
template <class S>
struct BufReg {
    using type = S;
};
template <>
struct BufReg<_Float16> {
    using type = unsigned;
};
template <class T, class R>
__device__ __forceinline__ T from_reg(R v) {
    if constexpr (sizeof(R) == 4 && !std::is_floating_point<R>::value)
        return (T)__builtin_bit_cast(_Float16, (unsigned short)v);
    else
        return (T)v;
}

__device__ __forceinline__ void buf_st(BufRsrc r, unsigned off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)buf_off(off), 0, 0);
}
__device__ __forceinline__ void buf_st(BufRsrc r, unsigned off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(BufU2, v), r, (int)buf_off(off), 0, 0);
}
__device__ __forceinline__ void buf_st(BufRsrc r, unsigned off, _Float16 v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)buf_off(off), 0, 0);
}

// Pull of a node for the single-step kernels. An interior node reads its Q
// populations through one buffer resource per plane whose base already
// holds that plane's uniform source shift (plane a starts at
// G + a N - off_a), so every load takes the same byte offset n sizeof(S):
// one vector instruction for all Q addresses instead of the 64-bit address
// arithmetic of each plain load. n - off_a lies in [0, N) for an interior
// node, so every access stays inside plane a. Boundary nodes take pull().
template <class L, class S, class T>
__device__ __forceinline__ void pull_buf(const S* __restrict__ G, const Geo& g, int n, int x, int y, int z,
                                         T h[L::Q]) {
    const bool interior = x > 0 && x < g.nx - 1 && y > 0 && y < g.ny - 1 &&
                          (L::D == 2 || (z > 0 && z < g.nz - 1));
    if (interior) {
        const unsigned vo = (unsigned)n * (unsigned)sizeof(S);
        const size_t pb = (size_t)g.N * sizeof(S);
#pragma unroll
        for (int a = 0; a < L::Q; ++a) {
            const long off = L::cx[a] + (long)L::cy[a] * g.nx + (long)L::cz[a] * g.nx * g.ny;
            typename BufReg<S>::type v;
            buf_ld(buf_rsrc(G + ((long)a * g.N - off), pb), vo, v);
            h[a] = from_reg<T>(v);
        }
        return;
    }
    pull<L, S, T>(G, g, n, x, y, z, h);
}

// Store of a node's Q post-collision populations through one buffer
// resource per plane (the same byte offset n sizeof(S) for every plane).
template <class L, class S, class T>
__device__ __forceinline__ void store_buf(S* __restrict__ G, int N, int n, const T out[L::Q]) {
    const unsigned vo = (unsigned)n * (unsigned)sizeof(S);
    const size_t pb = (size_t)N * sizeof(S);
#pragma unroll
    for (int a = 0; a < L::Q; ++a) buf_st(buf_rsrc(G + (size_t)a * N, pb), vo, (S)out[a]);
}

template <class L, class T>
__device__ __forceinline__ void node_samples(const Obj& ob, int x, int y, int z, T s, const Moments<L, T>& m,
                                             double v[3]) {
    double dp = 0.0;
    if (x == ob.in_x && y >= ob.in_lo && y < ob.in_hi) dp += (1.0 / 3.0) * (double)m.drho * ob.inv_nin;
    if (x == ob.out_x && y >= ob.out_lo && y < ob.out_hi) dp -= (1.0 / 3.0) * (double)m.drho * ob.inv_nout;
    double diss = 0.0;
    if (ob.obj == 1 || ob.mon == 1) diss = (double)dissipation<L, T>(m);
    double drag = 0.0;
    if ((ob.obj == 2 || ob.mon == 2) && in_force_box(ob, x, y, z)) drag = 2.0 * (double)s * (double)m.j[0];
    v[0] = (ob.obj <= 1 ? dp : 0.0) + (ob.obj == 1 ? diss : 0.0) + (ob.obj == 2 ? drag : 0.0);
    v[1] = (ob.mon <= 1 ? dp : 0.0) + (ob.mon == 1 ? diss : 0.0) + (ob.mon == 2 ? drag * ob.inv_dref : 0.0);
    if (ob.facc) {
        const int i = acc_index(ob, x, y, z);
        if (i >= 0) {
            if (ob.obj == 2) {
                ob.facc[i] += ob.wgt * 2.0 * (double)m.j[0];
            } else {
#pragma unroll
                for (int p = 0; p < L::D; ++p) ob.facc[p * ob.nb + i] += ob.wgt * (double)(m.j[p] * m.irho);
            }
        }
    }
    T uu = 0;
#pragma unroll
    for (int p = 0; p < L::D; ++p) uu += m.j[p] * m.j[p];
    uu *= m.irho * m.irho;
    v[2] = (uu < (T)0.16) ? 0.0 : 1.0;   // also catches NaN
}

// Forward step k: G_out = C(BC(S(G_in))). SAMPLE: write the block partials
// of the sampled quantities of f^k. WPRE: also store f^k (pre-collision,
// shifted) as a checkpoint. REC: also store the moment record of f^k (the
// recompute of an adjoint segment).
// Zeroes the partial slots [gridDim.x, stride) that this launch does not
// write, so that launches with different grids share one partials layout.
template <int NT>
__device__ __forceinline__ void zero_unused_partials_n(double* partials, int stride) {
    if (blockIdx.x != 0) return;
    for (int i = (int)gridDim.x + (int)threadIdx.x; i < stride; i += NT) {
        partials[3 * i + 0] = 0.0;
        partials[3 * i + 1] = 0.0;
        partials[3 * i + 2] = 0.0;
    }
}

__device__ __forceinline__ void zero_unused_partials(double* partials, int stride) {
    zero_unused_partials_n<BLOCK>(partials, stride);
}

template <class L, class S, class T, bool SAMPLE, bool WPRE, bool REC = false>
__global__ __launch_bounds__(BLOCK) void k_step(const S* __restrict__ gin, S* __restrict__ gout,
                                                S* __restrict__ pre, const T* __restrict__ sfield,
                                                Geo g, Phys ph, Obj ob, double* __restrict__ partials,
                                                int part_stride, T* __restrict__ rec = nullptr) {
    const int n = (int)(blockIdx.x * BLOCK + threadIdx.x);
    const bool active = n < g.N;
    double v[3] = {0.0, 0.0, 0.0};
    if (active) {
        int x, y, z;
        node_coords(g, n, x, y, z);
        const int oc = open_code<L>(g, x, y, z);
        T h[L::Q];
        pull_buf<L, S, T>(gin, g, n, x, y, z, h);
        if (oc) zou_he<L, T>(g, oc, y, h);
        if (WPRE) {
#pragma unroll
            for (int a = 0; a < L::Q; ++a) plane(pre, a, g.N)[(unsigned)n] = (S)h[a];
        }
        Moments<L, T> m;
        moments<L, T>(h, ph, m);
        if (REC) record_store<L, T>(rec, g.N, n, m);
        const T s = sfield[n];
        if (SAMPLE) node_samples<L, T>(ob, x, y, z, s, m, v);
        T out[L::Q];
        collide<L, T>(m, s, out);
        store_buf<L, S, T>(gout, g.N, n, out);
    }
    if (SAMPLE) {
        block_sum<3>(v, partials + 3 * (size_t)blockIdx.x);
        zero_unused_partials(partials, part_stride);
    }
}

// Temporally blocked forward steps (D2Q9): one launch advances NT steps.
// Each workgroup owns an output tile of ox x oy nodes. Step 1 pulls from
// the post-collision state in global memory over the tile grown by NT - 1
// nodes per side and keeps the new post-collision populations in LDS; each
// further step pulls from LDS over a region one node smaller per side; the
// last step writes the tile to global memory. Only the last step may be a
// sampled step (SAMPLE) or a checkpoint step (WPRE). Halo nodes are
// recomputed by neighbouring tiles; every node update uses the same device
// functions as the single-step kernel.
//
// Walls inside LDS: the LDS region keeps the cells beyond a non-periodic
// face as ghost cells. A node on such a face stores every population that
// would leave the domain into the ghost cell it would stream to, in the
// plane of the opposite direction; the pull of that node at the next step
// reads exactly that slot, which is the halfway bounce-back of Eq. wall.
// The LDS pull is therefore the same gather for every node, with no
// per-direction tests. The open-row codes and inlet speeds of the region's
// rows are cached in LDS during step 1.
//
// LDS: two buffers of Q planes of (ox + 2(NT-1)) x (oy + 2(NT-1)) values in
// compute precision, one plane of the bounce-back fraction (read from global
// memory once), and the row cache. TB threads (512 or 1024, whichever
// covers the first region in one round) update the nodes of a region.
//
// The region of a step is [m, LW - m) x [m, LH - m), cut to the domain on a
// non-periodic axis and, for the output step, to the tile's own nodes
// (unwrapped x < nx, y < ny, so that periodic wraps are not written twice).
// Its cells are dealt to threads in two parts: first the interior rectangle
// (nodes off every non-periodic face, which need neither the Zou-He rule nor
// ghost-cell stores), row by row; then the face frame (the node rows and
// columns on non-periodic faces, at most one wide on each side), which take
// the boundary work. The face cells thus share a few wavefronts instead of
// diverging every wavefront of a boundary tile.
struct TbPhase {
    int ax, ay, rw;           // cut region: first LDS column and row, width
    int ix0, iy0, iw, ih;     // interior rectangle: first column and row, width, height
    int ni;                   // interior cells (iw * ih)
    int nb, nt, nl;           // face frame: bottom row, top row, left column present (0/1)
    int count;                // all cells of the step
    float inv;                // 1 / iw
};

__device__ __forceinline__ TbPhase tb_phase(const Geo& g, int m, int LW, int LH, int x0, int y0, bool output) {
    int ax = m, bx = LW - m, ay = m, by = LH - m;
    if (!g.per_x) ax = max(ax, -x0);
    if (!g.per_y) ay = max(ay, -y0);
    if (!g.per_x || output) bx = min(bx, g.nx - x0);
    if (!g.per_y || output) by = min(by, g.ny - y0);
    bx = max(bx, ax);
    by = max(by, ay);
    int ix0 = ax, ix1 = bx, iy0 = ay, iy1 = by;
    if (!g.per_x) {
        ix0 = min(max(ax, 1 - x0), bx);
        ix1 = max(min(bx, g.nx - 1 - x0), ix0);
    }
    if (!g.per_y) {
        iy0 = min(max(ay, 1 - y0), by);
        iy1 = max(min(by, g.ny - 1 - y0), iy0);
    }
    TbPhase p;
    p.ax = ax;
    p.ay = ay;
    p.rw = bx - ax;
    p.ix0 = ix0;
    p.iy0 = iy0;
    p.iw = ix1 - ix0;
    p.ih = iy1 - iy0;
    p.ni = p.iw * p.ih;
    p.nb = iy0 - ay;        // 0 or 1
    p.nt = by - iy1;        // 0 or 1
    p.nl = ix0 - ax;        // 0 or 1; the right column has bx - ix1 cells per row
    p.count = p.rw * (by - ay);
    p.inv = 1.0f / (float)p.iw;
    return p;
}

// Cell i (< count) of a step: LDS coordinates and the (wrapped) global node.
// Returns true for a face cell.
struct TbCell {
    int lx, ly, x, y, n, cell;
};

__device__ __forceinline__ bool tb_cell(const Geo& g, int i, const TbPhase& p, int LW, int x0, int y0,
                                        TbCell& c) {
    bool face = false;
    if (i < p.ni) {
        const int qy = (int)(((float)i + 0.5f) * p.inv);   // exact for i < 2^12
        c.ly = p.iy0 + qy;
        c.lx = p.ix0 + (i - qy * p.iw);
    } else {
        face = true;
        int j = i - p.ni;
        const int nrow = p.rw * (p.nb + p.nt);
        if (j < nrow) {                                     // bottom row, then top row
            const bool top = j >= p.rw * p.nb;
            c.ly = top ? p.iy0 + p.ih : p.ay;
            c.lx = p.ax + (top ? j - p.rw * p.nb : j);
        } else {                                            // left column, then right column
            j -= nrow;
            const bool right = j >= p.ih * p.nl;
            c.ly = p.iy0 + (right ? j - p.ih * p.nl : j);
            c.lx = right ? p.ix0 + p.iw : p.ax;
        }
    }
    int x = x0 + c.lx, y = y0 + c.ly;
    if (g.per_x) x = ((x % g.nx) + g.nx) % g.nx;
    if (g.per_y) y = ((y % g.ny) + g.ny) % g.ny;
    c.x = x;
    c.y = y;
    c.n = y * g.nx + x;
    c.cell = c.ly * LW + c.lx;
    return face;
}

// Tile of this workgroup. Workgroups are dealt to the 8 XCDs of the chip
// round-robin (workgroup b runs on XCD b mod 8). The tiles are numbered down
// the columns and each XCD takes a contiguous run of those numbers, so that
// neighbouring tiles, whose halos overlap, mostly share an XCD and its L2.
__device__ __forceinline__ void tb_tile(int tiles_x, int& tx, int& ty) {
    const int T = (int)gridDim.x, tiles_y = T / tiles_x;
    const int b = (int)blockIdx.x, xcd = b & 7, idx = b >> 3;
    int start = 0;
    for (int k = 0; k < xcd; ++k) start += (T - k + 7) >> 3;   // workgroups on XCDs before this one
    const int t = start + idx;
    tx = t / tiles_y;
    ty = t - tx * tiles_y;
}

// Block number of this workgroup in an order where each of the 8 XCDs
// (workgroup b runs on XCD b mod 8) takes a contiguous range of numbers.
__device__ __forceinline__ int xcd_block() {
    const int T = (int)gridDim.x;
    const int b = (int)blockIdx.x, xcd = b & 7, idx = b >> 3;
    int start = 0;
    for (int k = 0; k < xcd; ++k) start += (T - k + 7) >> 3;   // workgroups on XCDs before this one
    return start + idx;
}

// True if cell c belongs to the tile's own output nodes (each node of the
// domain is owned by exactly one tile).
__device__ __forceinline__ bool tb_owned(const Geo& g, const TbCell& c, int H, int ox, int oy, int x0, int y0) {
    const int ux = x0 + c.lx, uy = y0 + c.ly;
    return c.lx >= H && c.lx < H + ox && c.ly >= H && c.ly < H + oy && ux < g.nx && uy < g.ny;
}

// Row cache of the LDS region (rows y0 .. y0 + LH - 1): Zou-He code of the
// west and east face nodes (open_code's values) and the inlet speed.
template <class T>
struct TbRows {
    T* u;
    signed char* west;
    signed char* east;
};

template <class T>
__device__ __forceinline__ TbRows<T> tb_rows(T* base, int LH) {
    TbRows<T> r;
    r.u = base;
    r.west = reinterpret_cast<signed char*>(base + LH);
    r.east = r.west + LH;
    return r;
}

template <class T, int TB>
__device__ __forceinline__ void tb_fill_rows(const Geo& g, const TbRows<T>& r, int LH, int y0) {
    for (int i = (int)threadIdx.x; i < LH; i += TB) {
        int y = y0 + i;
        if (g.per_y) y = ((y % g.ny) + g.ny) % g.ny;
        signed char wc = 0, ec = 0;
        T u = (T)0;
        if (y >= 0 && y < g.ny) {
            if (!g.per_x) {
                const int kw = g.west[y], ke = g.east[y];
                wc = (signed char)(kw ? 1 + kw : 0);
                ec = (signed char)(ke ? 4 + ke : 0);
            }
            u = (T)g.u_in[y];
        }
        r.u[i] = u;
        r.west[i] = wc;
        r.east[i] = ec;
    }
}

template <class T>
__device__ __forceinline__ int tb_open(const Geo& g, const TbRows<T>& r, const TbCell& c) {
    if (c.x == 0) return r.west[c.ly];
    if (c.x == g.nx - 1) return r.east[c.ly];
    return 0;
}

// Pull of node c from the previous step's LDS buffer (walls come from the
// ghost cells); on a face cell also the Zou-He rule of an open node.
template <class T, class LT>
__device__ __forceinline__ void tb_pull_lds(const Geo& g, const LT* __restrict__ srcb, int plane_sz, int LW,
                                            const TbRows<T>& rows, T d0, const TbCell& c, bool face, T h[9]) {
    using L = D2Q9;
#pragma unroll
    for (int a = 0; a < L::Q; ++a) h[a] = (T)srcb[a * plane_sz + c.cell - L::cy[a] * LW - L::cx[a]];
    if (face) {
        const int oc = tb_open<T>(g, rows, c);
        if (oc) zou_he_rows<L, T>(oc, rows.u[c.ly], d0, h);
    }
}

// Ghost-cell stores of a node on a non-periodic face. For every direction
// b that leaves the domain across a face the node lies on (the directions
// with c_b . n = +1 for the outward normal n), value(b) goes to the LDS cell
// at c.cell + SGN * c_b in plane opp(b). Forward: SGN = +1, value = G_b (the
// pull of opp(b) at the next step reads it). Adjoint: SGN = -1 with the
// directions b whose -c_b leaves, value = nu_hat_b or 0 (the gather of
// opp(b) reads it). A corner node stores its diagonal twice, with the same
// value. Nodes on the region's edge (only computed at step 1) pull nothing
// from LDS later and store no ghosts, which keeps every store in the region.
template <class LT, class T, int SGN, int NX, int NY>
__device__ __forceinline__ void tb_ghost_face(LT* __restrict__ dst, int psz, int LW, int cell, const T v[9]) {
    using L = D2Q9;
#pragma unroll
    for (int b = 1; b < L::Q; ++b) {
        if ((NX != 0 && SGN * L::cx[b] == NX) || (NY != 0 && SGN * L::cy[b] == NY))
            dst[L::opp[b] * psz + cell + SGN * (L::cy[b] * LW + L::cx[b])] = (LT)v[b];
    }
}

template <class LT, class T, int SGN>
__device__ __forceinline__ void tb_ghosts(const Geo& g, LT* __restrict__ dst, int psz, int LW, int LH,
                                          const TbCell& c, const T v[9]) {
    const bool inner = c.lx >= 1 && c.ly >= 1 && c.lx <= LW - 2 && c.ly <= LH - 2;
    if (!inner) return;
    if (!g.per_x && c.x == 0) tb_ghost_face<LT, T, SGN, -1, 0>(dst, psz, LW, c.cell, v);
    if (!g.per_x && c.x == g.nx - 1) tb_ghost_face<LT, T, SGN, 1, 0>(dst, psz, LW, c.cell, v);
    if (!g.per_y && c.y == 0) tb_ghost_face<LT, T, SGN, 0, -1>(dst, psz, LW, c.cell, v);
    if (!g.per_y && c.y == g.ny - 1) tb_ghost_face<LT, T, SGN, 0, 1>(dst, psz, LW, c.cell, v);
}

// Element type of the forward kernel's LDS state buffers: the compute type,
// except FP16 for FP16-shifted storage, so that every intermediate state of
// a blocked launch is rounded exactly as a single-step launch stores it.
template <class S, class T>
struct TbLds {
    using type = T;
};
template <>
struct TbLds<_Float16, float> {
    using type = _Float16;
};

// ALLOUT (recompute of an adjoint segment): every step t also stores the
// moment record of the tile's pre-collision state f (drho, j, Pi, after the
// boundary rules) to rec + (t - 1) * slot, which the adjoint reads instead
// of pulling the populations again.
// PS > 0: the planes of the LDS buffers are PS values apart (a compile-time
// stride, so a node reaches its nine planes with immediate offsets); PS = 0:
// they are LW * LH apart.
template <class S, class T, bool SAMPLE, bool WPRE, int TB, bool ALLOUT, int PS>
__global__ __launch_bounds__(TB) void k_step_tb(const S* __restrict__ gin, S* __restrict__ gout,
                                                S* __restrict__ pre, const T* __restrict__ sfield,
                                                Geo g, Phys ph, Obj ob, double* __restrict__ partials,
                                                int part_stride, int nt, int ox, int oy, int tiles_x,
                                                T* __restrict__ rec, size_t slot) {
    using L = D2Q9;
    using LT = typename TbLds<S, T>::type;
    extern __shared__ unsigned char lds_raw[];
    LT* lds = reinterpret_cast<LT*>(lds_raw);
    const int H = nt - 1;
    const int LW = ox + 2 * H, LH = oy + 2 * H;
    const int plane_sz = PS > 0 ? PS : LW * LH;
    const int bufsz = L::Q * plane_sz;                // buffer b starts at lds + b * bufsz
    T* sbuf = reinterpret_cast<T*>(lds + 2 * bufsz);  // s of the region, loaded at step 1
    const TbRows<T> rows = tb_rows<T>(sbuf + plane_sz, LH);
    const T d0 = (T)g.drho_out;
    int tx, ty;
    tb_tile(tiles_x, tx, ty);
    const int x0 = tx * ox - H, y0 = ty * oy - H;     // global coords of LDS cell (0, 0)

    // step 1: pull from global memory over the whole LDS region. A thread
    // takes cells i and i + TB together and issues the loads of both before
    // computing either, so a region of up to 2 TB cells waits on global
    // memory once.
    tb_fill_rows<T, TB>(g, rows, LH, y0);
    {
        const TbPhase ph1 = tb_phase(g, 0, LW, LH, x0, y0, false);
        LT* dst = lds + bufsz;
        for (int i = (int)threadIdx.x; i < ph1.count; i += 2 * TB) {
            TbCell c[2];
            bool v[2], face[2];
            T h[2][L::Q];
            T sv[2];
            int oc[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                v[u] = i + u * TB < ph1.count;
                if (v[u]) {
                    face[u] = tb_cell(g, i + u * TB, ph1, LW, x0, y0, c[u]);
                    oc[u] = face[u] ? open_code<L>(g, c[u].x, c[u].y, 0) : 0;
                    pull<L, S, T>(gin, g, c[u].n, c[u].x, c[u].y, 0, h[u]);
                    sv[u] = sfield[c[u].n];
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (!v[u]) continue;
                if (oc[u]) zou_he<L, T>(g, oc[u], c[u].y, h[u]);
                Moments<L, T> mo;
                moments<L, T>(h[u], ph, mo);
                if (ALLOUT && tb_owned(g, c[u], H, ox, oy, x0, y0)) record_store<L, T>(rec, g.N, c[u].n, mo);
                sbuf[c[u].cell] = sv[u];
                T out[L::Q];
                collide<L, T>(mo, sv[u], out);
#pragma unroll
                for (int a = 0; a < L::Q; ++a) dst[a * plane_sz + c[u].cell] = (LT)out[a];
                if (face[u]) tb_ghosts<LT, T, 1>(g, dst, plane_sz, LW, LH, c[u], out);
            }
        }
        __syncthreads();
    }
    // steps 2 .. nt-1: LDS to LDS over shrinking regions
    for (int t = 2; t < nt; ++t) {
        const TbPhase pt = tb_phase(g, t - 1, LW, LH, x0, y0, false);
        LT* dst = lds + (t & 1) * bufsz;
        const LT* srcb = lds + ((t - 1) & 1) * bufsz;
        for (int i = (int)threadIdx.x; i < pt.count; i += TB) {
            TbCell c;
            const bool face = tb_cell(g, i, pt, LW, x0, y0, c);
            T h[L::Q];
            tb_pull_lds<T, LT>(g, srcb, plane_sz, LW, rows, d0, c, face, h);
            Moments<L, T> mo;
            moments<L, T>(h, ph, mo);
            if (ALLOUT && tb_owned(g, c, H, ox, oy, x0, y0))
                record_store<L, T>(rec + (size_t)(t - 1) * slot, g.N, c.n, mo);
            T out[L::Q];
            collide<L, T>(mo, sbuf[c.cell], out);
#pragma unroll
            for (int a = 0; a < L::Q; ++a) dst[a * plane_sz + c.cell] = (LT)out[a];
            if (face) tb_ghosts<LT, T, 1>(g, dst, plane_sz, LW, LH, c, out);
        }
        __syncthreads();
    }
    // step nt: the output tile, from LDS to global memory (samples, checkpoint)
    double v[3] = {0.0, 0.0, 0.0};
    {
        const TbPhase pn = tb_phase(g, nt - 1, LW, LH, x0, y0, true);
        const LT* srcb = lds + ((nt - 1) & 1) * bufsz;
        for (int i = (int)threadIdx.x; i < pn.count; i += TB) {
            TbCell c;
            const bool face = tb_cell(g, i, pn, LW, x0, y0, c);
            T h[L::Q];
            tb_pull_lds<T, LT>(g, srcb, plane_sz, LW, rows, d0, c, face, h);
            if (WPRE) {
#pragma unroll
                for (int a = 0; a < L::Q; ++a) plane(pre, a, g.N)[(unsigned)c.n] = (S)h[a];
            }
            Moments<L, T> mo;
            moments<L, T>(h, ph, mo);
            if (ALLOUT) record_store<L, T>(rec + (size_t)(nt - 1) * slot, g.N, c.n, mo);
            if (SAMPLE) {
                double vv[3];
                node_samples<L, T>(ob, c.x, c.y, 0, sbuf[c.cell], mo, vv);
                v[0] += vv[0];
                v[1] += vv[1];
                v[2] += vv[2];
            }
            T out[L::Q];
            collide<L, T>(mo, sbuf[c.cell], out);
#pragma unroll
            for (int a = 0; a < L::Q; ++a) plane(gout, a, g.N)[(unsigned)c.n] = (S)out[a];
        }
    }
    if (SAMPLE) {
        block_sum_n<3, TB>(v, partials + 3 * (size_t)blockIdx.x);
        zero_unused_partials_n<TB>(partials, part_stride);
    }
}

// Two forward steps per launch for D3Q19, marching along z. A workgroup owns
// an output block of ox x oy x oz nodes: an xy tile and a run of oz planes.
// Step 1 is taken plane by plane, from the plane below the run to the plane
// above it, over the tile grown by one node in x and y (cut to the domain on
// non-periodic axes), and its post-collision state is kept in an LDS ring;
// step 2 of plane k follows once step 1 of plane k + 1 is in the ring, pulls
// from the planes k - 1, k and k + 1 there and writes to global memory. The
// global loads of the next step-1 planes are issued before step 2 of the
// current plane, so they are in flight while it computes. Halo work is only
// in x and y (plus two planes per run), unlike a tile grown in all three
// axes.
//
// The ring holds each direction of a plane only as long as it is read (see
// TbzRing): 43 plane slots instead of three whole planes (57), so a 48 x 16
// tile with its halo (900 cells, 158 KB in FP32) fits one compute unit with
// 1024 threads.
//
// Walls on x and y faces are ghost cells as in the D2Q9 kernel: a face node
// stores each population b leaving across the face at cell + c_b in the slot
// of direction opp(b) of plane k + c_bz, where step 2 of the plane that
// pulls it looks. A wall on a z face is the halfway reflection taken in the
// step-2 pull itself (the node's own opp(a) value of plane k); a whole plane
// lies on such a face, so that choice is uniform across the workgroup.
//
// LDS: the s values of two planes (compute type), then the 43 plane slots of
// (ox + 2) x (oy + 2) values in the storage-rounded LDS type. TB threads
// (256, 512, 768 or 1024 for planes of up to that many region cells) take
// one cell each of a plane (U = 1; the kernel is written for U cells).

// Open-face code of a node's (x, y) position (open_code without the z test).
__device__ __forceinline__ int open_code_xy(const Geo& g, int x, int y) {
    if (g.per_x) return 0;
    if (x == 0) {
        const int k = g.west[y];
        return k ? 1 + k : 0;
    }
    if (x == g.nx - 1) {
        const int k = g.east[y];
        return k ? 4 + k : 0;
    }
    return 0;
}

// Workgroup barrier that orders LDS accesses only, so global loads issued
// before it stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}


// Plane slots of the z-marching rings. Forward (SGN = +1): step 2 of plane
// k pulls its c_z = +1 directions from plane k - 1, its c_z = 0 directions
// from plane k and its c_z = -1 directions from plane k + 1, and runs in the
// ring level after step 1 of plane k + 1. So a plane's c_z = -1 directions
// are read in the level that writes them, its c_z = 0 directions one level
// later and its c_z = +1 directions two levels later. The adjoint (SGN = -1)
// gathers from plane k + c_z instead, so the roles of c_z = +1 and -1 swap.
// Counting also the ghosts that a face node of plane k writes into planes
// k - 1 and k + 1, the three classes need two, two and three slots:
// 2 * 5 + 2 * 9 + 3 * 5 = 43 planes instead of three whole planes (57),
// taken in turn by ring level (level j holds plane zs - 1 + j).
template <int SGN>
struct TbzRing {
    static constexpr int PLANES = 43;
    // 0: read in the writing level, 1: one level later, 2: two levels later
    static constexpr int cls(int a) { return SGN * D3Q19::cz[a] + 1; }
    static constexpr int slots(int k) { return k == 2 ? 3 : 2; }
    static constexpr int count(int k) { return k == 1 ? 9 : 5; }
    static constexpr int first(int k) { return k == 0 ? 0 : (k == 1 ? 10 : 28); }
    static constexpr int rank(int a) {
        int r = 0;
        for (int b = 0; b < a; ++b) r += D3Q19::cz[b] == D3Q19::cz[a] ? 1 : 0;
        return r;
    }
    // plane slot of direction a for ring level j >= -1
    static __device__ __forceinline__ int plane(int a, int j) {
        const int k = cls(a);
        return first(k) + ((j + 6) % slots(k)) * count(k) + rank(a);
    }
};

// Ghost-cell stores of a D3Q19 node of ring level j on non-periodic x or y
// faces. Forward (SGN = +1): each direction b leaving across such a face
// stores v[b] at cell + c_b (in x, y) in the slot of direction opp(b) of
// level j + c_bz. Adjoint (SGN = -1): each direction b whose -c_b leaves
// stores v[b] at cell - c_b in the slot of direction opp(b) of level
// j - c_bz.
template <class LT, class T, int SGN>
__device__ __forceinline__ void tbz_ghosts(const Geo& g, LT* __restrict__ ring, int psz, int LW, int LH, int j,
                                           const TbCell& c, const T v[19]) {
    using L = D3Q19;
    const bool inner = c.lx >= 1 && c.ly >= 1 && c.lx <= LW - 2 && c.ly <= LH - 2;
    if (!inner) return;
    const bool fx0 = !g.per_x && c.x == 0, fx1 = !g.per_x && c.x == g.nx - 1;
    const bool fy0 = !g.per_y && c.y == 0, fy1 = !g.per_y && c.y == g.ny - 1;
#pragma unroll
    for (int b = 1; b < L::Q; ++b) {
        const int sx = SGN * L::cx[b], sy = SGN * L::cy[b];
        const bool leaves = (sx < 0 && fx0) || (sx > 0 && fx1) || (sy < 0 && fy0) || (sy > 0 && fy1);
        if (leaves)
            ring[TbzRing<SGN>::plane(L::opp[b], j + SGN * L::cz[b]) * psz + c.cell + sy * LW + sx] = (LT)v[b];
    }
}

template <class S, class T, bool SAMPLE, bool WPRE, int TB, int U, bool REC = false>
__global__ __launch_bounds__(TB) void k_step_tbz(const S* __restrict__ gin, S* __restrict__ gout,
                                                 S* __restrict__ pre, const T* __restrict__ sfield, Geo g, Phys ph,
                                                 Obj ob, double* __restrict__ partials, int part_stride, int ox,
                                                 int oy, int oz, int tiles_x, int tiles_y, T* __restrict__ rec,
                                                 size_t rslot) {
    using L = D3Q19;
    constexpr int RS = record_size<L>();
    using LT = typename TbLds<S, T>::type;
    extern __shared__ unsigned char lds_raw[];
    const int LW = ox + 2, LH = oy + 2, psz = LW * LH;
    T* sring = reinterpret_cast<T*>(lds_raw);
    LT* ring = reinterpret_cast<LT*>(sring + 2 * psz);
    // blocks are numbered x fastest, then y, then z run; each XCD takes a
    // contiguous range of those numbers (workgroup b runs on XCD b mod 8), so
    // the tiles that share halo rows and cache lines mostly share an L2
    const int b = xcd_block();
    const int tx = b % tiles_x, ty = (b / tiles_x) % tiles_y, tz = b / (tiles_x * tiles_y);
    const int x0 = tx * ox - 1, y0 = ty * oy - 1;       // global x, y of LDS cell (0, 0)
    const int zs = tz * oz, nzc = min(oz, g.nz - zs);   // output planes zs .. zs + nzc - 1
    const int N = g.N, nxy = g.nx * g.ny;
    const T d0 = (T)g.drho_out;
    const size_t state_bytes = (size_t)L::Q * N * sizeof(S);
    const BufRsrc rin = buf_rsrc(gin, state_bytes);
    const BufRsrc rs = buf_rsrc(sfield, (size_t)N * sizeof(T));
    const BufRsrc rout = buf_rsrc(gout, state_bytes);
    const BufRsrc rpre = buf_rsrc(WPRE ? pre : gout, state_bytes);
    // REC: the moment records of f^{k+1} (step 1, owned cells) and f^{k+2}
    // (step 2), in two record slots rslot values apart
    const size_t rec_bytes = (size_t)RS * N * sizeof(T);
    const BufRsrc rrec1 = buf_rsrc(rec, REC ? rec_bytes : 0);
    const BufRsrc rrec2 = buf_rsrc(REC ? rec + rslot : rec, REC ? rec_bytes : 0);

    // this thread's cells of a plane, the same on every plane: up to U of
    // the step-1 region and U of the output tile; a lane without a cell
    // takes LDS cell (1, 1) and node 0 and stores nothing
    const TbPhase p1 = tb_phase(g, 0, LW, LH, x0, y0, false);
    const TbPhase p2 = tb_phase(g, 1, LW, LH, x0, y0, true);
    TbCell c1[U], c2[U];
    bool v1[U], v2[U], f1[U], f2[U], own1[U];
    int o1[U], o2[U];
    T u1[U], u2[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = (int)threadIdx.x + u * TB;
        const TbCell none = {1, 1, 0, 0, 0, LW + 1};
        c1[u] = none;
        c2[u] = none;
        v1[u] = i < p1.count;
        f1[u] = v1[u] && tb_cell(g, i, p1, LW, x0, y0, c1[u]);
        o1[u] = f1[u] ? open_code_xy(g, c1[u].x, c1[u].y) : 0;
        u1[u] = o1[u] ? (T)g.u_in[c1[u].y] : (T)0;
        own1[u] = v1[u] && tb_owned(g, c1[u], 1, ox, oy, x0, y0);
        v2[u] = i < p2.count;
        f2[u] = v2[u] && tb_cell(g, i, p2, LW, x0, y0, c2[u]);
        o2[u] = f2[u] ? open_code_xy(g, c2[u].x, c2[u].y) : 0;
        u2[u] = o2[u] ? (T)g.u_in[c2[u].y] : (T)0;
    }

    // plane of ring level j (zs - 1 + j); false beyond the run or a z wall
    auto level_z = [&](int j, int& z) {
        z = zs - 1 + j;
        if (j < 0 || j > nzc + 1) return false;
        if (g.per_z) {
            z = z < 0 ? z + g.nz : (z >= g.nz ? z - g.nz : z);
            return true;
        }
        return z >= 0 && z < g.nz;
    };
    // loads of the step-1 inputs of level j into a register set, in the
    // storage type (converted at their use, so nothing waits for them here)
    using R = typename BufReg<S>::type;
    auto load1 = [&](int j, R (&h)[U][L::Q], T (&s)[U]) {
        int z;
        const bool ok = level_z(j, z);
        const int zc = ok ? z : 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool live = ok && v1[u];
            const int n = zc * nxy + c1[u].n;
            unsigned e[L::Q];
            pull_index<L>(g, n, c1[u].x, c1[u].y, zc, e);
#pragma unroll
            for (int a = 0; a < L::Q; ++a) buf_ld(rin, live ? e[a] * (unsigned)sizeof(S) : BUF_OOB, h[u][a]);
            buf_ld(rs, live ? (unsigned)n * (unsigned)sizeof(T) : BUF_OOB, s[u]);
        }
    };
    // step 1 of level j into its ring slot (a uniform branch around LDS and
    // arithmetic), then REC's record stores
    auto step1 = [&](int j, const R (&h)[U][L::Q], const T (&s)[U]) {
        int z;
        const bool ok = level_z(j, z);
        T r1[U][RS];
        if (REC) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < RS; ++q) r1[u][q] = (T)0;
        }
        if (ok) {
            const bool zf = !g.per_z && (z == 0 || z == g.nz - 1);
            T* sdst = sring + ((j + 6) % 2) * psz;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!v1[u]) continue;
                T hh[L::Q];
#pragma unroll
                for (int a = 0; a < L::Q; ++a) hh[a] = from_reg<T>(h[u][a]);
                if (o1[u] && !zf) zou_he_rows<L, T>(o1[u], u1[u], d0, hh);
                Moments<L, T> mo;
                moments<L, T>(hh, ph, mo);
                if (REC) record_values<L, T>(mo, r1[u]);
                sdst[c1[u].cell] = s[u];
                T out[L::Q];
                collide<L, T>(mo, s[u], out);
#pragma unroll
                for (int a = 0; a < L::Q; ++a) ring[TbzRing<1>::plane(a, j) * psz + c1[u].cell] = (LT)out[a];
                if (f1[u]) tbz_ghosts<LT, T, 1>(g, ring, psz, LW, LH, j, c1[u], out);
            }
        }
        if (REC) {
            // records of the owned cells of an output plane (level 1 .. nzc),
            // stored by every lane on every level (out-of-range offsets
            // elsewhere)
            const int zc = ok ? z : 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool live = ok && own1[u] && j >= 1 && j <= nzc;
                const unsigned n = (unsigned)(zc * nxy + c1[u].n);
#pragma unroll
                for (int q = 0; q < RS; ++q)
                    buf_st(rrec1, live ? ((unsigned)q * N + n) * (unsigned)sizeof(T) : BUF_OOB, r1[u][q]);
            }
        }
    };
    // step 2 of level j - 1 (plane zs + j - 2) from the slots of levels
    // j - 2, j - 1, j, then its stores
    double v[3] = {0.0, 0.0, 0.0};
    auto step2 = [&](int j) {
        const int k = j - 1;
        const bool ok = k >= 1 && k <= nzc;
        const int z = ok ? zs + k - 1 : 0;
        T out[U][L::Q], hp[U][L::Q], rv[U][RS];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int a = 0; a < L::Q; ++a) out[u][a] = hp[u][a] = (T)0;
#pragma unroll
            for (int q = 0; q < RS; ++q) rv[u][q] = (T)0;
        }
        if (ok) {
            const bool zlo = !g.per_z && z == 0, zhi = !g.per_z && z == g.nz - 1;
            const bool zf = zlo || zhi;
            int off[L::Q];   // uniform source offset of each direction, relative to the cell
#pragma unroll
            for (int a = 0; a < L::Q; ++a) {
                const int shift = -(L::cy[a] * LW + L::cx[a]);
                // the source plane is k - c_az; beyond a z wall, the node's own opp(a)
                const bool refl = (L::cz[a] > 0 && zlo) || (L::cz[a] < 0 && zhi);
                off[a] = refl ? TbzRing<1>::plane(L::opp[a], k) * psz : TbzRing<1>::plane(a, k - L::cz[a]) * psz + shift;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const TbCell& c = c2[u];
                T h[L::Q];
#pragma unroll
                for (int a = 0; a < L::Q; ++a) h[a] = (T)ring[off[a] + c.cell];
                if (o2[u] && !zf) zou_he_rows<L, T>(o2[u], u2[u], d0, h);
                if (WPRE) {
#pragma unroll
                    for (int a = 0; a < L::Q; ++a) hp[u][a] = h[a];
                }
                Moments<L, T> mo;
                moments<L, T>(h, ph, mo);
                if (REC) record_values<L, T>(mo, rv[u]);
                const T sc = sring[((k + 6) % 2) * psz + c.cell];
                if (SAMPLE && v2[u]) {
                    double vv[3];
                    node_samples<L, T>(ob, c.x, c.y, z, sc, mo, vv);
                    v[0] += vv[0];
                    v[1] += vv[1];
                    v[2] += vv[2];
                }
                collide<L, T>(mo, sc, out[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool live = ok && v2[u];
            const unsigned n = (unsigned)(z * nxy + c2[u].n);
#pragma unroll
            for (int a = 0; a < L::Q; ++a) {
                const unsigned o = live ? ((unsigned)a * N + n) * (unsigned)sizeof(S) : BUF_OOB;
                buf_st(rout, o, (S)out[u][a]);
                if (WPRE) buf_st(rpre, o, (S)hp[u][a]);
            }
            if (REC) {
#pragma unroll
                for (int q = 0; q < RS; ++q)
                    buf_st(rrec2, live ? ((unsigned)q * N + n) * (unsigned)sizeof(T) : BUF_OOB, rv[u][q]);
            }
        }
    };
    // ring level j: step 1 of level j from its register set, the loads of
    // level j + 2 into that set, then step 2 of level j - 1, whose levels
    // j - 2 .. j are in the ring. Two register sets keep the loads of two
    // levels in flight; the loop is unrolled by two so that each set has
    // fixed registers, and starts at level -2 (no work, only the loads of
    // levels 0 and 1) so that every pass issues the same memory operations.
    R hA[U][L::Q], hB[U][L::Q];
    T sA[U], sB[U];
    auto level = [&](int j, R (&h)[U][L::Q], T (&s)[U]) {
        step1(j, h, s);
        load1(j + 2, h, s);
        lds_barrier();
        step2(j);
        lds_barrier();
    };
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int a = 0; a < L::Q; ++a) hA[u][a] = hB[u][a] = (R)0;
        sA[u] = sB[u] = (T)0;
    }
    if constexpr (TB <= 768) {
        for (int j = -2; j <= nzc + 1; j += 2) {
            level(j, hA, sA);
            level(j + 1, hB, sB);
        }
    } else {
        // 1024 threads: four waves per SIMD hide the loads, and one input set
        // (loads one level ahead) keeps the kernel within 128 VGPRs
        for (int j = -1; j <= nzc + 1; ++j) {
            step1(j, hA, sA);
            load1(j + 1, hA, sA);
            lds_barrier();
            step2(j);
            lds_barrier();
        }
    }
    if (SAMPLE) {
        block_sum_n<3, TB>(v, partials + 3 * (size_t)blockIdx.x);
        zero_unused_partials_n<TB>(partials, part_stride);
    }
}

// G = C(f) for a stored pre-collision state f (checkpoint restart).
template <class L, class S, class T>
__global__ __launch_bounds__(BLOCK) void k_collide(const S* __restrict__ pre, S* __restrict__ gout,
                                                   const T* __restrict__ sfield, Geo g, Phys ph) {
    const int n = (int)(blockIdx.x * BLOCK + threadIdx.x);
    if (n >= g.N) return;
    T h[L::Q];
#pragma unroll
    for (int a = 0; a < L::Q; ++a) h[a] = (T)plane(pre, a, g.N)[(unsigned)n];
    Moments<L, T> m;
    moments<L, T>(h, ph, m);
    T out[L::Q];
    collide<L, T>(m, sfield[n], out);
#pragma unroll
    for (int a = 0; a < L::Q; ++a) plane(gout, a, g.N)[(unsigned)n] = (S)out[a];
}

// f^0 = f^eq(rho_init, u_init) (Sec. 2.1.3), shifted.
template <class L, class S>
__global__ __launch_bounds__(BLOCK) void k_init_eq(S* __restrict__ pre, Geo g, double rho0, int umode) {
    const int n = (int)(blockIdx.x * BLOCK + threadIdx.x);
    if (n >= g.N) return;
    int x, y, z;
    node_coords(g, n, x, y, z);
    const double ux = umode ? g.u_in[y] : 0.0;
#pragma unroll
    for (int a = 0; a < L::Q; ++a) {
        const double cu = L::cx[a] * ux;
        const double feq = L::w[a] * rho0 * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * ux * ux);
        plane(pre, a, g.N)[(unsigned)n] = (S)(feq - L::w[a]);
    }
}

// Pre-collision state f^k at every node, unshifted FP64, from either a
// stored pre-collision state (DIRECT) or the previous post-collision state
// (pull + boundary rules). FIELDS: write rho and u instead.
template <class L, class S, bool DIRECT, bool FIELDS>
__global__ __launch_bounds__(BLOCK) void k_export(const S* __restrict__ src, double* __restrict__ out, Geo g) {
    const int n = (int)(blockIdx.x * BLOCK + threadIdx.x);
    if (n >= g.N) return;
    double h[L::Q];
    if (DIRECT) {
#pragma unroll
        for (int a = 0; a < L::Q; ++a) h[a] = (double)plane(src, a, g.N)[(unsigned)n];
    } else {
        int x, y, z;
        node_coords(g, n, x, y, z);
        const int oc = open_code<L>(g, x, y, z);
        pull<L, S, double>(src, g, n, x, y, z, h);
        if (oc) zou_he<L, double>(g, oc, y, h);
    }
    if (!FIELDS) {
#pragma unroll
        for (int a = 0; a < L::Q; ++a) plane(out, a, g.N)[(unsigned)n] = h[a] + L::w[a];
    } else {
        double rho = 1.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < L::Q; ++a) {
            rho += h[a];
            j[0] += L::cx[a] * h[a];
            j[1] += L::cy[a] * h[a];
            j[2] += L::cz[a] * h[a];
        }
        out[n] = rho;
#pragma unroll
        for (int p = 0; p < L::D; ++p) plane(out, p + 1, g.N)[(unsigned)n] = j[p] / rho;
    }
}

// Unshifted FP64 populations -> shifted storage.
template <class L, class S>
__global__ __launch_bounds__(BLOCK) void k_import(const double* __restrict__ f, S* __restrict__ pre, Geo g) {
    const int n = (int)(blockIdx.x * BLOCK + threadIdx.x);
    if (n >= g.N) return;
#pragma unroll
    for (int a = 0; a < L::Q; ++a) plane(pre, a, g.N)[(unsigned)n] = (S)(plane(f, a, g.N)[(unsigned)n] - L::w[a]);
}

// Sampled-objective source on the adjoint moments of node (x, y, z) with
// bounce-back fraction s, weighted src_w: the pressure-drop sections and the
// dissipation gradient; the drag 2 s j_x (d/dj_x = 2 s); the wake term
// sum_M |u_bar - u_ref|^2, whose derivative with respect to one sample's u
// is a = 2 (u_bar - u_ref), with d u / d j = 1 / rho, d u / d rho = -u / rho.
template <class L, class T>
__device__ __forceinline__ void adjoint_source(const Obj& ob, const Phys& ph, int x, int y, int z, T s,
                                               const Moments<L, T>& m, double src_w, MomentGrad<L, T>& gr) {
    if (ob.obj <= 1) {
        T dp = 0;
        if (x == ob.in_x && y >= ob.in_lo && y < ob.in_hi) dp += (T)((1.0 / 3.0) * ob.inv_nin * src_w);
        if (x == ob.out_x && y >= ob.out_lo && y < ob.out_hi) dp -= (T)((1.0 / 3.0) * ob.inv_nout * src_w);
        gr.gr += dp;
        if (ob.obj == 1) dissipation_adjoint<L, T>(m, ph, (T)src_w, gr);
    } else if (ob.obj == 2) {
        if (in_force_box(ob, x, y, z)) gr.gj[0] += (T)(2.0 * src_w) * s;
    } else {
        const int i = acc_index(ob, x, y, z);
        if (i >= 0) {
            T au = 0;
#pragma unroll
            for (int p = 0; p < L::D; ++p) {
                const T a = (T)(2.0 * src_w * (ob.fwin[p * ob.nb + i] - ob.uref[p * ob.nb + i]));
                gr.gj[p] += a * m.irho;
                au += a * m.j[p];
            }
            gr.gr -= au * m.irho * m.irho;
        }
    }
}

// Adjoint step for transition k (f^{k-1} -> f^k), reverse order.
//   kappa_a(y) = nu_hat_a(y + c_a)  (adjoint streaming), with the adjoint
//   wall rule kappa_a(y) = nu_hat_opp(a)(y) where y + c_a leaves through a
//   wall and 0 where it leaves through an open face;
//   sens(y) += d/ds <kappa, f**>  (FP64);
//   mu = (d f** / d f^{k-1})^T kappa  (+ sampled objective source);
//   nu_hat^{k-1} = BC^T mu on open nodes.
// The pre-state f^{k-1}(y) comes from a stored checkpoint (DIRECT), from
// its moment record (REC: a recomputed segment) or, for SEED, by pulling
// the post-collision state G^{k-2}; SEED only evaluates the source
// (terminal condition at the window end).
template <class L, class S, class T, class A, bool DIRECT, bool SEED, bool REC = false>
__global__ __launch_bounds__(BLOCK) void k_adjoint(const A* __restrict__ nu_in, A* __restrict__ nu_out,
                                                   const S* __restrict__ state, const T* __restrict__ sfield,
                                                   double* __restrict__ sens, Geo g, Phys ph, Obj ob,
                                                   double src_w) {
    const int n = (int)(blockIdx.x * BLOCK + threadIdx.x);
    if (n >= g.N) return;
    int x, y, z;
    node_coords(g, n, x, y, z);
    const int oc = open_code<L>(g, x, y, z);
    // pre-state of the transition
    Moments<L, T> m;
    if (REC) {
        record_load<L, T>(reinterpret_cast<const T*>(state), g.N, n, ph, m);
    } else {
        T h[L::Q];
        if (DIRECT) {
#pragma unroll
            for (int a = 0; a < L::Q; ++a) h[a] = (T)plane(state, a, g.N)[(unsigned)n];
        } else {
            pull<L, S, T>(state, g, n, x, y, z, h);
            if (oc) zou_he<L, T>(g, oc, y, h);
        }
        moments<L, T>(h, ph, m);
    }
    MomentGrad<L, T> gr;
    gr.gr = 0;
#pragma unroll
    for (int p = 0; p < L::D; ++p) gr.gj[p] = 0;
#pragma unroll
    for (int k = 0; k < Sym<L::D>::K; ++k) gr.GP[k] = 0;
    const T s = sfield[n];
    if (!SEED) {
        T kap[L::Q];
        const int N = g.N;
        const bool interior = x > 0 && x < g.nx - 1 && y > 0 && y < g.ny - 1 &&
                              (L::D == 2 || (z > 0 && z < g.nz - 1));
        if (interior) {
#pragma unroll
            for (int a = 0; a < L::Q; ++a) {
                const int off = L::cx[a] + L::cy[a] * g.nx + L::cz[a] * g.nx * g.ny;
                kap[a] = (T)plane(nu_in, a, N)[(unsigned)(n + off)];
            }
        } else {
#pragma unroll
            for (int a = 0; a < L::Q; ++a) {
                int xt = x + L::cx[a], yt = y + L::cy[a], zt = z + L::cz[a];
                bool out = false;
                if (xt < 0 || xt >= g.nx) {
                    if (g.per_x) xt = xt < 0 ? xt + g.nx : xt - g.nx;
                    else out = true;
                }
                if (yt < 0 || yt >= g.ny) {
                    if (g.per_y) yt = yt < 0 ? yt + g.ny : yt - g.ny;
                    else out = true;
                }
                if (L::D == 3 && (zt < 0 || zt >= g.nz)) {
                    if (g.per_z) zt = zt < 0 ? zt + g.nz : zt - g.nz;
                    else out = true;
                }
                if (!out) kap[a] = (T)plane(nu_in, a, N)[(unsigned)((zt * g.ny + yt) * g.nx + xt)];
                else if (oc == 0) kap[a] = (T)plane(nu_in, L::opp[a], N)[(unsigned)n];
                else kap[a] = (T)0;
            }
        }
        const T ds = collide_adjoint<L, T>(m, ph, s, kap, gr);
        sens[n] += (double)ds;
    }
    if (src_w != 0.0) adjoint_source<L, T>(ob, ph, x, y, z, s, m, src_w, gr);
    T mu[L::Q];
    expand<L, T>(m, gr, mu);
    if (oc) zou_he_adjoint<L, T>(g, oc, y, mu);
#pragma unroll
    for (int a = 0; a < L::Q; ++a) plane(nu_out, a, g.N)[(unsigned)n] = (A)mu[a];
}

// Temporally blocked adjoint steps (D2Q9) over a recomputed segment: one
// launch takes nu_hat^{k_hi} to nu_hat^{k_hi - nt}. Step t (t = 1 .. nt) is
// the transition k = k_hi - t + 1, whose pre-state enters through its
// moment record R^{k-1} = rseg + (k - 2 - kseg) * slot (global memory; the
// recompute stores one record per node and step of the segment). The
// adjoint populations stay in LDS between steps, on tiles grown by nt - 1
// nodes per side as in the forward blocked kernel. Adjoint streaming gathers
// kappa_a(y) = nu_hat_a(y + c_a); for a direction leaving through a wall it
// is nu_hat_opp(a)(y), for one leaving through an open face 0. In LDS both
// come from ghost cells: after its step a face node stores, for every b
// with y - c_b outside the domain, nu_hat_b(y) (0 on an open node) at
// y - c_b in plane opp(b), the slot it gathers kappa_opp(b) from next. The
// sensitivity of the tile's own nodes is summed over the launch's steps in
// an FP64 LDS plane and added to global memory once.
template <class S, class T, class A, int TB, int PS>
__global__ __launch_bounds__(TB) void k_adjoint_tb(const A* __restrict__ nu_in, A* __restrict__ nu_out,
                                                   const T* __restrict__ rseg, size_t slot, long kseg,
                                                   const T* __restrict__ sfield, double* __restrict__ sens,
                                                   Geo g, Phys ph, Obj ob, long k_hi, long ns, long dW, double wgt,
                                                   int nt, int ox, int oy, int tiles_x) {
    using L = D2Q9;
    extern __shared__ unsigned char lds_raw[];
    double* sacc = reinterpret_cast<double*>(lds_raw);   // ox * oy sensitivity sums
    T* lds = reinterpret_cast<T*>(sacc + ox * oy);
    const int H = nt - 1;
    const int LW = ox + 2 * H, LH = oy + 2 * H;
    const int plane_sz = PS > 0 ? PS : LW * LH;
    const int bufsz = L::Q * plane_sz;
    T* sbuf = lds + 2 * bufsz;
    const TbRows<T> rows = tb_rows<T>(sbuf + plane_sz, LH);
    int tx, ty;
    tb_tile(tiles_x, tx, ty);
    const int x0 = tx * ox - H, y0 = ty * oy - H;
    tb_fill_rows<T, TB>(g, rows, LH, y0);
    __syncthreads();
    for (int t = 1; t <= nt; ++t) {
        const long k = k_hi - t + 1;
        const T* Rk1 = rseg + (size_t)(k - 2 - kseg) * slot;
        const double src_w = (k > ns && (k - ns) % dW == 0) ? wgt : 0.0;
        const bool last = t == nt;
        const TbPhase pt = tb_phase(g, t - 1, LW, LH, x0, y0, last);
        const T* srcb = lds + ((t - 1) & 1) * bufsz;
        T* dst = lds + (t & 1) * bufsz;
        for (int i = (int)threadIdx.x; i < pt.count; i += TB) {
            TbCell c;
            const bool face = tb_cell(g, i, pt, LW, x0, y0, c);
            const int oc = face ? tb_open<T>(g, rows, c) : 0;
            const T u0 = rows.u[c.ly];
            // pre-state f^{k-1}: its moment record
            Moments<L, T> m;
            record_load<L, T>(Rk1, g.N, c.n, ph, m);
            // adjoint streaming
            T kap[L::Q];
            if (t == 1) {
                const bool interior = c.x > 0 && c.x < g.nx - 1 && c.y > 0 && c.y < g.ny - 1;
                if (interior) {
#pragma unroll
                    for (int a = 0; a < L::Q; ++a)
                        kap[a] = (T)plane(nu_in, a, g.N)[(unsigned)(c.n + L::cx[a] + L::cy[a] * g.nx)];
                } else {
#pragma unroll
                    for (int a = 0; a < L::Q; ++a) {
                        int xt = c.x + L::cx[a], yt = c.y + L::cy[a];
                        bool out = false;
                        if (xt < 0 || xt >= g.nx) {
                            if (g.per_x) xt = xt < 0 ? xt + g.nx : xt - g.nx;
                            else out = true;
                        }
                        if (yt < 0 || yt >= g.ny) {
                            if (g.per_y) yt = yt < 0 ? yt + g.ny : yt - g.ny;
                            else out = true;
                        }
                        const unsigned src = out ? (unsigned)c.n : (unsigned)(yt * g.nx + xt);
                        const int pa = out ? L::opp[a] : a;
                        const T v = (T)plane(nu_in, pa, g.N)[src];
                        kap[a] = (out && oc) ? (T)0 : v;
                    }
                }
            } else {
#pragma unroll
                for (int a = 0; a < L::Q; ++a) kap[a] = srcb[a * plane_sz + c.cell + L::cy[a] * LW + L::cx[a]];
            }
            T s;
            if (t == 1) {
                s = sfield[c.n];
                sbuf[c.cell] = s;
            } else {
                s = sbuf[c.cell];
            }
            MomentGrad<L, T> gr;
            gr.gr = 0;
#pragma unroll
            for (int p = 0; p < L::D; ++p) gr.gj[p] = 0;
#pragma unroll
            for (int q = 0; q < Sym<L::D>::K; ++q) gr.GP[q] = 0;
            const T ds = collide_adjoint<L, T>(m, ph, s, kap, gr);
            if (tb_owned(g, c, H, ox, oy, x0, y0)) {
                const int o = (c.ly - H) * ox + (c.lx - H);
                if (t == 1) sacc[o] = (double)ds;
                else if (!last) sacc[o] += (double)ds;
                else sens[c.n] += sacc[o] + (double)ds;
            }
            if (src_w != 0.0) adjoint_source<L, T>(ob, ph, c.x, c.y, 0, s, m, src_w, gr);
            T mu[L::Q];
            expand<L, T>(m, gr, mu);
            if (oc) zou_he_adjoint_rows<L, T>(oc, u0, mu);
            if (last) {
#pragma unroll
                for (int a = 0; a < L::Q; ++a) plane(nu_out, a, g.N)[(unsigned)c.n] = (A)mu[a];
            } else {
#pragma unroll
                for (int a = 0; a < L::Q; ++a) dst[a * plane_sz + c.cell] = mu[a];
                // ghost cells of the adjoint wall rule (0 on an open node)
                if (face) {
                    if (oc) {
#pragma unroll
                        for (int a = 0; a < L::Q; ++a) mu[a] = (T)0;
                    }
                    tb_ghosts<T, T, -1>(g, dst, plane_sz, LW, LH, c, mu);
                }
            }
        }
        __syncthreads();
    }
}

// Source of every kappa_a of the adjoint streaming into node (x, y, z), as
// element indices into nu_hat that include the plane: kappa_a(y) =
// nu_hat_a(y + c_a), periodic wraps; where y + c_a leaves through a wall,
// nu_hat_opp(a)(y); where it leaves through an open face (open node), no
// source: GATHER_ZERO, read as 0.
constexpr unsigned GATHER_ZERO = 0xFFFFFFFFu;

template <class L>
__device__ __forceinline__ void gather_index(const Geo& g, int n, int x, int y, int z, bool open,
                                             unsigned e[L::Q]) {
    const int N = g.N;
    const bool interior = x > 0 && x < g.nx - 1 && y > 0 && y < g.ny - 1 &&
                          (L::D == 2 || (z > 0 && z < g.nz - 1));
    if (interior) {
#pragma unroll
        for (int a = 0; a < L::Q; ++a) {
            const int off = L::cx[a] + L::cy[a] * g.nx + L::cz[a] * g.nx * g.ny;
            e[a] = (unsigned)(a * N + off) + (unsigned)n;
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < L::Q; ++a) {
        int xt = x + L::cx[a], yt = y + L::cy[a], zt = z + L::cz[a];
        bool out = false;
        if (xt < 0 || xt >= g.nx) {
            if (g.per_x) xt = xt < 0 ? xt + g.nx : xt - g.nx;
            else out = true;
        }
        if (yt < 0 || yt >= g.ny) {
            if (g.per_y) yt = yt < 0 ? yt + g.ny : yt - g.ny;
            else out = true;
        }
        if (L::D == 3 && (zt < 0 || zt >= g.nz)) {
            if (g.per_z) zt = zt < 0 ? zt + g.nz : zt - g.nz;
            else out = true;
        }
        e[a] = !out ? (unsigned)(a * N + (zt * g.ny + yt) * g.nx + xt)
                    : (open ? GATHER_ZERO : (unsigned)(L::opp[a] * N + n));
    }
}

// Two adjoint steps per launch for D3Q19 over a recomputed segment,
// marching along z (the mirror of k_step_tbz): transitions k_hi and
// k_hi - 1. Step 1 takes nu_hat^{k_hi} from global memory to
// nu_hat^{k_hi - 1} plane by plane over the xy tile grown by one node,
// into a three-slot LDS ring; step 2 of plane z gathers its kappa from the
// ring (planes z - 1, z, z + 1) and writes nu_hat^{k_hi - 2} for the tile;
// the ring keeps each direction of a plane only as long as step 2 reads it.
// Each step reads the moments of its own pre-state f^{k-1} from the
// segment's record of that step (record k - 2 - kseg).
// Walls on x and y faces are ghost cells written by step 1 (nu_hat_b, or 0
// on an open node, at y - c_b in plane opp(b) of the slot of plane
// z - c_bz); a wall on a z face is taken in the step-2 gather itself
// (kappa_a = nu_hat_opp(a) of the node, uniform over the workgroup). The
// step-1 sensitivity of the tile's nodes waits in an FP64 ring and is added
// after it, with step 2's, in one read-modify-write per node. As in
// k_step_tbz every global access is a raw buffer access issued on every
// plane (out-of-range offsets for no-ops), and the loads of the next plane
// are in flight while the current one computes.
//
// LDS: two plane slots each of the sensitivity (FP64) and s (compute
// type), then the 43 plane slots of the adjoint ring (TbzRing<-1>) of
// (ox + 2) x (oy + 2) values. TB threads (256, 512 or, below FP64, 768:
// the smallest that covers the region's cells) take one cell each of a plane.
template <class S, class T, class A, int TB>
__global__ __launch_bounds__(TB) void k_adjoint_tbz(const A* __restrict__ nu_in, A* __restrict__ nu_out,
                                                    const T* __restrict__ rseg, size_t slot, long kseg,
                                                    const T* __restrict__ sfield, double* __restrict__ sens, Geo g,
                                                    Phys ph, Obj ob, long k_hi, long ns, long dW, double wgt, int ox,
                                                    int oy, int oz, int tiles_x, int tiles_y) {
    using L = D3Q19;
    constexpr int RS = record_size<L>();
    extern __shared__ unsigned char lds_raw[];
    const int LW = ox + 2, LH = oy + 2, psz = LW * LH;
    double* dsring = reinterpret_cast<double*>(lds_raw);
    T* sring = reinterpret_cast<T*>(dsring + 2 * psz);
    A* ring = reinterpret_cast<A*>(sring + 2 * psz);
    using RG = TbzRing<-1>;
    const int b = xcd_block();
    const int tx = b % tiles_x, ty = (b / tiles_x) % tiles_y, tz = b / (tiles_x * tiles_y);
    const int x0 = tx * ox - 1, y0 = ty * oy - 1;
    const int zs = tz * oz, nzc = min(oz, g.nz - zs);
    const int N = g.N, nxy = g.nx * g.ny;
    const size_t rbytes = (size_t)RS * N * sizeof(T), abytes = (size_t)L::Q * N * sizeof(A);
    const BufRsrc rR1 = buf_rsrc(rseg + (size_t)(k_hi - 2 - kseg) * slot, rbytes);   // record of f^{k_hi - 1}
    const BufRsrc rR2 = buf_rsrc(rseg + (size_t)(k_hi - 3 - kseg) * slot, rbytes);   // record of f^{k_hi - 2}
    const BufRsrc rnu = buf_rsrc(nu_in, abytes);
    const BufRsrc rout = buf_rsrc(nu_out, abytes);
    const BufRsrc rs = buf_rsrc(sfield, (size_t)N * sizeof(T));
    const BufRsrc rsens = buf_rsrc(sens, (size_t)N * sizeof(double));
    const double w1 = (k_hi > ns && (k_hi - ns) % dW == 0) ? wgt : 0.0;
    const double w2 = (k_hi - 1 > ns && (k_hi - 1 - ns) % dW == 0) ? wgt : 0.0;

    // this thread's cell of the region (step 1) and of the tile (step 2)
    const TbPhase p1 = tb_phase(g, 0, LW, LH, x0, y0, false);
    const TbPhase p2 = tb_phase(g, 1, LW, LH, x0, y0, true);
    const TbCell none = {1, 1, 0, 0, 0, LW + 1};
    TbCell c1 = none, c2 = none;
    const int i = (int)threadIdx.x;
    const bool v1 = i < p1.count, v2 = i < p2.count;
    const bool f1 = v1 && tb_cell(g, i, p1, LW, x0, y0, c1);
    const bool f2 = v2 && tb_cell(g, i, p2, LW, x0, y0, c2);
    const int o1 = f1 ? open_code_xy(g, c1.x, c1.y) : 0;
    const int o2 = f2 ? open_code_xy(g, c2.x, c2.y) : 0;
    const T u1 = o1 ? (T)g.u_in[c1.y] : (T)0;
    const T u2 = o2 ? (T)g.u_in[c2.y] : (T)0;
    const bool own1 = v1 && tb_owned(g, c1, 1, ox, oy, x0, y0);

    auto level_z = [&](int j, int& z) {
        z = zs - 1 + j;
        if (j < 0 || j > nzc + 1) return false;
        if (g.per_z) {
            z = z < 0 ? z + g.nz : (z >= g.nz ? z - g.nz : z);
            return true;
        }
        return z >= 0 && z < g.nz;
    };
    // step-1 inputs of a level: pre-state record, nu_hat gather, s
    struct In1 {
        T r[RS];
        A nk[L::Q];
        T s;
    };
    // step-2 inputs of a level: pre-state record and the old sensitivity
    struct In2 {
        T r[RS];
        double sold;
    };
    auto load1 = [&](int j, In1& in) {
        int z;
        const bool ok = level_z(j, z);
        const int zc = ok ? z : 0;
        const bool live = ok && v1;
        const unsigned n = (unsigned)(zc * nxy + c1.n);
        const bool zf = !g.per_z && (zc == 0 || zc == g.nz - 1);
#pragma unroll
        for (int q = 0; q < RS; ++q)
            buf_ld(rR1, live ? ((unsigned)q * N + n) * (unsigned)sizeof(T) : BUF_OOB, in.r[q]);
        unsigned e[L::Q];
        gather_index<L>(g, (int)n, c1.x, c1.y, zc, o1 != 0 && !zf, e);
#pragma unroll
        for (int a = 0; a < L::Q; ++a)
            buf_ld(rnu, live && e[a] != GATHER_ZERO ? e[a] * (unsigned)sizeof(A) : BUF_OOB, in.nk[a]);
        buf_ld(rs, live ? (unsigned)n * (unsigned)sizeof(T) : BUF_OOB, in.s);
    };
    auto load2 = [&](int k, In2& in) {
        const bool ok = k >= 1 && k <= nzc;
        const int z = ok ? zs + k - 1 : 0;
        const bool live = ok && v2;
        const unsigned n = (unsigned)(z * nxy + c2.n);
#pragma unroll
        for (int q = 0; q < RS; ++q)
            buf_ld(rR2, live ? ((unsigned)q * N + n) * (unsigned)sizeof(T) : BUF_OOB, in.r[q]);
        buf_ld(rsens, live ? n * 8u : BUF_OOB, in.sold);
    };
    // one adjoint node update: moments of the pre-state (post-boundary),
    // kappa -> mu, ds
    auto update = [&](const T (&r)[RS], const T (&kap)[L::Q], T s, int oc, T u0, int x, int y, int z, double w,
                      T (&mu)[L::Q]) {
        Moments<L, T> m;
        record_moments<L, T>(r, ph, m);
        MomentGrad<L, T> gr;
        gr.gr = 0;
#pragma unroll
        for (int p = 0; p < L::D; ++p) gr.gj[p] = 0;
#pragma unroll
        for (int q = 0; q < Sym<L::D>::K; ++q) gr.GP[q] = 0;
        const T ds = collide_adjoint<L, T>(m, ph, s, kap, gr);
        if (w != 0.0) adjoint_source<L, T>(ob, ph, x, y, z, s, m, w, gr);
        expand<L, T>(m, gr, mu);
        if (oc) zou_he_adjoint_rows<L, T>(oc, u0, mu);
        return ds;
    };
    auto step1 = [&](int j, const In1& in) {
        int z;
        if (!level_z(j, z)) return;
        const bool zf = !g.per_z && (z == 0 || z == g.nz - 1);
        const int oc = zf ? 0 : o1;
        const int s1 = (j + 6) % 2;
        if (!v1) return;
        T kap[L::Q], mu[L::Q];
#pragma unroll
        for (int a = 0; a < L::Q; ++a) kap[a] = (T)in.nk[a];
        const T ds = update(in.r, kap, in.s, oc, u1, c1.x, c1.y, z, w1, mu);
#pragma unroll
        for (int a = 0; a < L::Q; ++a) ring[RG::plane(a, j) * psz + c1.cell] = (A)mu[a];
        sring[s1 * psz + c1.cell] = in.s;
        if (own1) dsring[s1 * psz + c1.cell] = (double)ds;
        if (f1) {
            // ghost cells of the adjoint wall rule (0 on an open node)
            if (oc) {
#pragma unroll
                for (int a = 0; a < L::Q; ++a) mu[a] = (T)0;
            }
            tbz_ghosts<A, T, -1>(g, ring, psz, LW, LH, j, c1, mu);
        }
    };
    auto step2 = [&](int k, const In2& in) {
        const bool ok = k >= 1 && k <= nzc;
        const int z = ok ? zs + k - 1 : 0;
        const int n = z * nxy + c2.n;
        T mu[L::Q];
        double snew = 0.0;
#pragma unroll
        for (int a = 0; a < L::Q; ++a) mu[a] = (T)0;
        if (ok) {
            const bool zlo = !g.per_z && z == 0, zhi = !g.per_z && z == g.nz - 1;
            const int oc = (zlo || zhi) ? 0 : o2;
            const int s0 = (k + 6) % 2;
            int off[L::Q];   // uniform gather offset of each direction, relative to the cell
#pragma unroll
            for (int a = 0; a < L::Q; ++a) {
                const int shift = L::cy[a] * LW + L::cx[a];
                // the target plane is k + c_az; beyond a z wall, the node's own opp(a)
                const bool refl = (L::cz[a] > 0 && zhi) || (L::cz[a] < 0 && zlo);
                off[a] = refl ? RG::plane(L::opp[a], k) * psz : RG::plane(a, k + L::cz[a]) * psz + shift;
            }
            T kap[L::Q];
#pragma unroll
            for (int a = 0; a < L::Q; ++a) kap[a] = (T)ring[off[a] + c2.cell];
            const T ds = update(in.r, kap, sring[s0 * psz + c2.cell], oc, u2, c2.x, c2.y, z, w2, mu);
            snew = (in.sold + dsring[s0 * psz + c2.cell]) + (double)ds;
        }
        const bool live = ok && v2;
#pragma unroll
        for (int a = 0; a < L::Q; ++a)
            buf_st(rout, live ? ((unsigned)a * N + (unsigned)n) * (unsigned)sizeof(A) : BUF_OOB, (A)mu[a]);
        buf_st(rsens, live ? (unsigned)n * 8u : BUF_OOB, snew);
    };
    In1 a1, b1;
    In2 a2, b2;
#pragma unroll
    for (int q = 0; q < RS; ++q) a1.r[q] = b1.r[q] = a2.r[q] = b2.r[q] = (T)0;
#pragma unroll
    for (int a = 0; a < L::Q; ++a) a1.nk[a] = b1.nk[a] = (A)0;
    a1.s = b1.s = (T)0;
    a2.sold = b2.sold = 0.0;
    if constexpr (sizeof(A) == 4 && TB <= 512) {
        // ring level j: step 1 of level j from its input set, the step-1
        // loads of level j + 2 into that set, then step 2 of level j - 1
        // and the step-2 loads of level j + 1 into its set. Two sets of each
        // keep the loads of two levels in flight; the loop is unrolled by
        // two so that each set has fixed registers, and starts at level -2
        // (only loads) so that every pass issues the same memory operations.
        auto pass = [&](int j, In1& i1, In2& i2) {
            step1(j, i1);
            load1(j + 2, i1);
            lds_barrier();
            step2(j - 1, i2);
            load2(j + 1, i2);
            lds_barrier();
        };
        for (int j = -2; j <= nzc + 1; j += 2) {
            pass(j, a1, b2);
            pass(j + 1, b1, a2);
        }
    } else {
        // FP64, and 768 threads (no registers for a second set): one level
        // ahead, from -1
        for (int j = -1; j <= nzc + 1; ++j) {
            step1(j, a1);
            load1(j + 1, a1);
            lds_barrier();
            step2(j - 1, a2);
            load2(j, a2);
            lds_barrier();
        }
    }
}

// Per-sample sums of the block partials in a fixed order (deterministic).
__global__ __launch_bounds__(BLOCK) void k_reduce_samples(const double* __restrict__ partials, long nblocks,
                                                          double* __restrict__ samples) {
    const double* p = partials + (long)blockIdx.x * nblocks * 3;
    double v[3] = {0.0, 0.0, 0.0};
    for (long b = threadIdx.x; b < nblocks; b += BLOCK) {
        v[0] += p[3 * b + 0];
        v[1] += p[3 * b + 1];
        v[2] += p[3 * b + 2];
    }
    block_sum<3>(v, samples + 3 * (long)blockIdx.x);
}

// Window sums: acc[c] = weight * sum over samples, in sample order.
__global__ void k_window_sum(const double* __restrict__ samples, int nsamples, double weight,
                             double* __restrict__ acc) {
    const int c = threadIdx.x;
    if (c >= 3) return;
    double a = 0.0;
    for (int i = 0; i < nsamples; ++i) a += samples[3 * i + c];
    acc[c] = c < 2 ? weight * a : a;
}

// s(gamma): linear, or the paper's convex interpolation with phi = 1 - gamma.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_design(const double* __restrict__ gamma, T* __restrict__ s, long N,
                                                  int map, double q) {
    const int n = (int)(blockIdx.x * BLOCK + threadIdx.x);
    if (n >= N) return;
    const double gm = gamma[n];
    double v;
    if (map == 0) {
        v = gm;
    } else {
        const double phi = 1.0 - gm;
        v = 0.5 * (1.0 - phi * (1.0 + q) / (phi + q));
    }
    s[n] = (T)v;
}

// dJ/dgamma = s'(gamma) * dJ/ds (Eq. sensitivity, chain rule through s).
__global__ __launch_bounds__(BLOCK) void k_finalize(const double* __restrict__ gamma,
                                                    const double* __restrict__ sens, double* __restrict__ out,
                                                    long N, int map, double q) {
    const int n = (int)(blockIdx.x * BLOCK + threadIdx.x);
    if (n >= N) return;
    double d = 1.0;
    if (map != 0) {
        const double phi = 1.0 - gamma[n];
        d = 0.5 * q * (1.0 + q) / ((phi + q) * (phi + q));
    }
    out[n] = d * sens[n];
}

__global__ __launch_bounds__(BLOCK) void k_fill(double* __restrict__ p, long n, double v) {
    const long i = (long)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) p[i] = v;
}

// Block partials of sum (a - b)^2 (each block strides over the values).
__global__ __launch_bounds__(BLOCK) void k_sq_diff_parts(const double* __restrict__ a, const double* __restrict__ b,
                                                         long n, double* __restrict__ parts) {
    double v[1] = {0.0};
    for (long i = (long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long)gridDim.x * BLOCK) {
        const double d = a[i] - b[i];
        v[0] += d * d;
    }
    block_sum<1>(v, parts + blockIdx.x);
}

__global__ __launch_bounds__(BLOCK) void k_sum_parts(const double* __restrict__ parts, int nparts,
                                                     double* __restrict__ out) {
    double v[1] = {0.0};
    for (int i = (int)threadIdx.x; i < nparts; i += BLOCK) v[0] += parts[i];
    block_sum<1>(v, out);
}

// sens[node] += field[i], i the node's index in the accumulator box.
__global__ __launch_bounds__(BLOCK) void k_box_add(double* __restrict__ sens, const double* __restrict__ field,
                                                   Geo g, Obj ob) {
    const int i = (int)(blockIdx.x * BLOCK + threadIdx.x);
    if (i >= ob.nb) return;
    const int x = ob.ax0 + i % ob.anx;
    const int r = i / ob.anx;
    const int y = ob.ay0 + r % ob.any;
    const int z = ob.az0 + r / ob.any;
    sens[((long)z * g.ny + y) * g.nx + x] += field[i];
}

__global__ __launch_bounds__(BLOCK) void k_copy_bytes(const unsigned int* __restrict__ a,
                                                      unsigned int* __restrict__ b, long nwords) {
    const long i = (long)blockIdx.x * BLOCK + threadIdx.x;
    if (i < nwords) b[i] = a[i];
}

// ------------------------------------------------------------ launchers

static inline dim3 grid_for(long n) { return dim3((unsigned)((n + BLOCK - 1) / BLOCK)); }

// Compile-time plane strides of the blocked kernels' LDS buffers (values of
// the compute type); each keeps the largest immediate LDS offset of a node,
// 8 planes, below 64 KB. Regions of more than 512 nodes use the smallest
// that holds them when the LDS allows; other launches use their region size.
static constexpr int TB_PS32[2] = {1856, 2040};
static constexpr int TB_PS64 = 1020;
static constexpr int TB_PS16[2] = {1856, 3584};   // FP16 LDS state (FP16S forward)

template <class S, class T, bool SAMPLE, bool WPRE, int TB, bool ALLOUT, int PS>
static void launch_tb_ps(const StepLaunch& a, int tiles_x, int tiles_y, size_t lds) {
    hipLaunchKernelGGL((k_step_tb<S, T, SAMPLE, WPRE, TB, ALLOUT, PS>), dim3(tiles_x * tiles_y), dim3(TB), lds,
                       a.stream, (const S*)a.gin, (S*)a.gout, (S*)a.pre, (const T*)a.s, a.geo, a.ph, a.ob,
                       a.partials, a.part_stride, a.nsteps, a.tile_x, a.tile_y, tiles_x, (T*)a.rec,
                       a.rec_slot / sizeof(T));
}

template <class S, class T, bool SAMPLE, bool WPRE, bool ALLOUT>
static void launch_tb(const StepLaunch& a) {
    const Geo& g = a.geo;
    const int tiles_x = (g.nx + a.tile_x - 1) / a.tile_x;
    const int tiles_y = (g.ny + a.tile_y - 1) / a.tile_y;
    using LT = typename TbLds<S, T>::type;
    const size_t lds = tb_lds_bytes(a.nsteps, a.tile_x, a.tile_y, sizeof(LT), sizeof(T));
    const int ps = tb_plane(a.nsteps, a.tile_x, a.tile_y, sizeof(LT), sizeof(T), 0);
    if (tb_threads(a.nsteps, a.tile_x, a.tile_y) == 512) {
        launch_tb_ps<S, T, SAMPLE, WPRE, 512, ALLOUT, 0>(a, tiles_x, tiles_y, lds);
        return;
    }
    if constexpr (sizeof(LT) == 2) {
        if (ps == TB_PS16[0]) return launch_tb_ps<S, T, SAMPLE, WPRE, 1024, ALLOUT, TB_PS16[0]>(a, tiles_x, tiles_y, lds);
        if (ps == TB_PS16[1]) return launch_tb_ps<S, T, SAMPLE, WPRE, 1024, ALLOUT, TB_PS16[1]>(a, tiles_x, tiles_y, lds);
    } else if constexpr (sizeof(T) == 4) {
        if (ps == TB_PS32[0]) return launch_tb_ps<S, T, SAMPLE, WPRE, 1024, ALLOUT, TB_PS32[0]>(a, tiles_x, tiles_y, lds);
        if (ps == TB_PS32[1]) return launch_tb_ps<S, T, SAMPLE, WPRE, 1024, ALLOUT, TB_PS32[1]>(a, tiles_x, tiles_y, lds);
    } else {
        if (ps == TB_PS64) return launch_tb_ps<S, T, SAMPLE, WPRE, 1024, ALLOUT, TB_PS64>(a, tiles_x, tiles_y, lds);
    }
    launch_tb_ps<S, T, SAMPLE, WPRE, 1024, ALLOUT, 0>(a, tiles_x, tiles_y, lds);
}

template <class S, class T, bool SAMPLE, bool WPRE, bool REC = false>
static hipError_t launch_tbz(const StepLaunch& a) {
    using LT = typename TbLds<S, T>::type;
    const Geo& g = a.geo;
    const int tiles_x = (g.nx + a.tile_x - 1) / a.tile_x;
    const int tiles_y = (g.ny + a.tile_y - 1) / a.tile_y;
    const int tiles_z = (g.nz + a.tile_z - 1) / a.tile_z;
    const size_t lds = tbz_lds_bytes(a.tile_x, a.tile_y, sizeof(LT), sizeof(T));
    const dim3 grid(tiles_x * tiles_y * tiles_z);
    const int nt = tbz_threads(a.tile_x, a.tile_y);   // one cell per thread
#define LBM_TBZ(TB, U)                                                                                          \
    hipLaunchKernelGGL((k_step_tbz<S, T, SAMPLE, WPRE, TB, U, REC>), grid, dim3(TB), lds, a.stream,             \
                       (const S*)a.gin, (S*)a.gout, (S*)a.pre, (const T*)a.s, g, a.ph, a.ob, a.partials,        \
                       a.part_stride, a.tile_x, a.tile_y, a.tile_z, tiles_x, tiles_y, (T*)a.rec,                \
                       a.rec_slot / sizeof(T))
    if (nt == 256) {
        LBM_TBZ(256, 1);
    } else if (nt == 512) {
        LBM_TBZ(512, 1);
    } else if constexpr (sizeof(T) == 4) {
        if (nt == 768) {
            LBM_TBZ(768, 1);
        } else {
            LBM_TBZ(1024, 1);
        }
    } else {
        return hipErrorInvalidValue;   // FP64 regions above 512 cells do not fit the LDS
    }
#undef LBM_TBZ
    return hipGetLastError();
}

template <class L, class S, class T>
static hipError_t step_t(const StepLaunch& a) {
    const Geo& g = a.geo;
    const S* gin = (const S*)a.gin;
    S* gout = (S*)a.gout;
    S* pre = (S*)a.pre;
    const T* sf = (const T*)a.s;
    if (L::D == 3 && a.nsteps > 1) {
        if (a.nsteps != 2) return hipErrorInvalidValue;
        if (a.rec) {
            if (a.sample || pre) return hipErrorInvalidValue;
            return launch_tbz<S, T, false, false, true>(a);
        }
        if (a.sample) return pre ? launch_tbz<S, T, true, true>(a) : launch_tbz<S, T, true, false>(a);
        return pre ? launch_tbz<S, T, false, true>(a) : launch_tbz<S, T, false, false>(a);
    }
    if (a.nsteps > 1) {
        if (L::D != 2) return hipErrorInvalidValue;
        if (a.rec) {
            if (a.sample || pre) return hipErrorInvalidValue;
            launch_tb<S, T, false, false, true>(a);
        } else if (a.sample) {
            if (pre) launch_tb<S, T, true, true, false>(a);
            else launch_tb<S, T, true, false, false>(a);
        } else {
            if (pre) launch_tb<S, T, false, true, false>(a);
            else launch_tb<S, T, false, false, false>(a);
        }
        return hipGetLastError();
    }
    dim3 gr = grid_for(g.N);
    const int ps = a.part_stride;
    if (a.rec) {
        if (a.sample || pre) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_step<L, S, T, false, false, true>), gr, dim3(BLOCK), 0, a.stream, gin, gout, pre, sf, g,
                           a.ph, a.ob, a.partials, ps, (T*)a.rec);
    } else if (a.sample) {
        if (pre) hipLaunchKernelGGL((k_step<L, S, T, true, true>), gr, dim3(BLOCK), 0, a.stream, gin, gout, pre, sf, g, a.ph, a.ob, a.partials, ps);
        else hipLaunchKernelGGL((k_step<L, S, T, true, false>), gr, dim3(BLOCK), 0, a.stream, gin, gout, pre, sf, g, a.ph, a.ob, a.partials, ps);
    } else {
        if (pre) hipLaunchKernelGGL((k_step<L, S, T, false, true>), gr, dim3(BLOCK), 0, a.stream, gin, gout, pre, sf, g, a.ph, a.ob, a.partials, ps);
        else hipLaunchKernelGGL((k_step<L, S, T, false, false>), gr, dim3(BLOCK), 0, a.stream, gin, gout, pre, sf, g, a.ph, a.ob, a.partials, ps);
    }
    return hipGetLastError();
}

template <class L, class S, class T, class A>
static hipError_t adj_t(const AdjLaunch& a) {
    const Geo& g = a.geo;
    dim3 gr = grid_for(g.N);
    const A* nin = (const A*)a.nu_in;
    A* nout = (A*)a.nu_out;
    const S* st = (const S*)a.state;
    const T* sf = (const T*)a.s;
    if (L::D == 3 && a.nsteps > 1) {
        if (a.seed || a.direct || a.nsteps != 2) return hipErrorInvalidValue;
        const int tiles_x = (g.nx + a.tile_x - 1) / a.tile_x;
        const int tiles_y = (g.ny + a.tile_y - 1) / a.tile_y;
        const int tiles_z = (g.nz + a.tile_z - 1) / a.tile_z;
        const size_t lds = adj_tbz_lds_bytes(a.tile_x, a.tile_y, sizeof(A), sizeof(T));
        const dim3 grid(tiles_x * tiles_y * tiles_z);
        if (!a.rec) return hipErrorInvalidValue;          // the segments are moment records
        const T* gs = (const T*)a.gseg;
        const size_t slot = a.slot / sizeof(T);
#define LBM_ADJ_TBZ(TBV)                                                                                      \
    hipLaunchKernelGGL((k_adjoint_tbz<S, T, A, TBV>), grid, dim3(TBV), lds, a.stream, nin, nout, gs, slot,      \
                       a.kseg, sf, a.sens, g, a.ph, a.ob, a.k_hi, a.ns, a.dW, a.wgt, a.tile_x, a.tile_y,        \
                       a.tile_z, tiles_x, tiles_y)
        const int nt = tbz_threads(a.tile_x, a.tile_y);
        if (nt == 256) {
            LBM_ADJ_TBZ(256);
        } else if (nt == 512) {
            LBM_ADJ_TBZ(512);
        } else if constexpr (sizeof(A) == 4) {
            if (nt == 768) {
                LBM_ADJ_TBZ(768);
            } else {
                return hipErrorInvalidValue;   // regions above 768 cells (register budget)
            }
        } else {
            return hipErrorInvalidValue;       // FP64 regions above 512 cells do not fit the LDS
        }
#undef LBM_ADJ_TBZ
        return hipGetLastError();
    }
    if (L::D == 2 && a.nsteps > 1) {
        if (a.seed || a.direct) return hipErrorInvalidValue;
        const int tiles_x = (g.nx + a.tile_x - 1) / a.tile_x;
        const int tiles_y = (g.ny + a.tile_y - 1) / a.tile_y;
        const size_t lds = adj_tb_lds_bytes(a.nsteps, a.tile_x, a.tile_y, sizeof(T));
        const int ps = tb_plane(a.nsteps, a.tile_x, a.tile_y, sizeof(T), sizeof(T), (size_t)a.tile_x * a.tile_y * 8);
        const int tb = tb_threads(a.nsteps, a.tile_x, a.tile_y);
        const dim3 grid(tiles_x * tiles_y);
        if (!a.rec) return hipErrorInvalidValue;          // the segments are moment records
        const T* gs = (const T*)a.gseg;
        const size_t slot = a.slot / sizeof(T);
#define LBM_ADJ_TB(TBV, PSV)                                                                                \
    hipLaunchKernelGGL((k_adjoint_tb<S, T, A, TBV, PSV>), grid, dim3(TBV), lds, a.stream, nin, nout, gs, slot, \
                       a.kseg, sf, a.sens, g, a.ph, a.ob, a.k_hi, a.ns, a.dW, a.wgt, a.nsteps, a.tile_x,       \
                       a.tile_y, tiles_x)
        bool done = false;
        if (tb == 512) {
            LBM_ADJ_TB(512, 0);
            done = true;
        } else if constexpr (sizeof(T) == 4) {
            if (ps == TB_PS32[0]) {
                LBM_ADJ_TB(1024, TB_PS32[0]);
                done = true;
            } else if (ps == TB_PS32[1]) {
                LBM_ADJ_TB(1024, TB_PS32[1]);
                done = true;
            }
        } else {
            if (ps == TB_PS64) {
                LBM_ADJ_TB(1024, TB_PS64);
                done = true;
            }
        }
        if (!done) LBM_ADJ_TB(1024, 0);
#undef LBM_ADJ_TB
    } else if (a.seed) {
        hipLaunchKernelGGL((k_adjoint<L, S, T, A, false, true>), gr, dim3(BLOCK), 0, a.stream, nin, nout, st, sf, a.sens, g, a.ph, a.ob, a.src_w);
    } else if (a.direct) {
        hipLaunchKernelGGL((k_adjoint<L, S, T, A, true, false>), gr, dim3(BLOCK), 0, a.stream, nin, nout, st, sf, a.sens, g, a.ph, a.ob, a.src_w);
    } else if (a.rec) {
        hipLaunchKernelGGL((k_adjoint<L, S, T, A, false, false, true>), gr, dim3(BLOCK), 0, a.stream, nin, nout, st, sf, a.sens, g, a.ph, a.ob, a.src_w);
    } else {
        return hipErrorInvalidValue;   // a transition reads a checkpoint or a moment record
    }
    return hipGetLastError();
}

template <class L, class S, class T>
static hipError_t aux_t(const AuxLaunch& a) {
    const Geo& g = a.geo;
    dim3 gr = grid_for(g.N);
    switch (a.op) {
        case AUX_COLLIDE:
            hipLaunchKernelGGL((k_collide<L, S, T>), gr, dim3(BLOCK), 0, a.stream, (const S*)a.src, (S*)a.dst, (const T*)a.s, g, a.ph);
            break;
        case AUX_INIT_EQ:
            hipLaunchKernelGGL((k_init_eq<L, S>), gr, dim3(BLOCK), 0, a.stream, (S*)a.dst, g, a.rho0, a.umode);
            break;
        case AUX_EXPORT_DIRECT:
            hipLaunchKernelGGL((k_export<L, S, true, false>), gr, dim3(BLOCK), 0, a.stream, (const S*)a.src, (double*)a.dst, g);
            break;
        case AUX_EXPORT_PULL:
            hipLaunchKernelGGL((k_export<L, S, false, false>), gr, dim3(BLOCK), 0, a.stream, (const S*)a.src, (double*)a.dst, g);
            break;
        case AUX_FIELDS_DIRECT:
            hipLaunchKernelGGL((k_export<L, S, true, true>), gr, dim3(BLOCK), 0, a.stream, (const S*)a.src, (double*)a.dst, g);
            break;
        case AUX_FIELDS_PULL:
            hipLaunchKernelGGL((k_export<L, S, false, true>), gr, dim3(BLOCK), 0, a.stream, (const S*)a.src, (double*)a.dst, g);
            break;
        case AUX_IMPORT:
            hipLaunchKernelGGL((k_import<L, S>), gr, dim3(BLOCK), 0, a.stream, (const double*)a.src, (S*)a.dst, g);
            break;
        case AUX_DESIGN:
            hipLaunchKernelGGL((k_design<T>), gr, dim3(BLOCK), 0, a.stream, (const double*)a.src, (T*)a.dst, g.N, a.map, a.q);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Dispatch on (lattice, precision): F64 stores and computes in double;
// F32 stores float; F16S stores _Float16; both compute in float.
#define LBM_DISPATCH(FN, ARG)                                                                        \
    switch (ARG.lattice * 3 + ARG.prec) {                                                           \
        case 0: return FN<D2Q9, double, double>(ARG);                                               \
        case 1: return FN<D2Q9, float, float>(ARG);                                                 \
        case 2: return FN<D2Q9, _Float16, float>(ARG);                                              \
        case 3: return FN<D3Q19, double, double>(ARG);                                              \
        case 4: return FN<D3Q19, float, float>(ARG);                                                \
        case 5: return FN<D3Q19, _Float16, float>(ARG);                                             \
        default: return hipErrorInvalidValue;                                                        \
    }

hipError_t launch_step(const StepLaunch& a) { LBM_DISPATCH(step_t, a) }

hipError_t launch_aux(const AuxLaunch& a) { LBM_DISPATCH(aux_t, a) }

hipError_t launch_adjoint(const AdjLaunch& a) {
    switch (a.lattice * 3 + a.prec) {
        case 0: return adj_t<D2Q9, double, double, double>(a);
        case 1: return adj_t<D2Q9, float, float, float>(a);
        case 2: return adj_t<D2Q9, _Float16, float, float>(a);
        case 3: return adj_t<D3Q19, double, double, double>(a);
        case 4: return adj_t<D3Q19, float, float, float>(a);
        case 5: return adj_t<D3Q19, _Float16, float, float>(a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce(const double* partials, long nblocks, int nsamples, double* samples,
                         double weight, double* acc, hipStream_t stream) {
    hipLaunchKernelGGL(k_reduce_samples, dim3(nsamples), dim3(BLOCK), 0, stream, partials, nblocks, samples);
    hipLaunchKernelGGL(k_window_sum, dim3(1), dim3(64), 0, stream, samples, nsamples, weight, acc);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* gamma, const double* sens, double* out, long N, int map, double q,
                           hipStream_t stream) {
    hipLaunchKernelGGL(k_finalize, grid_for(N), dim3(BLOCK), 0, stream, gamma, sens, out, N, map, q);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, long n, double v, hipStream_t stream) {
    hipLaunchKernelGGL(k_fill, grid_for(n), dim3(BLOCK), 0, stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_sq_diff_sum(const double* a, const double* b, long n, double* parts, int nparts, double* out,
                              hipStream_t stream) {
    long nblk = (n + BLOCK - 1) / BLOCK;
    if (nblk > nparts) nblk = nparts;
    if (nblk < 1) nblk = 1;
    hipLaunchKernelGGL(k_sq_diff_parts, dim3((unsigned)nblk), dim3(BLOCK), 0, stream, a, b, n, parts);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(BLOCK), 0, stream, parts, (int)nblk, out);
    return hipGetLastError();
}

hipError_t launch_box_add(double* sens, const double* field, const Geo& g, const Obj& ob, hipStream_t stream) {
    hipLaunchKernelGGL(k_box_add, grid_for(ob.nb), dim3(BLOCK), 0, stream, sens, field, g, ob);
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t stream) {
    const long nwords = (long)(bytes / 4);
    hipLaunchKernelGGL(k_copy_bytes, grid_for(nwords), dim3(BLOCK), 0, stream, (const unsigned int*)src,
                       (unsigned int*)dst, nwords);
    return hipGetLastError();
}

long blocks_for(long n) { return (n + BLOCK - 1) / BLOCK; }

// Plane stride (elements) of a blocked launch: LDS state elements of lsize
// bytes, s plane and row cache of vsize-byte values, and `extra` bytes more.
int tb_plane(int nsteps, int tile_x, int tile_y, size_t lsize, size_t vsize, size_t extra) {
    const long lw = tile_x + 2 * (nsteps - 1), lh = tile_y + 2 * (nsteps - 1);
    const long region = lw * lh;
    extra += lh * (vsize + 2);   // row cache
    auto fits = [&](long ps) { return (size_t)ps * (2 * 9 * lsize + vsize) + extra <= TB_LDS_MAX; };
    if (region > 512) {
        if (lsize == 2) {
            for (int ps : TB_PS16)
                if (ps >= region && fits(ps)) return ps;
        } else if (lsize == 4) {
            for (int ps : TB_PS32)
                if (ps >= region && fits(ps)) return ps;
        } else if (lsize == 8) {
            if (TB_PS64 >= region && fits(TB_PS64)) return TB_PS64;
        }
    }
    return (int)region;
}

size_t tb_lds_bytes(int nsteps, int tile_x, int tile_y, size_t lsize, size_t vsize) {
    const size_t lh = tile_y + 2 * (nsteps - 1);
    // two state buffers and the s plane, then the row cache
    const size_t ps = tb_plane(nsteps, tile_x, tile_y, lsize, vsize, 0);
    return ps * (2 * 9 * lsize + vsize) + lh * (vsize + 2);
}

size_t adj_tb_lds_bytes(int nsteps, int tile_x, int tile_y, size_t vsize) {
    // sensitivity sums of the tile (FP64), then the forward kernel's layout
    const size_t sens = (size_t)tile_x * tile_y * 8;
    const size_t lh = tile_y + 2 * (nsteps - 1);
    const size_t ps = tb_plane(nsteps, tile_x, tile_y, vsize, vsize, sens);
    return sens + ps * (2 * 9 * vsize + vsize) + lh * (vsize + 2);
}

size_t tb_lds_bytes_prec(int nsteps, int tile_x, int tile_y, int prec) {
    return prec == 0 ? tb_lds_bytes(nsteps, tile_x, tile_y, 8, 8)
                     : tb_lds_bytes(nsteps, tile_x, tile_y, prec == 1 ? 4 : 2, 4);
}

size_t tbz_lds_bytes(int tile_x, int tile_y, size_t lsize, size_t vsize) {
    // s values of two planes, then the plane slots of the ring
    const size_t psz = (size_t)(tile_x + 2) * (tile_y + 2);
    return psz * (2 * vsize + TbzRing<1>::PLANES * lsize);
}

size_t tbz_lds_bytes_prec(int tile_x, int tile_y, int prec) {
    return prec == 0 ? tbz_lds_bytes(tile_x, tile_y, 8, 8)
                     : tbz_lds_bytes(tile_x, tile_y, prec == 1 ? 4 : 2, 4);
}

int tbz_threads(int tile_x, int tile_y) {
    const long cells = (long)(tile_x + 2) * (tile_y + 2);
    return cells <= 256 ? 256 : (cells <= 512 ? 512 : (cells <= 768 ? 768 : 1024));
}

size_t adj_tbz_lds_bytes(int tile_x, int tile_y, size_t asize, size_t tsize) {
    // FP64 sensitivity and s of two planes, then the plane slots of the ring
    const size_t psz = (size_t)(tile_x + 2) * (tile_y + 2);
    return psz * (2 * 8 + 2 * tsize + TbzRing<-1>::PLANES * asize);
}


long tb_blocks(int nx, int ny, int tile_x, int tile_y) {
    return (long)((nx + tile_x - 1) / tile_x) * ((ny + tile_y - 1) / tile_y);
}

int tb_threads(int nsteps, int tile_x, int tile_y) {
    const long lw = tile_x + 2 * (nsteps - 1), lh = tile_y + 2 * (nsteps - 1);
    return lw * lh <= 512 ? 512 : 1024;
}

template <class S, class T, int NT, int PS>
static hipError_t tb_attr_fwd(int b) {
    const hipFuncAttribute at = hipFuncAttributeMaxDynamicSharedMemorySize;
    hipError_t e = hipFuncSetAttribute((const void*)k_step_tb<S, T, false, false, NT, false, PS>, at, b);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_step_tb<S, T, true, false, NT, false, PS>, at, b);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_step_tb<S, T, false, true, NT, false, PS>, at, b);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_step_tb<S, T, true, true, NT, false, PS>, at, b);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_step_tb<S, T, false, false, NT, true, PS>, at, b);
    return e;
}

template <class S, class T, class A, int NT, int PS>
static hipError_t tb_attr_adj(int b) {
    return hipFuncSetAttribute((const void*)k_adjoint_tb<S, T, A, NT, PS>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, b);
}

template <class S, class T, class A, int NT, int PS>
static hipError_t tb_attr(int b) {
    hipError_t e = tb_attr_fwd<S, T, NT, PS>(b);
    if (e == hipSuccess) e = tb_attr_adj<S, T, A, NT, PS>(b);
    return e;
}

template <class S, class T, int NT, int U>
static hipError_t tbz_attr(int b) {
    const hipFuncAttribute at = hipFuncAttributeMaxDynamicSharedMemorySize;
    hipError_t e = hipFuncSetAttribute((const void*)k_step_tbz<S, T, false, false, NT, U>, at, b);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_step_tbz<S, T, true, false, NT, U>, at, b);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_step_tbz<S, T, false, true, NT, U>, at, b);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_step_tbz<S, T, true, true, NT, U>, at, b);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_step_tbz<S, T, false, false, NT, U, true>, at, b);
    return e;
}

template <class S, class T, class A>
static hipError_t tb_attr_all(int b) {
    hipError_t e = hipFuncSetAttribute((const void*)k_adjoint_tbz<S, T, A, 256>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_adjoint_tbz<S, T, A, 512>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                b);
    if constexpr (sizeof(A) == 4) {
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_adjoint_tbz<S, T, A, 768>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, b);
    }
    if (e == hipSuccess) e = tbz_attr<S, T, 256, 1>(b);
    if (e == hipSuccess) e = tbz_attr<S, T, 512, 1>(b);
    if constexpr (sizeof(T) == 4) {
        if (e == hipSuccess) e = tbz_attr<S, T, 768, 1>(b);
        if (e == hipSuccess) e = tbz_attr<S, T, 1024, 1>(b);
    }
    if (e == hipSuccess) e = tb_attr<S, T, A, 512, 0>(b);
    if (e == hipSuccess) e = tb_attr<S, T, A, 1024, 0>(b);
    if constexpr (sizeof(S) == 2) {
        // forward kernels take the FP16 strides, the adjoint the FP32 ones
        if (e == hipSuccess) e = tb_attr_fwd<S, T, 1024, TB_PS16[0]>(b);
        if (e == hipSuccess) e = tb_attr_fwd<S, T, 1024, TB_PS16[1]>(b);
        if (e == hipSuccess) e = tb_attr_adj<S, T, A, 1024, TB_PS32[0]>(b);
        if (e == hipSuccess) e = tb_attr_adj<S, T, A, 1024, TB_PS32[1]>(b);
    } else if constexpr (sizeof(T) == 4) {
        if (e == hipSuccess) e = tb_attr<S, T, A, 1024, TB_PS32[0]>(b);
        if (e == hipSuccess) e = tb_attr<S, T, A, 1024, TB_PS32[1]>(b);
    } else {
        if (e == hipSuccess) e = tb_attr<S, T, A, 1024, TB_PS64>(b);
    }
    return e;
}

hipError_t tb_prepare(int prec) {
    // opt in to the LDS of a compute unit (beyond the default 64 KB) for the
    // blocked kernels; launches check their own size against TB_LDS_MAX
    const int b = (int)TB_LDS_MAX;
    if (prec == 0) return tb_attr_all<double, double, double>(b);
    if (prec == 1) return tb_attr_all<float, float, float>(b);
    return tb_attr_all<_Float16, float, float>(b);
}

}  // namespace lbm
