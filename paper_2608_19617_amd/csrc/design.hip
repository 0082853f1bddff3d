// Design update of the optimisation loop (include/lbm_design.h; Sec.
// "Topology optimization procedure", Algorithm "Optimization iteration"):
// density filter, Heaviside projection, volume fraction, the chain rule back
// to the design variables, and the projected-gradient step that stands in
// for MMA. Everything is FP64.
//
// The filter and its transpose are one LDS-tiled stencil kernel: a
// workgroup of 256 threads owns an output tile (32 x 8 in 2D, 8 x 8 x 4 in
// 3D), stages the tile grown by the halo H = ceil(r) - 1 in LDS, and sums
// the neighbours of each node over a list of (LDS offset, weight) pairs that
// the host builds once per context (the integer points of the ball |o| < r,
// weights r - |o|). The list is read with uniform loads. The filter pass
// also projects and writes the per-workgroup volume partials.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "launch.hpp"
#include "lbm_design.h"

// Scratch of lbm_design_map_noalloc: per-workgroup partials (volume sum and
// design-node count, two doubles per block) for at most DZ_NOALLOC_BLOCKS
// blocks, then the two final sums. Each GPU holds its own copy for the life
// of the process; host code never uses this name as an address (it is a
// host-side stand-in): it passes the address hipGetSymbolAddress returned
// for the current device.
constexpr int DZ_NOALLOC_BLOCKS = 65536;
static __device__ __align__(256) double scratch[2 * DZ_NOALLOC_BLOCKS + 32];

namespace lbm {
namespace {

constexpr int DZ_TB = 256;
constexpr int DZ_HMAX = 4;   // radius <= 5

template <int D>
struct DzTile;
template <>
struct DzTile<2> {
    static constexpr int X = 32, Y = 8, Z = 1;
};
template <>
struct DzTile<3> {
    static constexpr int X = 8, Y = 8, Z = 4;
};

template <int D>
constexpr int dz_region_max() {
    return (DzTile<D>::X + 2 * DZ_HMAX) * (DzTile<D>::Y + 2 * DZ_HMAX) * (D == 3 ? DzTile<D>::Z + 2 * DZ_HMAX : 1);
}

struct DzOff {
    int off;     // LDS offset of the neighbour relative to the node's cell
    int pad;
    double w;    // r - |o|
};

struct DzGeo {
    int nx, ny, nz, N;
    int H;                  // halo
    int rx, ry, rz;         // LDS region of a tile
    int tiles_x, tiles_y;
    int noff;
    const DzOff* offs;
};

enum DzMode { DZ_WSUM = 0, DZ_FILTER = 1, DZ_CHAIN = 2 };

// Block sum of NV doubles over DZ_TB threads into out[blockIdx * NV + k].
template <int NV>
__device__ __forceinline__ void dz_block_sum(double v[NV], double* out) {
    __shared__ double red[NV][DZ_TB / 64];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < DZ_TB / 64; ++w) s += red[k][w];
            out[(size_t)blockIdx.x * NV + k] = s;
        }
    }
}

// The stencil pass. Staged per region cell (0 outside the grid):
//   WSUM:   m                              -> out0 = W = sum_o w_o m(i+o)
//   FILTER: m x                            -> out0 = x~ (x off D), out1 =
//           gamma (H(x~) on D, base off D); volume partial sum_{D} gamma
//   CHAIN:  m H'(x~) g / W, m H'(x~) / (n_D W)
//                                          -> out0 = m sum_o w_o (first),
//                                             out1 = m sum_o w_o (second)
// with a = x (FILTER) or x~ (CHAIN), b = g = dJ/dgamma (CHAIN).
template <int D, int MODE>
__global__ __launch_bounds__(DZ_TB) void k_dz_stencil(DzGeo g, const unsigned char* __restrict__ mask,
                                                      const double* __restrict__ a, const double* __restrict__ b,
                                                      const double* __restrict__ W, const double* __restrict__ base,
                                                      double beta, double eta, double hn, double hd, double inv_nd,
                                                      double* __restrict__ out0, double* __restrict__ out1,
                                                      double* __restrict__ partials) {
    using TL = DzTile<D>;
    __shared__ double s0[dz_region_max<D>()];
    __shared__ double s1[MODE == DZ_CHAIN ? dz_region_max<D>() : 1];
    const int bidx = (int)blockIdx.x;
    const int btx = bidx % g.tiles_x, bty = (bidx / g.tiles_x) % g.tiles_y, btz = bidx / (g.tiles_x * g.tiles_y);
    const int x0 = btx * TL::X - g.H, y0 = bty * TL::Y - g.H, z0 = (D == 3 ? btz * TL::Z - g.H : 0);
    const int rcount = g.rx * g.ry * g.rz;
    for (int c = (int)threadIdx.x; c < rcount; c += DZ_TB) {
        const int lz = c / (g.rx * g.ry), r2 = c - lz * g.rx * g.ry;
        const int ly = r2 / g.rx, lx = r2 - ly * g.rx;
        const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        double v0 = 0.0, v1 = 0.0;
        if (x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz) {
            const int n = (z * g.ny + y) * g.nx + x;
            if (mask[n]) {
                if (MODE == DZ_WSUM) {
                    v0 = 1.0;
                } else if (MODE == DZ_FILTER) {
                    v0 = a[n];
                } else {
                    const double th = tanh(beta * (a[n] - eta));
                    const double dH = beta * (1.0 - th * th) * hd;
                    v0 = dH * b[n] / W[n];
                    v1 = dH * inv_nd / W[n];
                }
            }
        }
        s0[c] = v0;
        if (MODE == DZ_CHAIN) s1[c] = v1;
    }
    __syncthreads();
    const int t = (int)threadIdx.x;
    const int ox = t % TL::X, oy = (t / TL::X) % TL::Y, oz = t / (TL::X * TL::Y);
    const int x = btx * TL::X + ox, y = bty * TL::Y + oy, z = (D == 3 ? btz * TL::Z + oz : 0);
    const bool in = x < g.nx && y < g.ny && z < g.nz;
    double vol = 0.0;
    if (in) {
        const int n = (z * g.ny + y) * g.nx + x;
        const int cell = ((oz + (D == 3 ? g.H : 0)) * g.ry + (oy + g.H)) * g.rx + (ox + g.H);
        double acc0 = 0.0, acc1 = 0.0;
        for (int k = 0; k < g.noff; ++k) {
            const DzOff o = g.offs[k];
            acc0 += o.w * s0[cell + o.off];
            if (MODE == DZ_CHAIN) acc1 += o.w * s1[cell + o.off];
        }
        const bool m = mask[n] != 0;
        if (MODE == DZ_WSUM) {
            out0[n] = acc0;
        } else if (MODE == DZ_FILTER) {
            const double xt = m ? acc0 / W[n] : a[n];
            const double gam = m ? (hn + tanh(beta * (xt - eta))) * hd : base[n];
            out0[n] = xt;
            out1[n] = gam;
            if (m) vol = gam;
        } else {
            out0[n] = m ? acc0 : 0.0;
            if (out1) out1[n] = m ? acc1 : 0.0;
        }
    }
    if (MODE == DZ_FILTER) {
        double v[1] = {vol};
        dz_block_sum<1>(v, partials);
    }
}

// Per-block count of design nodes (as doubles).
__global__ __launch_bounds__(DZ_TB) void k_dz_count(const unsigned char* __restrict__ mask, int N,
                                                    double* __restrict__ partials) {
    const int n = (int)(blockIdx.x * DZ_TB + threadIdx.x);
    double v[1] = {(n < N && mask[n]) ? 1.0 : 0.0};
    dz_block_sum<1>(v, partials);
}

// Per-block largest |g| over D of two fields.
__global__ __launch_bounds__(DZ_TB) void k_dz_absmax(const unsigned char* __restrict__ mask,
                                                     const double* __restrict__ g0, const double* __restrict__ g1,
                                                     int N, double* __restrict__ partials) {
    __shared__ double red[2][DZ_TB / 64];
    const int n = (int)(blockIdx.x * DZ_TB + threadIdx.x);
    double v0 = 0.0, v1 = 0.0;
    if (n < N && mask[n]) {
        v0 = fabs(g0[n]);
        v1 = fabs(g1[n]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v0 = fmax(v0, __shfl_down(v0, o, 64));
        v1 = fmax(v1, __shfl_down(v1, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = v0;
        red[1][threadIdx.x >> 6] = v1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m0 = 0.0, m1 = 0.0;
        for (int w = 0; w < DZ_TB / 64; ++w) {
            m0 = fmax(m0, red[0][w]);
            m1 = fmax(m1, red[1][w]);
        }
        partials[2 * blockIdx.x] = m0;
        partials[2 * blockIdx.x + 1] = m1;
    }
}

// Final reduction of per-block partials (NV values each, nb blocks) in a
// fixed order: out[k] = sum (MAXR = 0) or max (MAXR = 1) over the blocks.
template <int NV, int MAXR>
__global__ __launch_bounds__(DZ_TB) void k_dz_final(const double* __restrict__ partials, int nb,
                                                    double* __restrict__ out) {
    __shared__ double red[NV][DZ_TB];
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int i = (int)threadIdx.x; i < nb; i += DZ_TB) {
            const double v = partials[(size_t)i * NV + k];
            s = MAXR ? fmax(s, v) : s + v;
        }
        red[k][threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < DZ_TB; ++w) s = MAXR ? fmax(s, red[k][w]) : s + red[k][w];
            out[k] = s;
        }
    }
}

// Trial design of the update: x(lam) on D, x elsewhere; top = the largest
// magnitudes of the two gradients on D (0: that direction is dropped).
__global__ __launch_bounds__(DZ_TB) void k_dz_trial(const unsigned char* __restrict__ mask,
                                                    const double* __restrict__ x, const double* __restrict__ gJ,
                                                    const double* __restrict__ gV, const double* __restrict__ top,
                                                    double move, double lam, int N, double* __restrict__ xn) {
    const int n = (int)(blockIdx.x * DZ_TB + threadIdx.x);
    if (n >= N) return;
    const double xv = x[n];
    if (!mask[n]) {
        xn[n] = xv;
        return;
    }
    const double sJ = top[0] > 0.0 ? gJ[n] / top[0] : 0.0;
    const double sV = top[1] > 0.0 ? gV[n] / top[1] : 0.0;
    const double lo = fmax(0.0, xv - move), hi = fmin(1.0, xv + move);
    xn[n] = fmin(fmax(xv - move * (sJ + lam * sV), lo), hi);
}

// Allocation-free map (lbm_design_map_noalloc): the filter with its
// normalisation in one stencil pass, no neighbour list. A workgroup stages
// m x and m over its tile and halo in LDS and walks the integer offsets of
// the ball |o| < r in the order the host list of a context uses (z, then y,
// then x), with weights r - |o|, so each sum takes the same terms in the
// same order as the context's two passes. Per-block partials of the volume
// sum and of the design-node count go to `partials`.
template <int D>
__global__ __launch_bounds__(DZ_TB) void k_dz_map_direct(DzGeo g, const unsigned char* __restrict__ mask,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ base, double radius,
                                                         double beta, double eta, double hn, double hd,
                                                         double* __restrict__ gamma, double* __restrict__ partials) {
    using TL = DzTile<D>;
    __shared__ double s0[dz_region_max<D>()];
    __shared__ double s1[dz_region_max<D>()];
    const int bidx = (int)blockIdx.x;
    const int btx = bidx % g.tiles_x, bty = (bidx / g.tiles_x) % g.tiles_y, btz = bidx / (g.tiles_x * g.tiles_y);
    const int x0 = btx * TL::X - g.H, y0 = bty * TL::Y - g.H, z0 = (D == 3 ? btz * TL::Z - g.H : 0);
    const int rcount = g.rx * g.ry * g.rz;
    for (int c = (int)threadIdx.x; c < rcount; c += DZ_TB) {
        const int lz = c / (g.rx * g.ry), r2 = c - lz * g.rx * g.ry;
        const int ly = r2 / g.rx, lx = r2 - ly * g.rx;
        const int xx = x0 + lx, yy = y0 + ly, zz = z0 + lz;
        double v0 = 0.0, v1 = 0.0;
        if (xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny && zz >= 0 && zz < g.nz) {
            const int n = (zz * g.ny + yy) * g.nx + xx;
            if (mask[n]) {
                v0 = x[n];
                v1 = 1.0;
            }
        }
        s0[c] = v0;
        s1[c] = v1;
    }
    __syncthreads();
    const int t = (int)threadIdx.x;
    const int ox = t % TL::X, oy = (t / TL::X) % TL::Y, oz = t / (TL::X * TL::Y);
    const int xx = btx * TL::X + ox, yy = bty * TL::Y + oy, zz = (D == 3 ? btz * TL::Z + oz : 0);
    double vol = 0.0, cnt = 0.0;
    if (xx < g.nx && yy < g.ny && zz < g.nz) {
        const int n = (zz * g.ny + yy) * g.nx + xx;
        const int cell = ((oz + (D == 3 ? g.H : 0)) * g.ry + (oy + g.H)) * g.rx + (ox + g.H);
        const bool m = mask[n] != 0;
        double gam = base[n];
        if (m) {
            double acc = 0.0, wsum = 0.0;
            const int hz = D == 3 ? g.H : 0;
            for (int dz = -hz; dz <= hz; ++dz)
                for (int dy = -g.H; dy <= g.H; ++dy)
                    for (int dx = -g.H; dx <= g.H; ++dx) {
                        const double dist = sqrt((double)(dx * dx + dy * dy + dz * dz));
                        if (dist < radius) {
                            const double w = radius - dist;
                            const int off = (dz * g.ry + dy) * g.rx + dx;
                            acc += w * s0[cell + off];
                            wsum += w * s1[cell + off];
                        }
                    }
            const double xt = acc / wsum;
            gam = (hn + tanh(beta * (xt - eta))) * hd;
            vol = gam;
            cnt = 1.0;
        }
        gamma[n] = gam;
    }
    double v[2] = {vol, cnt};
    dz_block_sum<2>(v, partials);
}

// volume = sums[0] / sums[1] (NaN for an empty design domain).
__global__ void k_dz_ratio(const double* __restrict__ sums, double* __restrict__ volume) {
    if (threadIdx.x == 0) volume[0] = sums[0] / sums[1];
}

size_t dz_align(size_t v) { return (v + 255) / 256 * 256; }

int dz_halo(double r) { return (int)std::ceil(r) - 1; }

struct DzLayout {
    size_t mask, base, W, xt, xtrial, gtrial, offs, partials, scal, total;
    int nb_tiles, nb_elems;
};

DzLayout dz_layout(int nx, int ny, int nz) {
    const size_t N = (size_t)nx * ny * nz;
    DzLayout L;
    const bool d3 = nz > 1;
    const int tx = d3 ? DzTile<3>::X : DzTile<2>::X, ty = d3 ? DzTile<3>::Y : DzTile<2>::Y;
    const int tz = d3 ? DzTile<3>::Z : 1;
    L.nb_tiles = ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty) * ((nz + tz - 1) / tz);
    L.nb_elems = (int)((N + DZ_TB - 1) / DZ_TB);
    const int nbp = L.nb_tiles > L.nb_elems ? L.nb_tiles : L.nb_elems;
    size_t o = 0;
    L.mask = o;     o += dz_align(N);
    L.base = o;     o += dz_align(N * 8);
    L.W = o;        o += dz_align(N * 8);
    L.xt = o;       o += dz_align(N * 8);
    L.xtrial = o;   o += dz_align(N * 8);
    L.gtrial = o;   o += dz_align(N * 8);
    L.offs = o;     o += dz_align(sizeof(DzOff) * 9 * 9 * 9);
    L.partials = o; o += dz_align((size_t)nbp * 2 * 8);
    L.scal = o;     o += dz_align(8 * 8);
    L.total = o;
    return L;
}

}  // namespace
}  // namespace lbm

using namespace lbm;

struct lbm_design {
    int nx, ny, nz, N, D;
    double radius;
    DzLayout L;
    char* ws;
    hipStream_t stream;
    DzGeo geo;
    double nd;   // design nodes
    unsigned char* mask() const { return (unsigned char*)(ws + L.mask); }
    double* fld(size_t off) const { return (double*)(ws + off); }
};

namespace {

#define DZCHK(expr)                                                                                       \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) return record_error(LBM_E_HIP, (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

lbm_status dz_bad(const char* msg) { return record_error(LBM_E_INVALID, msg); }

bool dz_valid_grid(int nx, int ny, int nz, double r) {
    return nx >= 1 && ny >= 1 && nz >= 1 && (long)nx * ny * nz < (1L << 30) && r >= 1.0 && r <= 5.0;
}

template <int MODE>
void dz_launch(const lbm_design* d, const double* a, const double* b, double beta, double eta, double* out0,
               double* out1, double* partials) {
    const double hn = std::tanh(beta * eta);
    const double hd = 1.0 / (hn + std::tanh(beta * (1.0 - eta)));
    const double inv_nd = d->nd > 0 ? 1.0 / d->nd : 0.0;
    const dim3 grid(d->L.nb_tiles), block(DZ_TB);
    if (d->D == 2)
        hipLaunchKernelGGL((k_dz_stencil<2, MODE>), grid, block, 0, d->stream, d->geo, d->mask(), a, b,
                           d->fld(d->L.W), d->fld(d->L.base), beta, eta, hn, hd, inv_nd, out0, out1, partials);
    else
        hipLaunchKernelGGL((k_dz_stencil<3, MODE>), grid, block, 0, d->stream, d->geo, d->mask(), a, b,
                           d->fld(d->L.W), d->fld(d->L.base), beta, eta, hn, hd, inv_nd, out0, out1, partials);
}

// gamma = map(x) into gout; the volume lands in scal[0] (device).
lbm_status dz_map(lbm_design* d, const double* x, double beta, double eta, double* gout) {
    double* part = d->fld(d->L.partials);
    dz_launch<DZ_FILTER>(d, x, nullptr, beta, eta, d->fld(d->L.xt), gout, part);
    DZCHK(hipGetLastError());
    hipLaunchKernelGGL((k_dz_final<1, 0>), dim3(1), dim3(DZ_TB), 0, d->stream, part, d->L.nb_tiles, d->fld(d->L.scal));
    DZCHK(hipGetLastError());
    return LBM_OK;
}

lbm_status dz_volume(lbm_design* d, double* v) {
    double s = 0.0;
    DZCHK(hipMemcpyAsync(&s, d->fld(d->L.scal), 8, hipMemcpyDeviceToHost, d->stream));
    DZCHK(hipStreamSynchronize(d->stream));
    *v = s / d->nd;
    return LBM_OK;
}

bool dz_params(double beta, double eta) { return std::isfinite(beta) && beta > 0.0 && eta > 0.0 && eta < 1.0; }

// Device address of `scratch` on each GPU, taken with that GPU current on
// the first allocation-free call there; never the array's host-side name.
constexpr int DZ_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[DZ_MAX_DEVICES] = {};

lbm_status noalloc_scratch(double** out) {
    int dev = -1;
    DZCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= DZ_MAX_DEVICES) return record_error(LBM_E_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        DZCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return record_error(LBM_E_HIP, "hipGetSymbolAddress returned a null address");
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_design_workspace_bytes(int nx, int ny, int nz, double radius, size_t* bytes) {
    if (!bytes) return dz_bad("bytes is NULL");
    if (!dz_valid_grid(nx, ny, nz, radius)) return dz_bad("grid sizes must be >= 1 and radius in [1, 5]");
    *bytes = dz_layout(nx, ny, nz).total;
    return LBM_OK;
}

lbm_status lbm_design_init(int nx, int ny, int nz, double radius, const unsigned char* mask_dev,
                           const double* base_dev, void* workspace_dev, size_t bytes, void* stream,
                           lbm_design** out) {
    if (!out || !mask_dev || !base_dev || !workspace_dev) return dz_bad("NULL argument");
    if (!dz_valid_grid(nx, ny, nz, radius)) return dz_bad("grid sizes must be >= 1 and radius in [1, 5]");
    if ((uintptr_t)workspace_dev % 256 != 0) return dz_bad("workspace must be 256-byte aligned");
    const DzLayout L = dz_layout(nx, ny, nz);
    if (bytes < L.total) return dz_bad("workspace too small");
    lbm_design* d = new lbm_design();
    d->nx = nx;
    d->ny = ny;
    d->nz = nz;
    d->N = nx * ny * nz;
    d->D = nz > 1 ? 3 : 2;
    d->radius = radius;
    d->L = L;
    d->ws = (char*)workspace_dev;
    d->stream = (hipStream_t)stream;
    // offsets of the ball |o| < r in the LDS region of a tile
    const int H = dz_halo(radius);
    DzGeo& g = d->geo;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.N = d->N;
    g.H = H;
    g.rx = (d->D == 3 ? DzTile<3>::X : DzTile<2>::X) + 2 * H;
    g.ry = (d->D == 3 ? DzTile<3>::Y : DzTile<2>::Y) + 2 * H;
    g.rz = d->D == 3 ? DzTile<3>::Z + 2 * H : 1;
    g.tiles_x = (nx + (d->D == 3 ? DzTile<3>::X : DzTile<2>::X) - 1) / (d->D == 3 ? DzTile<3>::X : DzTile<2>::X);
    g.tiles_y = (ny + (d->D == 3 ? DzTile<3>::Y : DzTile<2>::Y) - 1) / (d->D == 3 ? DzTile<3>::Y : DzTile<2>::Y);
    std::vector<DzOff> offs;
    const int hz = d->D == 3 ? H : 0;
    for (int oz = -hz; oz <= hz; ++oz)
        for (int oy = -H; oy <= H; ++oy)
            for (int ox = -H; ox <= H; ++ox) {
                const double dist = std::sqrt((double)(ox * ox + oy * oy + oz * oz));
                if (dist < radius) offs.push_back({(oz * g.ry + oy) * g.rx + ox, 0, radius - dist});
            }
    g.noff = (int)offs.size();
    g.offs = (const DzOff*)(d->ws + L.offs);
    auto bail = [&](lbm_status st) {
        delete d;
        return st;
    };
#define DZINIT(expr)                                                                                      \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess)                                                                             \
            return bail(record_error(LBM_E_HIP, (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str())); \
    } while (0)
    DZINIT(hipMemcpyAsync(d->ws + L.offs, offs.data(), offs.size() * sizeof(DzOff), hipMemcpyHostToDevice, d->stream));
    DZINIT(hipMemcpyAsync(d->mask(), mask_dev, (size_t)d->N, hipMemcpyDeviceToDevice, d->stream));
    DZINIT(hipMemcpyAsync(d->fld(L.base), base_dev, (size_t)d->N * 8, hipMemcpyDeviceToDevice, d->stream));
    dz_launch<DZ_WSUM>(d, nullptr, nullptr, 1.0, 0.5, d->fld(L.W), nullptr, nullptr);
    DZINIT(hipGetLastError());
    double* part = d->fld(L.partials);
    hipLaunchKernelGGL(k_dz_count, dim3(L.nb_elems), dim3(DZ_TB), 0, d->stream, d->mask(), d->N, part);
    hipLaunchKernelGGL((k_dz_final<1, 0>), dim3(1), dim3(DZ_TB), 0, d->stream, part, L.nb_elems, d->fld(L.scal));
    DZINIT(hipGetLastError());
    double nd = 0.0;
    DZINIT(hipMemcpyAsync(&nd, d->fld(L.scal), 8, hipMemcpyDeviceToHost, d->stream));
    DZINIT(hipStreamSynchronize(d->stream));
#undef DZINIT
    if (nd < 1.0) return bail(dz_bad("the design domain is empty"));
    d->nd = nd;
    *out = d;
    return LBM_OK;
}

lbm_status lbm_design_map(lbm_design* d, const double* x_dev, double beta, double eta, double* gamma_dev,
                          double* volume) {
    if (!d || !x_dev || !gamma_dev) return dz_bad("NULL argument");
    if (!dz_params(beta, eta)) return dz_bad("need beta > 0 and 0 < eta < 1");
    lbm_status st = dz_map(d, x_dev, beta, eta, gamma_dev);
    if (st != LBM_OK) return st;
    if (volume) return dz_volume(d, volume);
    return LBM_OK;
}

lbm_status lbm_design_chain(lbm_design* d, const double* x_dev, double beta, double eta,
                            const double* dJdgamma_dev, double* dJdx_dev, double* dVdx_dev) {
    if (!d || !x_dev || !dJdgamma_dev || !dJdx_dev) return dz_bad("NULL argument");
    if (!dz_params(beta, eta)) return dz_bad("need beta > 0 and 0 < eta < 1");
    // x~ of this design (the projected field goes to scratch)
    lbm_status st = dz_map(d, x_dev, beta, eta, d->fld(d->L.gtrial));
    if (st != LBM_OK) return st;
    dz_launch<DZ_CHAIN>(d, d->fld(d->L.xt), dJdgamma_dev, beta, eta, dJdx_dev, dVdx_dev, nullptr);
    DZCHK(hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_design_update(lbm_design* d, const double* x_dev, const double* dJdx_dev,
                             const double* dVdx_dev, double beta, double eta, double move, double vmin,
                             double vmax, double* x_new_dev, double* volume, double* lambda) {
    if (!d || !x_dev || !dJdx_dev || !dVdx_dev || !x_new_dev) return dz_bad("NULL argument");
    if (x_new_dev == x_dev) return dz_bad("x_new_dev must not alias x_dev");
    if (!dz_params(beta, eta)) return dz_bad("need beta > 0 and 0 < eta < 1");
    if (!(move > 0.0 && move <= 1.0) || !(vmin >= 0.0 && vmin <= vmax && vmax <= 1.0))
        return dz_bad("need 0 < move <= 1 and 0 <= vmin <= vmax <= 1");
    const DzLayout& L = d->L;
    double* part = d->fld(L.partials);
    double* top = d->fld(L.scal) + 2;
    hipLaunchKernelGGL(k_dz_absmax, dim3(L.nb_elems), dim3(DZ_TB), 0, d->stream, d->mask(), dJdx_dev, dVdx_dev,
                       d->N, part);
    hipLaunchKernelGGL((k_dz_final<2, 1>), dim3(1), dim3(DZ_TB), 0, d->stream, part, L.nb_elems, top);
    DZCHK(hipGetLastError());
    auto vol_at = [&](double lam, double* xn, double* v) -> lbm_status {
        hipLaunchKernelGGL(k_dz_trial, dim3(L.nb_elems), dim3(DZ_TB), 0, d->stream, d->mask(), x_dev, dJdx_dev,
                           dVdx_dev, top, move, lam, d->N, xn);
        DZCHK(hipGetLastError());
        lbm_status st = dz_map(d, xn, beta, eta, d->fld(L.gtrial));
        if (st != LBM_OK) return st;
        return dz_volume(d, v);
    };
    double v = 0.0, lam = 0.0;
    double* xt = d->fld(L.xtrial);
    lbm_status st = vol_at(0.0, xt, &v);
    if (st != LBM_OK) return st;
    if (v > vmax || v < vmin) {
        // V(x(lam)) does not increase with lam: lam > 0 above vmax, < 0 below vmin
        const bool above = v > vmax;
        auto feasible = [&](double vv) { return above ? vv <= vmax : vv >= vmin; };
        double a = 0.0, b = above ? 1.0 : -1.0, vb = 0.0;
        for (int k = 0; k < 60; ++k) {
            if ((st = vol_at(b, xt, &vb)) != LBM_OK) return st;
            if (feasible(vb)) break;
            a = b;
            b = 2.0 * b;
        }
        for (int k = 0; k < 60; ++k) {
            const double c = 0.5 * (a + b);
            double vc = 0.0;
            if ((st = vol_at(c, xt, &vc)) != LBM_OK) return st;
            if (feasible(vc)) b = c;
            else a = c;
        }
        lam = b;
    }
    if ((st = vol_at(lam, x_new_dev, &v)) != LBM_OK) return st;
    if (volume) *volume = v;
    if (lambda) *lambda = lam;
    return LBM_OK;
}

void lbm_design_destroy(lbm_design* d) { delete d; }

lbm_status lbm_design_map_noalloc(int nx, int ny, int nz, double radius, const unsigned char* mask_dev,
                                  const double* base_dev, const double* x_dev, double beta, double eta,
                                  double* gamma_dev, double* volume_dev, void* stream) {
    if (!mask_dev || !base_dev || !x_dev || !gamma_dev) return dz_bad("NULL argument");
    if (!dz_valid_grid(nx, ny, nz, radius)) return dz_bad("grid sizes must be >= 1 and radius in [1, 5]");
    if (!dz_params(beta, eta)) return dz_bad("need beta > 0 and 0 < eta < 1");
    const DzLayout L = dz_layout(nx, ny, nz);
    if (L.nb_tiles > DZ_NOALLOC_BLOCKS)
        return dz_bad("grid too large for lbm_design_map_noalloc (at most 65536 tiles of 256 nodes)");
    double* scr = nullptr;
    lbm_status st = noalloc_scratch(&scr);
    if (st != LBM_OK) return st;
    const int D = nz > 1 ? 3 : 2;
    const int H = dz_halo(radius);
    DzGeo g{};
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.N = nx * ny * nz;
    g.H = H;
    g.rx = (D == 3 ? DzTile<3>::X : DzTile<2>::X) + 2 * H;
    g.ry = (D == 3 ? DzTile<3>::Y : DzTile<2>::Y) + 2 * H;
    g.rz = D == 3 ? DzTile<3>::Z + 2 * H : 1;
    g.tiles_x = (nx + (D == 3 ? DzTile<3>::X : DzTile<2>::X) - 1) / (D == 3 ? DzTile<3>::X : DzTile<2>::X);
    g.tiles_y = (ny + (D == 3 ? DzTile<3>::Y : DzTile<2>::Y) - 1) / (D == 3 ? DzTile<3>::Y : DzTile<2>::Y);
    g.noff = 0;
    g.offs = nullptr;
    const double hn = std::tanh(beta * eta);
    const double hd = 1.0 / (hn + std::tanh(beta * (1.0 - eta)));
    hipStream_t sm = (hipStream_t)stream;
    double* sums = scr + 2 * DZ_NOALLOC_BLOCKS;
    if (D == 2)
        hipLaunchKernelGGL(k_dz_map_direct<2>, dim3(L.nb_tiles), dim3(DZ_TB), 0, sm, g, mask_dev, x_dev, base_dev,
                           radius, beta, eta, hn, hd, gamma_dev, scr);
    else
        hipLaunchKernelGGL(k_dz_map_direct<3>, dim3(L.nb_tiles), dim3(DZ_TB), 0, sm, g, mask_dev, x_dev, base_dev,
                           radius, beta, eta, hn, hd, gamma_dev, scr);
    DZCHK(hipGetLastError());
    if (volume_dev) {
        hipLaunchKernelGGL((k_dz_final<2, 0>), dim3(1), dim3(DZ_TB), 0, sm, scr, L.nb_tiles, sums);
        hipLaunchKernelGGL(k_dz_ratio, dim3(1), dim3(64), 0, sm, sums, volume_dev);
        DZCHK(hipGetLastError());
    }
    return LBM_OK;
}

}  // extern "C"
