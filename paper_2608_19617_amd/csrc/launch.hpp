// Launch descriptors between the host driver and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"
#include "lbm.h"

namespace lbm {

struct StepLaunch {
    int lattice, prec;
    const void* gin;       // post-collision state G^{k-1}
    void* gout;            // post-collision state G^k
    void* pre;             // if not null: also store f^k here (checkpoint)
    const void* s;         // bounce-back fraction plane
    int sample;            // write block partials of the samples of f^k (last step)
    double* partials;      // [part_stride][3]
    int part_stride;       // partial slots per sample (unused slots are zeroed)
    int nsteps;            // 1: single step; > 1: temporally blocked launch (D2Q9; 2 for D3Q19)
    int tile_x, tile_y;    // output tile of a blocked launch
    int tile_z;            // D3Q19: two steps on tile_x x tile_y tiles, tile_z planes per workgroup
    void* rec;             // recompute: the moment record of step t's pre-collision state goes
    size_t rec_slot;       // to rec + (t-1) * rec_slot bytes (compute type, record_size planes of N)
    Geo geo;
    Phys ph;
    Obj ob;
    hipStream_t stream;
};

struct AdjLaunch {
    int lattice, prec;
    const void* nu_in;     // nu_hat^k
    void* nu_out;          // nu_hat^{k-1}
    const void* state;     // f^{k-1} (direct), its moment record (rec) or the G it is pulled from (seed)
    const void* s;
    double* sens;
    int direct, seed;
    int rec;               // state / gseg hold moment records, slot bytes apart
    double src_w;          // weight of the objective source on f^{k-1} (0: none)
    // blocked launch (nsteps > 1; D3Q19: 2): steps k_hi .. k_hi - nsteps + 1, each
    // reading the moment record of its pre-state f^{k-1} at gseg + (k - 2 - kseg) * slot
    // bytes
    int nsteps, tile_x, tile_y;
    int tile_z;            // D3Q19 (nsteps = 2): z planes per workgroup
    const void* gseg;
    size_t slot;
    long kseg, k_hi, ns, dW;
    double wgt;
    Geo geo;
    Phys ph;
    Obj ob;
    hipStream_t stream;
};

enum AuxOp {
    AUX_COLLIDE = 0,       // dst = C(src) with s
    AUX_INIT_EQ,           // dst = f^eq(rho0, u_init) - w
    AUX_EXPORT_DIRECT,     // dst (FP64) = src + w
    AUX_EXPORT_PULL,       // dst (FP64) = BC(S(src)) + w
    AUX_FIELDS_DIRECT,     // dst (FP64) = rho, u of src + w
    AUX_FIELDS_PULL,       // dst (FP64) = rho, u of BC(S(src)) + w
    AUX_IMPORT,            // dst = src (FP64) - w
    AUX_DESIGN             // dst = s(src = gamma)
};

struct AuxLaunch {
    int lattice, prec;
    int op;
    const void* src;
    void* dst;
    const void* s;
    double rho0;
    int umode;
    int map;
    double q;
    Geo geo;
    Phys ph;
    hipStream_t stream;
};

// LDS a blocked launch may use (of the 160 KB of a compute unit)
constexpr size_t TB_LDS_MAX = 159 * 1024;
// Largest state (bytes) of a blocked D3Q19 launch, which addresses it with
// 32-bit byte offsets and keeps the offsets above this for no-op accesses.
constexpr size_t TBZ_STATE_MAX = 0xFFFFFF00u;

// Sets the thread-local message that lbm_last_error returns; returns st.
lbm_status record_error(lbm_status st, const char* msg);

hipError_t launch_step(const StepLaunch& a);
hipError_t launch_adjoint(const AdjLaunch& a);
hipError_t launch_aux(const AuxLaunch& a);
hipError_t launch_reduce(const double* partials, long nblocks, int nsamples, double* samples, double weight,
                         double* acc, hipStream_t stream);
hipError_t launch_finalize(const double* gamma, const double* sens, double* out, long N, int map, double q,
                           hipStream_t stream);
hipError_t launch_fill(double* p, long n, double v, hipStream_t stream);
// out[0] = sum_i (a_i - b_i)^2 over n values: nparts block partials into
// parts (nparts doubles), then one block sums them in a fixed order.
hipError_t launch_sq_diff_sum(const double* a, const double* b, long n, double* parts, int nparts, double* out,
                              hipStream_t stream);
// sens[node] += field[i] over the nodes of the objective's accumulator box.
hipError_t launch_box_add(double* sens, const double* field, const Geo& g, const Obj& ob, hipStream_t stream);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t stream);
long blocks_for(long n);
int tb_plane(int nsteps, int tile_x, int tile_y, size_t lsize, size_t vsize, size_t extra);
size_t tb_lds_bytes(int nsteps, int tile_x, int tile_y, size_t lsize, size_t vsize);
size_t tb_lds_bytes_prec(int nsteps, int tile_x, int tile_y, int prec);   // forward kernel of a precision
size_t adj_tb_lds_bytes(int nsteps, int tile_x, int tile_y, size_t vsize);
long tb_blocks(int nx, int ny, int tile_x, int tile_y);
size_t tbz_lds_bytes(int tile_x, int tile_y, size_t lsize, size_t vsize);
size_t tbz_lds_bytes_prec(int tile_x, int tile_y, int prec);
int tbz_threads(int tile_x, int tile_y);
size_t adj_tbz_lds_bytes(int tile_x, int tile_y, size_t asize, size_t tsize);
hipError_t tb_prepare(int prec);
int tb_threads(int nsteps, int tile_x, int tile_y);

}  // namespace lbm
