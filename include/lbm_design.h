/*
 * lbm_design.h - C ABI of the design update of the optimisation loop
 * (Sec. "Topology optimization procedure" and Algorithm "Optimization
 * iteration"): density filter of radius r, Heaviside projection, volume
 * fraction, the chain-rule transposes that carry dJ/dgamma back to the
 * design variables, and a projected-gradient update under the volume
 * constraint, which stands in for MMA (MMA itself is not provided).
 *
 * Conventions (as lbm.h): node = (z * ny + y) * nx + x; gamma = 1 solid.
 *   - The design variables x (FP64, one per node) act on the design domain
 *     D, a byte mask (nonzero = design node). Every other node keeps the
 *     fixed value base[node] in the physical field.
 *   - Filter: for i in D, x~_i = sum_{j in D} w_ij x_j / sum_{j in D} w_ij,
 *     w_ij = r - |x_i - x_j| where |x_i - x_j| < r, else 0 (no periodic
 *     wrap). Projection: gamma_i = H(x~_i) = [tanh(beta eta) +
 *     tanh(beta (x~_i - eta))] / [tanh(beta eta) + tanh(beta (1 - eta))].
 *   - Volume fraction: V = (1 / n_D) sum_{i in D} gamma_i (the paper's mean
 *     of 1 - phi over the design domain).
 *   - Update: with g_J = dJ/dx and g_V = dV/dx each divided by its largest
 *     magnitude on D, x(lam) = clip(x - move (g_J + lam g_V),
 *     max(0, x - move), min(1, x + move)) on D (x elsewhere); V(x(lam))
 *     does not increase with lam. lam = 0 when vmin <= V(x(0)) <= vmax;
 *     above vmax the smallest lam > 0 with V(x(lam)) <= vmax, below vmin the
 *     lam < 0 of smallest magnitude with V(x(lam)) >= vmin, each found by
 *     doubling |lam| from 1 and 60 bisection halvings (the feasible end).
 *     If the move limit keeps V out of the bounds, the most feasible step
 *     after 60 doublings is returned.
 *
 * Memory and streams: the caller owns all device memory (the workspace
 * sized by lbm_design_workspace_bytes and every field). All work goes to
 * the caller's stream; lbm_design_init, and the calls that return a volume
 * or a multiplier, synchronise it. A context is not thread-safe.
 * Errors: LBM_E_INVALID for bad arguments (checked before any HIP call),
 * LBM_E_HIP for HIP failures; lbm_last_error() has the message.
 */
#ifndef LBM_DESIGN_H
#define LBM_DESIGN_H

#include <stddef.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_design lbm_design;

/* Device workspace bytes for a design context on an nx x ny x nz grid
 * (nz = 1 in 2D) with filter radius 1 <= radius <= 5. */
lbm_status lbm_design_workspace_bytes(int nx, int ny, int nz, double radius, size_t* bytes);

/* Creates a context: copies the mask (device bytes, N) and base (device
 * FP64, N) into the workspace (device, 256-byte aligned, at least
 * lbm_design_workspace_bytes), computes the filter normalisation and counts
 * the design nodes. Errors: LBM_E_INVALID for bad sizes, a radius outside
 * [1, 5], a small workspace or an empty design domain. */
lbm_status lbm_design_init(int nx, int ny, int nz, double radius, const unsigned char* mask_dev,
                           const double* base_dev, void* workspace_dev, size_t bytes, void* stream,
                           lbm_design** out);

/* Physical field: gamma_dev (device FP64, N) = H(F x) on D, base elsewhere;
 * volume (host, may be NULL) = V(gamma). Requires beta > 0, 0 < eta < 1. */
lbm_status lbm_design_map(lbm_design* d, const double* x_dev, double beta, double eta, double* gamma_dev,
                          double* volume);

/* Chain rule (Sec. "Topology optimization procedure", standard filter and
 * projection transposes): dJdx_dev = dJ/dx and dVdx_dev = dV/dx (device
 * FP64, N; 0 off D) for the sensitivity dJdgamma_dev (device FP64, N, e.g.
 * from lbm_adjoint) at the design x_dev. dVdx_dev may be NULL. */
lbm_status lbm_design_chain(lbm_design* d, const double* x_dev, double beta, double eta,
                            const double* dJdgamma_dev, double* dJdx_dev, double* dVdx_dev);

/* Projected-gradient step under vmin <= V <= vmax (see the conventions
 * above): x_new_dev (device FP64, N; may not alias x_dev) receives x(lam);
 * volume and lambda (host, may be NULL) receive V(x(lam)) and lam. Requires
 * 0 < move <= 1 and 0 <= vmin <= vmax <= 1. */
lbm_status lbm_design_update(lbm_design* d, const double* x_dev, const double* dJdx_dev,
                             const double* dVdx_dev, double beta, double eta, double move, double vmin,
                             double vmax, double* x_new_dev, double* volume, double* lambda);

/* Frees the host-side context. */
void lbm_design_destroy(lbm_design* d);

/* Allocation-free form of lbm_design_map, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. It needs no context and no workspace and
 * calls no allocating routine. Same result as lbm_design_init on (nx, ny,
 * nz, radius, mask_dev, base_dev) followed by lbm_design_map(x_dev, beta,
 * eta): gamma_dev (device FP64, N, caller-owned) = H(F x) on the design
 * domain, base elsewhere; if volume_dev (device FP64, one value, may be
 * NULL) is given it receives V(gamma) (NaN for an empty design domain).
 * Inputs mask_dev (device bytes, N), base_dev and x_dev (device FP64, N)
 * are read only. Everything is enqueued on `stream`; nothing is
 * synchronised.
 * Limits: at most 65536 tiles of 256 nodes (32 x 8 in 2D, 8 x 8 x 4 in 3D;
 * 16 777 216 nodes when the grid is a multiple of the tile), else
 * LBM_E_INVALID. Scratch: a fixed 1 MB device array of the library, one per
 * GPU, held until the process ends; every call on a GPU uses that GPU's
 * array (it rewrites all it reads, nothing needs clearing), so calls that
 * overlap on one GPU (other streams or threads) race. The first call on
 * each GPU looks up the array's device address (hipGetSymbolAddress, not a
 * stream operation); make that first call before any graph capture.
 * Errors: LBM_E_INVALID for NULL inputs, bad sizes, radius outside [1, 5],
 * beta <= 0 or eta outside (0, 1), all before any HIP call; LBM_E_HIP for
 * HIP failures. */
lbm_status lbm_design_map_noalloc(int nx, int ny, int nz, double radius, const unsigned char* mask_dev,
                                  const double* base_dev, const double* x_dev, double beta, double eta,
                                  double* gamma_dev, double* volume_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif
