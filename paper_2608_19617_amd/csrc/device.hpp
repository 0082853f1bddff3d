// Device-side building blocks of the lattice kernels: node geometry, the
// pull with halfway bounce-back, the Zou-He rules and their transposes, the
// regularized Smagorinsky collision with partial bounce-back, and its
// reverse-mode derivative in moment space.
//
// Populations are held shifted, h_a = f_a - w_a, so that the small
// deviations from rest keep their precision in FP32 / FP16 storage; every
// formula below is the paper's, rewritten in h (the shift cancels exactly in
// the moments because sum w = 1, sum w c = 0, sum w c c = c_s^2 I).
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace lbm {

enum RowKind : int { ROW_WALL = 0, ROW_VELOCITY = 1, ROW_PRESSURE = 2 };

// Geometry and boundary description shared by every kernel.
struct Geo {
    int nx, ny, nz;
    int N;                     // nodes (the host keeps Q * N below 2^31)
    double inv_nx, inv_ny;     // 1/nx, 1/ny for the node-index split
    int per_x, per_y, per_z;   // periodic axes
    const signed char* west;   // per row kind of the x = 0 face
    const signed char* east;   // per row kind of the x = nx-1 face
    const double* u_in;        // per row inlet velocity
    double drho_out;           // rho_0 - 1 of pressure rows
};

// Collision constants.
struct Phys {
    double tau;
    double c2;                 // C_s^2 (filter width 1)
};

// Objective / monitor description (per-node contributions). Kinds: 0
// pressure drop, 1 dissipation + pressure drop, 2 drag (objective: the drag
// force over the force box; monitor: C_d = drag * inv_dref), 3 wake
// recovery (objective only).
struct Obj {
    int obj, mon;
    int in_x, in_lo, in_hi;
    int out_x, out_lo, out_hi;
    double inv_nin, inv_nout;  // 1 / section node counts
    int fx0, fx1, fy0, fy1, fz0, fz1;   // force box, half-open
    double inv_dref;           // 1 / (rho_0 u_0^2 L_ref / 2)
    // window field accumulator: 2 dD/ds per force-box node (drag) or the
    // velocity components per measurement-box node (wake), FP64, component
    // planes of nb values over the box [ax0, ax0 + anx) x [ay0, ay0 + any)
    // x [az0, az0 + nb / (anx * any)), x fastest
    int ax0, ay0, az0, anx, any, anz, nb;
    double wgt;                // dW / |W|
    double* facc;              // forward / replay accumulation (null: none)
    const double* fwin;        // the objective window's accumulation (adjoint)
    const double* uref;        // wake reference mean velocity on the box
};

__device__ __forceinline__ bool in_force_box(const Obj& ob, int x, int y, int z) {
    return x >= ob.fx0 && x < ob.fx1 && y >= ob.fy0 && y < ob.fy1 && z >= ob.fz0 && z < ob.fz1;
}

// Index of node (x, y, z) in the accumulator box, or -1 outside it.
__device__ __forceinline__ int acc_index(const Obj& ob, int x, int y, int z) {
    const int i = x - ob.ax0, j = y - ob.ay0, k = z - ob.az0;
    if ((unsigned)i >= (unsigned)ob.anx || (unsigned)j >= (unsigned)ob.any || (unsigned)k >= (unsigned)ob.anz)
        return -1;
    return (k * ob.any + j) * ob.anx + i;
}

// q = floor(n / d) through an FP64 product (exact to within one for
// n < 2^31), corrected once.
__device__ __forceinline__ void divmod(int n, int d, double inv_d, int& q, int& r) {
    q = (int)((double)n * inv_d);
    r = n - q * d;
    if (r < 0) {
        q -= 1;
        r += d;
    } else if (r >= d) {
        q += 1;
        r -= d;
    }
}

__device__ __forceinline__ void node_coords(const Geo& g, int n, int& x, int& y, int& z) {
    int r;
    divmod(n, g.nx, g.inv_nx, r, x);
    if (g.nz == 1) {
        y = r;
        z = 0;
    } else {
        divmod(r, g.ny, g.inv_ny, z, y);
    }
}

// Reciprocal and square root: hardware 1-ulp instructions in FP32, IEEE in FP64.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }

// Base pointer of population plane a (uniform across the wave).
template <class P>
__device__ __forceinline__ P* plane(P* base, int a, int N) { return base + (size_t)a * (size_t)N; }

// Open-face code of a node: 0 = not open; 1 + face * 3 + kind otherwise
// (face 0 = west, 1 = east). Rows touching a non-periodic y (or z) wall
// are wall nodes, which the host validation guarantees for the row tables.
template <class L>
__device__ __forceinline__ int open_code(const Geo& g, int x, int y, int z) {
    if (g.per_x) return 0;
    if (L::D == 3 && !g.per_z && (z == 0 || z == g.nz - 1)) return 0;
    if (x == 0) {
        int k = g.west[y];
        return k ? 1 + k : 0;
    }
    if (x == g.nx - 1) {
        int k = g.east[y];
        return k ? 4 + k : 0;
    }
    return 0;
}

template <class S>
__device__ __forceinline__ float to_f(S v) { return (float)v; }

// Pull of the post-collision populations into node (x, y, z) (Eq.
// streaming_step): h_a(x) = G_a(x - c_a). A source outside a non-periodic
// axis is the halfway bounce-back of Eq. wall, h_a(x) = G_opp(a)(x). On an
// open node those directions are exactly the unknowns that the Zou-He rule
// overwrites afterwards (rows touching a wall face are wall rows), so the
// same rule serves every node and the load never depends on the row kind.
template <class L, class S, class T>
__device__ __forceinline__ void pull(const S* __restrict__ G, const Geo& g, int n, int x, int y,
                                     int z, T h[L::Q]) {
    const int N = g.N;
    const bool interior = x > 0 && x < g.nx - 1 && y > 0 && y < g.ny - 1 &&
                          (L::D == 2 || (z > 0 && z < g.nz - 1));
    if (interior) {
#pragma unroll
        for (int a = 0; a < L::Q; ++a) {
            const int off = L::cx[a] + L::cy[a] * g.nx + L::cz[a] * g.nx * g.ny;
            h[a] = (T)plane(G, a, N)[(unsigned)(n - off)];
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < L::Q; ++a) {
        int xs = x - L::cx[a], ys = y - L::cy[a], zs = z - L::cz[a];
        bool out = false;
        if (xs < 0 || xs >= g.nx) {
            if (g.per_x) xs = xs < 0 ? xs + g.nx : xs - g.nx;
            else out = true;
        }
        if (ys < 0 || ys >= g.ny) {
            if (g.per_y) ys = ys < 0 ? ys + g.ny : ys - g.ny;
            else out = true;
        }
        if (L::D == 3 && (zs < 0 || zs >= g.nz)) {
            if (g.per_z) zs = zs < 0 ? zs + g.nz : zs - g.nz;
            else out = true;
        }
        // the plane is chosen by value (pointer arithmetic), so h keeps
        // compile-time indices
        const unsigned src = out ? (unsigned)n : (unsigned)((zs * g.ny + ys) * g.nx + xs);
        const int pa = out ? L::opp[a] : a;
        h[a] = (T)plane(G, pa, N)[src];
    }
}

// Source of every population of the pull into node (x, y, z), as element
// indices into the state that include the plane (a * N + node); the same
// sources as pull. The branch between interior and boundary nodes only
// computes indices, so the loads that follow are one straight run with no
// join between them (no wait on loads already in flight at a join).
template <class L>
__device__ __forceinline__ void pull_index(const Geo& g, int n, int x, int y, int z, unsigned e[L::Q]) {
    const int N = g.N;
    const bool interior = x > 0 && x < g.nx - 1 && y > 0 && y < g.ny - 1 &&
                          (L::D == 2 || (z > 0 && z < g.nz - 1));
    if (interior) {
#pragma unroll
        for (int a = 0; a < L::Q; ++a) {
            const int off = L::cx[a] + L::cy[a] * g.nx + L::cz[a] * g.nx * g.ny;
            e[a] = (unsigned)(a * N - off) + (unsigned)n;
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < L::Q; ++a) {
        int xs = x - L::cx[a], ys = y - L::cy[a], zs = z - L::cz[a];
        bool out = false;
        if (xs < 0 || xs >= g.nx) {
            if (g.per_x) xs = xs < 0 ? xs + g.nx : xs - g.nx;
            else out = true;
        }
        if (ys < 0 || ys >= g.ny) {
            if (g.per_y) ys = ys < 0 ? ys + g.ny : ys - g.ny;
            else out = true;
        }
        if (L::D == 3 && (zs < 0 || zs >= g.nz)) {
            if (g.per_z) zs = zs < 0 ? zs + g.nz : zs - g.nz;
            else out = true;
        }
        e[a] = out ? (unsigned)(L::opp[a] * N + n) : (unsigned)(a * N + (zs * g.ny + ys) * g.nx + xs);
    }
}

// Zou-He rule on an open x-face node (Eqs. inlet, outlet; the west
// pressure outlet is their x-mirror; in 3D the same rule with the
// tangential momentum correction of every transverse axis). In shifted
// form: with b = sum_{c_x=0} h + 2 sum_{leaving} h, the mass balance gives
// rho = (1 + b)/(1 - u0) on a velocity row and rho u_x = rho_0 - (1 + b)
// (west) or (1 + b) - rho_0 (east) on a pressure row; each entering
// population is h_a = h_opp(a) + 6 w_a c_ax rho u_x - 1/2 sum_p c_ap N_p with
// N_p = sum_{c_x=0} c_p h.
template <class L, class T, int SGN>
__device__ __forceinline__ void zou_he_face(int kind, T u0, T d0, T h[L::Q]) {
    T b = 0, Ny = 0, Nz = 0;
#pragma unroll
    for (int a = 0; a < L::Q; ++a) {
        if (L::cx[a] == 0) {
            b += h[a];
            Ny += (T)L::cy[a] * h[a];
            if (L::D == 3) Nz += (T)L::cz[a] * h[a];
        } else if (L::cx[a] == -SGN) {
            b += (T)2 * h[a];
        }
    }
    T rux;
    if (kind == ROW_VELOCITY) {
        rux = ((T)1 + b) * u0 / ((T)1 - u0);
    } else {
        rux = SGN == 1 ? d0 - b : b - d0;
    }
#pragma unroll
    for (int a = 0; a < L::Q; ++a) {
        if (L::cx[a] == SGN) {
            T v = h[L::opp[a]] + (T)(6.0 * L::w[a] * L::cx[a]) * rux;
            if (L::cy[a] != 0) v -= (T)(0.5 * L::cy[a]) * Ny;
            if (L::D == 3 && L::cz[a] != 0) v -= (T)(0.5 * L::cz[a]) * Nz;
            h[a] = v;
        }
    }
}

// Both faces are evaluated and the result selected element by element, so
// that every array index stays a compile-time constant (a branch per face
// lets the compiler merge the two faces' stores into one with a selected
// address, which moves the array to scratch memory). u0 is the row's inlet
// speed, d0 = rho_0 - 1 of the pressure rows.
template <class L, class T>
__device__ __forceinline__ void zou_he_rows(int oc, T u0, T d0, T h[L::Q]) {
    const int kind = (oc - 1) % 3;
    const bool west = oc <= 3;
    T hw[L::Q], he[L::Q];
#pragma unroll
    for (int a = 0; a < L::Q; ++a) hw[a] = he[a] = h[a];
    zou_he_face<L, T, 1>(kind, u0, d0, hw);
    zou_he_face<L, T, -1>(kind, u0, d0, he);
#pragma unroll
    for (int a = 0; a < L::Q; ++a) h[a] = west ? hw[a] : he[a];
}

template <class L, class T>
__device__ __forceinline__ void zou_he(const Geo& g, int oc, int y, T h[L::Q]) {
    zou_he_rows<L, T>(oc, (T)g.u_in[y], (T)g.drho_out, h);
}

// Transpose of zou_he on the adjoint populations mu of the post-boundary
// state: entering directions get 0, the others collect their Jacobian
// column. With chi = u0/(1 - u0) (velocity), -1 (west pressure) or +1 (east
// pressure): mu_b += A m_b (m = 1 tangential, 2 leaving), mu_opp(a) += mu_a,
// and tangential directions lose sum_p c_bp B_p, where
// A = 6 chi sum_{entering} w_a c_ax mu_a and B_p = 1/2 sum_{entering} c_ap mu_a.
// For D2Q9 this is Eqs. adjoint_inlet_bc and adjoint_outlet_bc.
template <class L, class T, int SGN>
__device__ __forceinline__ void zou_he_adjoint_face(int kind, T u0, T mu[L::Q]) {
    T chi;
    if (kind == ROW_VELOCITY) {
        chi = u0 / ((T)1 - u0);
    } else {
        chi = SGN == 1 ? (T)-1 : (T)1;
    }
    T A = 0, By = 0, Bz = 0;
#pragma unroll
    for (int a = 0; a < L::Q; ++a) {
        if (L::cx[a] == SGN) {
            A += (T)(6.0 * L::w[a] * L::cx[a]) * mu[a];
            By += (T)(0.5 * L::cy[a]) * mu[a];
            if (L::D == 3) Bz += (T)(0.5 * L::cz[a]) * mu[a];
        }
    }
    A *= chi;
    T out[L::Q];
#pragma unroll
    for (int a = 0; a < L::Q; ++a) {
        if (L::cx[a] == SGN) {
            out[a] = 0;
        } else if (L::cx[a] == 0) {
            T v = mu[a] + A;
            if (L::cy[a] != 0) v -= (T)L::cy[a] * By;
            if (L::D == 3 && L::cz[a] != 0) v -= (T)L::cz[a] * Bz;
            out[a] = v;
        } else {
            out[a] = mu[a] + (T)2 * A + mu[L::opp[a]];
        }
    }
#pragma unroll
    for (int a = 0; a < L::Q; ++a) mu[a] = out[a];
}

// u0 is the row's inlet speed; both faces are evaluated and selected by
// value (see zou_he_rows).
template <class L, class T>
__device__ __forceinline__ void zou_he_adjoint_rows(int oc, T u0, T mu[L::Q]) {
    const int kind = (oc - 1) % 3;
    const bool west = oc <= 3;
    T mw[L::Q], me[L::Q];
#pragma unroll
    for (int a = 0; a < L::Q; ++a) mw[a] = me[a] = mu[a];
    zou_he_adjoint_face<L, T, 1>(kind, u0, mw);
    zou_he_adjoint_face<L, T, -1>(kind, u0, me);
#pragma unroll
    for (int a = 0; a < L::Q; ++a) mu[a] = west ? mw[a] : me[a];
}

template <class L, class T>
__device__ __forceinline__ void zou_he_adjoint(const Geo& g, int oc, int y, T mu[L::Q]) {
    zou_he_adjoint_rows<L, T>(oc, (T)g.u_in[y], mu);
}

// Symmetric-tensor helpers over D x D, stored as the upper triangle in the
// order xx, xy, (xz,) yy, (yz,) zz.
template <int D>
struct Sym;
template <>
struct Sym<2> {
    static constexpr int K = 3;
    static constexpr int idx[2][2] = {{0, 1}, {1, 2}};
};
template <>
struct Sym<3> {
    static constexpr int K = 6;
    static constexpr int idx[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
};

// Moments of a shifted node state: drho = sum h, j = sum c h, and the
// non-equilibrium second moment Pi = sum (c c - c_s^2 I) h - j j / rho
// (Eq. Pi, with sum c c f^eq = rho c_s^2 I + rho u u).
template <class L, class T>
struct Moments {
    T drho, rho, irho;
    T j[L::D];
    T Pi[Sym<L::D>::K];
    T PP;       // Pi : Pi (full contraction)
    T norm;     // ||Pi|| = sqrt(2 Pi:Pi)
    T R;        // sqrt(tau^2 + 2 C^2 ||Pi|| / (rho c_s^4))
    T te, ite;  // tau_eff (Eq. tau_eff) and its reciprocal
};

// Completes the moments from rho, 1/rho and Pi: Pi:Pi, ||Pi||, and the
// effective relaxation time of Eq. tau_eff with its reciprocal.
template <class L, class T>
__device__ __forceinline__ void moments_finish(const Phys& ph, Moments<L, T>& m) {
    constexpr int D = L::D;
    using SY = Sym<D>;
    T PP = 0;
#pragma unroll
    for (int p = 0; p < D; ++p) {
#pragma unroll
        for (int q = p; q < D; ++q) {
            const T v = m.Pi[SY::idx[p][q]];
            PP += (p == q ? (T)1 : (T)2) * v * v;
        }
    }
    m.PP = PP;
    m.norm = fsqrt((T)2 * PP);
    const T tau = (T)ph.tau;
    m.R = fsqrt(tau * tau + (T)(18.0 * ph.c2) * m.norm * m.irho);
    m.te = (T)0.5 * (tau + m.R);
    m.ite = rcp(m.te);
}

// Directions come in opposite pairs (a, opp(a)); sums over a pair of the
// even (c c) and odd (c) moments share h_a + h_opp and h_a - h_opp.
template <class L, class T>
__device__ __forceinline__ void moments(const T h[L::Q], const Phys& ph, Moments<L, T>& m) {
    constexpr int D = L::D;
    using SY = Sym<D>;
    T drho = h[0];
    T j[D];
    T M[SY::K];
#pragma unroll
    for (int p = 0; p < D; ++p) j[p] = 0;
#pragma unroll
    for (int k = 0; k < SY::K; ++k) M[k] = 0;
#pragma unroll
    for (int a = 1; a < L::Q; ++a) {
        if (L::opp[a] < a) continue;
        const T sp = h[a] + h[L::opp[a]];
        const T dm = h[a] - h[L::opp[a]];
        drho += sp;
#pragma unroll
        for (int p = 0; p < D; ++p) {
            const int cp = comp<L>(a, p);
            if (cp == 1) j[p] += dm;
            if (cp == -1) j[p] -= dm;
#pragma unroll
            for (int q = p; q < D; ++q) {
                const int cc = cp * comp<L>(a, q);
                if (cc == 1) M[SY::idx[p][q]] += sp;
                if (cc == -1) M[SY::idx[p][q]] -= sp;
            }
        }
    }
    const T rho = (T)1 + drho;
    const T irho = rcp(rho);
#pragma unroll
    for (int p = 0; p < D; ++p) {
#pragma unroll
        for (int q = p; q < D; ++q) {
            const int k = SY::idx[p][q];
            T v = M[k] - j[p] * j[q] * irho;
            if (p == q) v -= (T)(1.0 / 3.0) * drho;
            m.Pi[k] = v;
        }
    }
    m.drho = drho;
    m.rho = rho;
    m.irho = irho;
#pragma unroll
    for (int p = 0; p < D; ++p) m.j[p] = j[p];
    moments_finish<L, T>(ph, m);
}

// Moment record of a node state (the recompute of an adjoint segment keeps
// one per node and step instead of the populations): drho, j, Pi, that is
// 1 + D + K values in planes of N.
template <class L>
constexpr int record_size() {
    return 1 + L::D + Sym<L::D>::K;
}

template <class L, class T>
__device__ __forceinline__ void record_store(T* __restrict__ rec, int N, int n, const Moments<L, T>& m) {
    rec[n] = m.drho;
#pragma unroll
    for (int p = 0; p < L::D; ++p) rec[(size_t)(1 + p) * N + n] = m.j[p];
#pragma unroll
    for (int k = 0; k < Sym<L::D>::K; ++k) rec[(size_t)(1 + L::D + k) * N + n] = m.Pi[k];
}

// The moments of a record's values r (drho, j, Pi), completed exactly as
// moments() completes the sums of a state.
template <class L, class T>
__device__ __forceinline__ void record_moments(const T (&r)[record_size<L>()], const Phys& ph, Moments<L, T>& m) {
    m.drho = r[0];
#pragma unroll
    for (int p = 0; p < L::D; ++p) m.j[p] = r[1 + p];
#pragma unroll
    for (int k = 0; k < Sym<L::D>::K; ++k) m.Pi[k] = r[1 + L::D + k];
    m.rho = (T)1 + m.drho;
    m.irho = rcp(m.rho);
    moments_finish<L, T>(ph, m);
}

template <class L, class T>
__device__ __forceinline__ void record_load(const T* __restrict__ rec, int N, int n, const Phys& ph,
                                            Moments<L, T>& m) {
    T r[record_size<L>()];
#pragma unroll
    for (int c = 0; c < record_size<L>(); ++c) r[c] = rec[(size_t)c * N + n];
    record_moments<L, T>(r, ph, m);
}

// The values of a record, in the order record_moments() takes them.
template <class L, class T>
__device__ __forceinline__ void record_values(const Moments<L, T>& m, T (&r)[record_size<L>()]) {
    r[0] = m.drho;
#pragma unroll
    for (int p = 0; p < L::D; ++p) r[1 + p] = m.j[p];
#pragma unroll
    for (int k = 0; k < Sym<L::D>::K; ++k) r[1 + L::D + k] = m.Pi[k];
}

// Regularized collision (Eq. modified_collision) followed by the partial
// bounce-back (Eq. external_force), in closed form: with a = 1 - 1/tau_eff,
//   f**_a - w_a = w_a [drho + 3(1 - 2s) c.j + 4.5 (c.j)^2/rho - 1.5 j.j/rho]
//               + 4.5 a w_a (c c - c_s^2 I) : Pi,
// since f*_opp - f*_a = -6 w_a c_a.j for the regularized post-collision state.
// The even part is shared by a and opp(a); the odd part changes sign.
template <class L, class T>
__device__ __forceinline__ void collide(const Moments<L, T>& m, T s, T out[L::Q]) {
    constexpr int D = L::D;
    using SY = Sym<D>;
    const T ev = (T)4.5 * ((T)1 - m.ite);
    T jj = 0, tr = 0;
#pragma unroll
    for (int p = 0; p < D; ++p) {
        jj += m.j[p] * m.j[p];
        tr += m.Pi[SY::idx[p][p]];
    }
    const T A = m.drho - (T)1.5 * jj * m.irho - ev * (T)(1.0 / 3.0) * tr;
    const T B = (T)4.5 * m.irho;
    const T odd = (T)3 - (T)6 * s;
    out[0] = (T)L::w[0] * A;
#pragma unroll
    for (int al = 1; al < L::Q; ++al) {
        if (L::opp[al] < al) continue;
        T cj = 0, cPc = 0;
#pragma unroll
        for (int p = 0; p < D; ++p) {
            const int cp = comp<L>(al, p);
            if (cp == 1) cj += m.j[p];
            if (cp == -1) cj -= m.j[p];
#pragma unroll
            for (int q = 0; q < D; ++q) {
                const int cc = cp * comp<L>(al, q);
                if (cc == 1) cPc += m.Pi[SY::idx[p][q]];
                if (cc == -1) cPc -= m.Pi[SY::idx[p][q]];
            }
        }
        const T wa = (T)L::w[al];
        const T E = A + B * cj * cj + ev * cPc;
        const T O = odd * cj;
        out[al] = wa * (E + O);
        out[L::opp[al]] = wa * (E - O);
    }
}

// Node dissipation 2 rho nu_eff S:S with S from Eq. Lallemand_equation:
// (tau_eff - 1/2) Pi:Pi / (2 rho c_s^2 tau_eff^2).
template <class L, class T>
__device__ __forceinline__ T dissipation(const Moments<L, T>& m) {
    return (T)1.5 * (m.te - (T)0.5) * m.PP * m.irho * m.ite * m.ite;
}

// Gradient of a scalar with respect to the node moments (rho, j, Pi), with
// Pi held as its own variable; chain() maps it to (rho, j, M = sum c c f),
// after which d/df_a = g_rho + g_j . c_a + c_a . G_M . c_a.
template <class L, class T>
struct MomentGrad {
    T gr;
    T gj[L::D];
    T GP[Sym<L::D>::K];   // symmetric tensor, full-contraction convention
};

// Adds d/d(rho, Pi) of a function of tau_eff only: dT * d tau_eff.
template <class L, class T>
__device__ __forceinline__ void add_tau_grad(const Moments<L, T>& m, const Phys& ph, T dT,
                                             MomentGrad<L, T>& g) {
    // tau_eff = (tau + R)/2, R^2 = tau^2 + 18 C^2 ||Pi|| / rho
    // d tau_eff / d||Pi|| = 4.5 C^2 / (rho R);  d tau_eff / d rho = -4.5 C^2 ||Pi|| / (rho^2 R)
    if (ph.c2 == 0.0) return;
    const T k = (T)(4.5 * ph.c2) * m.irho * rcp(m.R);
    g.gr += -dT * k * m.norm * m.irho;
    if (m.norm > (T)0) {
        // d||Pi|| / dPi = 2 Pi / ||Pi||
        const T f = dT * k * (T)2 * rcp(m.norm);
#pragma unroll
        for (int k2 = 0; k2 < Sym<L::D>::K; ++k2) g.GP[k2] += f * m.Pi[k2];
    }
}

// Reverse mode of collide(): given kappa (adjoint of f**), accumulate the
// moment gradient of sum_a kappa_a f**_a and return d/ds of it
// (= sum_a kappa_a (f*_opp - f*_a) = -6 sum_a w_a kappa_a c_a . j).
template <class L, class T>
__device__ __forceinline__ T collide_adjoint(const Moments<L, T>& m, const Phys& ph, T s,
                                             const T kappa[L::Q], MomentGrad<L, T>& g) {
    constexpr int D = L::D;
    using SY = Sym<D>;
    // K0 = sum w kappa, K1 = sum w kappa c, K2 = sum w kappa c c (pairwise)
    T K0 = (T)L::w[0] * kappa[0];
    T K1[D];
    T K2[SY::K];
#pragma unroll
    for (int p = 0; p < D; ++p) K1[p] = 0;
#pragma unroll
    for (int k = 0; k < SY::K; ++k) K2[k] = 0;
#pragma unroll
    for (int a = 1; a < L::Q; ++a) {
        if (L::opp[a] < a) continue;
        const T sp = (T)L::w[a] * (kappa[a] + kappa[L::opp[a]]);
        const T dm = (T)L::w[a] * (kappa[a] - kappa[L::opp[a]]);
        K0 += sp;
#pragma unroll
        for (int p = 0; p < D; ++p) {
            const int cp = comp<L>(a, p);
            if (cp == 1) K1[p] += dm;
            if (cp == -1) K1[p] -= dm;
#pragma unroll
            for (int q = p; q < D; ++q) {
                const int cc = cp * comp<L>(a, q);
                if (cc == 1) K2[SY::idx[p][q]] += sp;
                if (cc == -1) K2[SY::idx[p][q]] -= sp;
            }
        }
    }
    const T irho = m.irho;
    const T a = (T)1 - m.ite;
    // T = K2 - K0/3 I ; P = T : Pi
    T Tt[SY::K];
#pragma unroll
    for (int k = 0; k < SY::K; ++k) Tt[k] = K2[k];
#pragma unroll
    for (int p = 0; p < D; ++p) Tt[SY::idx[p][p]] -= K0 * (T)(1.0 / 3.0);
    T P = 0;
#pragma unroll
    for (int p = 0; p < D; ++p)
#pragma unroll
        for (int q = 0; q < D; ++q) P += Tt[SY::idx[p][q]] * m.Pi[SY::idx[p][q]];
    // explicit dependence on (rho, j) of the equilibrium-like part
    T jK2j = 0, jj = 0, K1j = 0;
    T K2j[D];
#pragma unroll
    for (int p = 0; p < D; ++p) {
        T v = 0;
#pragma unroll
        for (int q = 0; q < D; ++q) v += K2[SY::idx[p][q]] * m.j[q];
        K2j[p] = v;
        jK2j += m.j[p] * v;
        jj += m.j[p] * m.j[p];
        K1j += K1[p] * m.j[p];
    }
    g.gr += K0 - ((T)4.5 * jK2j - (T)1.5 * K0 * jj) * irho * irho;
    const T odd = (T)3 - (T)6 * s;
#pragma unroll
    for (int p = 0; p < D; ++p)
        g.gj[p] += odd * K1[p] + ((T)9 * K2j[p] - (T)3 * K0 * m.j[p]) * irho;
    // direct Pi dependence: 4.5 a T ; through a(tau_eff): 4.5 P / tau_eff^2
#pragma unroll
    for (int k = 0; k < SY::K; ++k) g.GP[k] += (T)4.5 * a * Tt[k];
    add_tau_grad<L, T>(m, ph, (T)4.5 * P * m.ite * m.ite, g);
    return (T)-6 * K1j;
}

// Moment gradient of the node dissipation (for sampled objectives).
template <class L, class T>
__device__ __forceinline__ void dissipation_adjoint(const Moments<L, T>& m, const Phys& ph, T wgt,
                                                    MomentGrad<L, T>& g) {
    // D = 1.5 (te - 1/2) Z / (rho te^2), Z = Pi:Pi
    const T te = m.te, ite = m.ite;
    const T dZ = wgt * (T)1.5 * (te - (T)0.5) * m.irho * ite * ite;
#pragma unroll
    for (int k = 0; k < Sym<L::D>::K; ++k) g.GP[k] += dZ * (T)2 * m.Pi[k];
    const T D = (T)1.5 * (te - (T)0.5) * m.PP * m.irho * ite * ite;
    g.gr += -wgt * D * m.irho;
    const T dte = wgt * (T)1.5 * m.PP * ((T)1 - te) * m.irho * ite * ite * ite;
    add_tau_grad<L, T>(m, ph, dte, g);
}

// Maps a gradient in (rho, j, Pi) to (rho, j, M = sum c c f) through
// Pi = M - c_s^2 rho I - j j / rho, then to the populations:
// mu_a = g_rho + g_j . c_a + c_a . G_M . c_a (even part shared by a pair).
template <class L, class T>
__device__ __forceinline__ void expand(const Moments<L, T>& m, MomentGrad<L, T>& g, T mu[L::Q]) {
    constexpr int D = L::D;
    using SY = Sym<D>;
    const T irho = m.irho;
    T tr = 0, jGj = 0;
    T Gj[D];
#pragma unroll
    for (int p = 0; p < D; ++p) {
        tr += g.GP[SY::idx[p][p]];
        T v = 0;
#pragma unroll
        for (int q = 0; q < D; ++q) v += g.GP[SY::idx[p][q]] * m.j[q];
        Gj[p] = v;
        jGj += m.j[p] * v;
    }
    const T gr = g.gr - tr * (T)(1.0 / 3.0) + jGj * irho * irho;
    T gj[D];
#pragma unroll
    for (int p = 0; p < D; ++p) gj[p] = g.gj[p] - (T)2 * Gj[p] * irho;
    mu[0] = gr;
#pragma unroll
    for (int a = 1; a < L::Q; ++a) {
        if (L::opp[a] < a) continue;
        T E = gr, O = 0;
#pragma unroll
        for (int p = 0; p < D; ++p) {
            const int cp = comp<L>(a, p);
            if (cp == 1) O += gj[p];
            if (cp == -1) O -= gj[p];
#pragma unroll
            for (int q = 0; q < D; ++q) {
                const int cc = cp * comp<L>(a, q);
                if (cc == 1) E += g.GP[SY::idx[p][q]];
                if (cc == -1) E -= g.GP[SY::idx[p][q]];
            }
        }
        mu[a] = E + O;
        mu[L::opp[a]] = E - O;
    }
}

}  // namespace lbm
