// HIP kernels of the reactive-mixture lattice Boltzmann step for gfx950.
//
// One time step is three launches over a (possibly batched) work list:
//   k_boundary  interface nodes: advection + wall / inlet / outlet
//               reconstruction (section 4) into an FP64 side buffer;
//   k_moments   every node: advection, moments, temperature (eq. temperature),
//               then rho, u, T, Y and Phi_a = rho u_a (1 - 3 R T) - rho u_a^3
//               are published for the neighbours;
//   k_collide   every node: advection and moments again, same-time
//               gradients from the neighbours' published fields, relaxation
//               parameters, Stefan-Maxwell solve, reaction sub-steps and the
//               collisions of all stored lattices, written to the other
//               population buffer.
// Populations are structure-of-arrays [L][27][N] (x fastest), pulled from the
// source buffer, so every load and store of a wavefront is coalesced.  The
// storage type S is double (FP64) or float (FP32 deviation from a reference
// population per lattice and velocity, decoded to FP64 on load).

#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "physics.hpp"

namespace rlbm {

// ---------------------------------------------------------------------------
// storage codecs
// ---------------------------------------------------------------------------
template <typename S>
struct Codec;

template <>
struct Codec<double> {
    static __device__ __forceinline__ double ld(const void* p, size_t idx, const double*, int) {
        return static_cast<const double*>(p)[idx];
    }
    static __device__ __forceinline__ void st(void* p, size_t idx, double v, const double*, int) {
        static_cast<double*>(p)[idx] = v;
    }
};

template <>
struct Codec<float> {
    static __device__ __forceinline__ double ld(const void* p, size_t idx, const double* ref, int li) {
        return (double)static_cast<const float*>(p)[idx] + ref[li];
    }
    static __device__ __forceinline__ void st(void* p, size_t idx, double v, const double* ref, int li) {
        static_cast<float*>(p)[idx] = __double2float_rn(v - ref[li]);
    }
};

// ---------------------------------------------------------------------------
// work-list helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_lattice(const int* blk, int n_lat, int b) {
    int lo = 0, hi = n_lat - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blk[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

struct Nbr {
    int x, y, z;
    int xw[3], yw[3], zw[3];   // wrapped x-1, x, x+1 (pull: bulk nodes never leave the box)
    int xg[3], yg[3], zg[3];   // gradient stencil: wrapped (periodic) or clamped
};

__device__ __forceinline__ void make_nbr(const LatDev& L, long long node, Nbr& n) {
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    n.x = (int)(node % nx);
    const long long r = node / nx;
    n.y = (int)(r % ny);
    n.z = (int)(r / ny);
    const int d[3] = {n.x, n.y, n.z};
    const int e[3] = {nx, ny, nz};
    int* w[3] = {n.xw, n.yw, n.zw};
    int* g[3] = {n.xg, n.yg, n.zg};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int v = d[ax], m = e[ax];
        const int vm = v == 0 ? m - 1 : v - 1;
        const int vp = v == m - 1 ? 0 : v + 1;
        w[ax][0] = vm; w[ax][1] = v; w[ax][2] = vp;
        if (L.per[ax]) {
            g[ax][0] = vm; g[ax][1] = v; g[ax][2] = vp;
        } else {
            g[ax][0] = v == 0 ? 0 : v - 1;
            g[ax][1] = v;
            g[ax][2] = v == m - 1 ? m - 1 : v + 1;
        }
    }
}

// Source node of velocity i for a pull at this node: x - c_i (wrapped).
__device__ __forceinline__ long long pull_src(const LatDev& L, const Nbr& n, int i) {
    const int xs = n.xw[1 - cx_of(i)], ys = n.yw[1 - cy_of(i)], zs = n.zw[1 - cz_of(i)];
    return ((long long)zs * L.ny + ys) * L.nx + xs;
}

// Population (lattice l, velocity i) after advection (and boundary
// reconstruction, if this is an interface node with slot k >= 0).
template <typename S>
__device__ __forceinline__ double gather(const LatDev& L, const void* src, int k, const Nbr& n,
                                         long long node, int l, int i) {
    const int li = l * Q + i;
    if (k >= 0) return L.bcbuf[(size_t)li * L.n_if + k];
    return Codec<S>::ld(src, (size_t)li * L.N + pull_src(L, n, i), L.ref, li);
}

template <int M>
__device__ __forceinline__ int lat_of(int a, int slaved) { return a - (a > slaved ? 1 : 0); }

// ---------------------------------------------------------------------------
// moments of one node's (post-advection, post-boundary) populations
// ---------------------------------------------------------------------------
template <int M>
struct Moments {
    double rho, j[3], rhoE, q[3], P[6];   // P: xx, yy, zz, xy, xz, yz
    double rho_a[M], j_a[M][3];
};

template <int M, typename S, bool FULL>
__device__ __forceinline__ void node_moments(const LatDev& L, const void* src, int k, const Nbr& n,
                                             long long node, Moments<M>& m) {
    const int s = L.slaved;
    m.rho = m.rhoE = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) m.j[d] = m.q[d] = 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) m.P[d] = 0.0;
    const int lf = M - 1, lg = M;
#pragma unroll 1
    for (int i = 0; i < Q; ++i) {
        const double cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
        const double f = gather<S>(L, src, k, n, node, lf, i);
        m.rho += f;
        m.j[0] += f * cx; m.j[1] += f * cy; m.j[2] += f * cz;
        if (FULL) {
            m.P[0] += f * cx * cx; m.P[1] += f * cy * cy; m.P[2] += f * cz * cz;
            m.P[3] += f * cx * cy; m.P[4] += f * cx * cz; m.P[5] += f * cy * cz;
        }
        const double g = gather<S>(L, src, k, n, node, lg, i);
        m.rhoE += g;
        if (FULL) { m.q[0] += g * cx; m.q[1] += g * cy; m.q[2] += g * cz; }
    }
#pragma unroll
    for (int a = 0; a < M; ++a) {
        m.rho_a[a] = 0.0;
        m.j_a[a][0] = m.j_a[a][1] = m.j_a[a][2] = 0.0;
        if (a == s) continue;
        const int l = lat_of<M>(a, s);
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll 1
        for (int i = 0; i < Q; ++i) {
            const double f = gather<S>(L, src, k, n, node, l, i);
            r += f;
            jx += f * (double)cx_of(i); jy += f * (double)cy_of(i); jz += f * (double)cz_of(i);
        }
        m.rho_a[a] = r; m.j_a[a][0] = jx; m.j_a[a][1] = jy; m.j_a[a][2] = jz;
    }
    // slaved species (section 3.6, eq. strongest)
    double rs = m.rho, jsx = m.j[0], jsy = m.j[1], jsz = m.j[2];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        if (a == s) continue;
        rs -= m.rho_a[a]; jsx -= m.j_a[a][0]; jsy -= m.j_a[a][1]; jsz -= m.j_a[a][2];
    }
#pragma unroll
    for (int a = 0; a < M; ++a) {
        if (a == s) { m.rho_a[a] = rs; m.j_a[a][0] = jsx; m.j_a[a][1] = jsy; m.j_a[a][2] = jsz; }
    }
}

// ---------------------------------------------------------------------------
// k_moments
// ---------------------------------------------------------------------------
template <int M, typename S>
__global__ __launch_bounds__(256) void k_moments(const LatDev* __restrict__ lats, const int* __restrict__ blk,
                                                 int n_lat, long long t, int* __restrict__ flag) {
    const int b = blockIdx.x;
    const int lj = find_lattice(blk, n_lat, b);
    const LatDev& L = lats[lj];
    if (t >= L.t_end) return;
    const long long node = (long long)(b - blk[lj]) * 256 + threadIdx.x;
    if (node >= L.N) return;
    const MechDev& mc = *L.mech;
    const void* src = L.pop[(L.parity0 + t) & 1];
    Nbr n;
    make_nbr(L, node, n);
    const int k = L.n_if ? L.if_index[node] : -1;
    Moments<M> m;
    node_moments<M, S, false>(L, src, k, n, node, m);
    const double inv_rho = 1.0 / m.rho;
    double Y[M];
#pragma unroll
    for (int a = 0; a < M; ++a) Y[a] = m.rho_a[a] * inv_rho;
    const double u[3] = {m.j[0] * inv_rho, m.j[1] * inv_rho, m.j[2] * inv_rho};
    const double U = m.rhoE * inv_rho - 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double* aux = L.aux;
    const size_t N = (size_t)L.N;
    int fail = 0;
    const double T = solve_T<M>(mc, Y, U, aux[AUX_T * N + node], &fail);
    if (fail) atomicOr(flag, 1);
    const double th = mc.R_univ * mix_inv_m<M>(mc, Y) * T;
    aux[AUX_RHO * N + node] = m.rho;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        aux[(AUX_U + d) * N + node] = u[d];
        aux[(AUX_PHI + d) * N + node] = m.rho * u[d] * (1.0 - 3.0 * th) - m.rho * u[d] * u[d] * u[d];
    }
    aux[AUX_T * N + node] = T;
#pragma unroll
    for (int a = 0; a < M; ++a) aux[(AUX_Y + a) * N + node] = Y[a];
}

// ---------------------------------------------------------------------------
// k_collide
// ---------------------------------------------------------------------------
template <int M, typename S>
__global__ __launch_bounds__(256) void k_collide(const LatDev* __restrict__ lats, const int* __restrict__ blk,
                                                 int n_lat, long long t, int* __restrict__ flag) {
    const int b = blockIdx.x;
    const int lj = find_lattice(blk, n_lat, b);
    const LatDev& L = lats[lj];
    if (t >= L.t_end) return;
    const long long node = (long long)(b - blk[lj]) * 256 + threadIdx.x;
    if (node >= L.N) return;
    const MechDev& mc = *L.mech;
    const int par = (L.parity0 + t) & 1;
    const void* src = L.pop[par];
    void* dst = L.pop[par ^ 1];
    const int s = L.slaved;
    Nbr n;
    make_nbr(L, node, n);
    const int k = L.n_if ? L.if_index[node] : -1;
    Moments<M> m;
    node_moments<M, S, true>(L, src, k, n, node, m);
    const double* aux = L.aux;
    const size_t N = (size_t)L.N;

    const double rho = m.rho, inv_rho = 1.0 / rho;
    const double u[3] = {m.j[0] * inv_rho, m.j[1] * inv_rho, m.j[2] * inv_rho};
    const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double Y[M];
#pragma unroll
    for (int a = 0; a < M; ++a) Y[a] = m.rho_a[a] * inv_rho;
    const double T = aux[AUX_T * N + node];
    const double U = m.rhoE * inv_rho - 0.5 * usq;
    const double inv_mix_m = mix_inv_m<M>(mc, Y);
    const double th = mc.R_univ * inv_mix_m * T;
    const double P = rho * th;

    // same-time gradients, isotropic D3Q27 stencil: d phi/dx_a = 3 sum_i w_i c_ia phi(x + c_i)
    double d[3] = {0.0, 0.0, 0.0};
    double G[M][3];
#pragma unroll
    for (int a = 0; a < M; ++a) G[a][0] = G[a][1] = G[a][2] = 0.0;
#pragma unroll 1
    for (int i = 0; i < Q; ++i) {
        if (i == 13) continue;
        const int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
        const double w = 3.0 * (cx ? 1.0 / 6.0 : 2.0 / 3.0) * (cy ? 1.0 / 6.0 : 2.0 / 3.0) *
                         (cz ? 1.0 / 6.0 : 2.0 / 3.0);
        const size_t nb = ((size_t)n.zg[1 + cz] * L.ny + n.yg[1 + cy]) * L.nx + n.xg[1 + cx];
        if (cx) d[0] += w * cx * aux[(AUX_PHI + 0) * N + nb];
        if (cy) d[1] += w * cy * aux[(AUX_PHI + 1) * N + nb];
        if (cz) d[2] += w * cz * aux[(AUX_PHI + 2) * N + nb];
#pragma unroll
        for (int a = 0; a < M; ++a) {
            const double y = aux[(AUX_Y + a) * N + nb];
            G[a][0] += w * cx * y; G[a][1] += w * cy * y; G[a][2] += w * cz * y;
        }
    }

    // relaxation parameters (sections 2.3 and 3.4)
    const double lnr = log(T * mc.inv_T_ref);
    const double common = mc.R_univ * T / inv_mix_m * P * mc.inv_P_ref * exp(-mc.D_exp * lnr);
    double inv_tau[M], beta[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        double sum = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c)
            if (c != a) sum += Y[c] * mc.Kab[a][c];
        inv_tau[a] = common * sum;
        beta[a] = inv_tau[a] / (2.0 + inv_tau[a]);
    }
    const double mu = mc.mu_ref * exp(mc.mu_exp * lnr);
    const double omega = 1.0 / (mu / P + 0.5);
    const double omega1 = 1.0 / (mu * mc.inv_Pr / P + 0.5);

    // Stefan-Maxwell diffusion velocities (eq. transform1)
    double V[M][3];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const bool small = m.rho_a[a] <= 1e-14 * rho;
        const double inv = small ? 0.0 : 1.0 / m.rho_a[a];
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) V[a][dd] = small ? 0.0 : m.j_a[a][dd] * inv - u[dd];
    }
    {
        double itab[M][M];
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int c = 0; c < M; ++c) itab[a][c] = common * mc.Kab[a][c];
        sm_solve<M>(Y, itab, inv_tau, V);
    }

    // reaction sub-steps (eq. R3)
    double drho[M];
    int fail = 0;
    reaction_increment<M>(mc, m.rho_a, rho, U, T, L.substeps, drho, &fail);
    if (fail) atomicOr(flag, 1);

    // energy-lattice quasi-equilibrium flux, singularity-free form:
    //   Q = (omega - omega1)(q - u.(P - P^eq) + q^ex - q^eq)
    //       + omega1 rho sum_a H_a Y_a V_a + (2 - omega1)/2 P sum_a H_a grad Y_a
    double Qv[3];
    {
        double diff[3] = {0.0, 0.0, 0.0}, corr[3] = {0.0, 0.0, 0.0};
        double H = 0.0;
#pragma unroll
        for (int a = 0; a < M; ++a) {
            const double Ha = species_U(mc, a, T) + mc.Ra[a] * T;
            H += Y[a] * Ha;
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) {
                diff[dd] += Ha * Y[a] * V[a][dd];
                corr[dd] += Ha * G[a][dd];
            }
        }
        const double hq = rho * (H + 0.5 * usq);
        const double Pt[3][3] = {{m.P[0], m.P[3], m.P[4]}, {m.P[3], m.P[1], m.P[5]}, {m.P[4], m.P[5], m.P[2]}};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double uP = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double Peq = rho * ((a == c ? th : 0.0) + u[c] * u[a]);
                uP += u[c] * (Pt[c][a] - Peq);
            }
            const double qex = -0.5 * u[a] * d[a];
            Qv[a] = (omega - omega1) * (m.q[a] - uP + qex - hq * u[a]) + omega1 * rho * diff[a] +
                    0.5 * (2.0 - omega1) * P * corr[a];
        }
    }

    // per-species product-form parameters: equilibrium (u, u^2 + theta_b) and
    // quasi-equilibrium (u + V_b, (u + V_b)^2 + theta_b)
    double hE[M][3], hS[M][3], xS[M][3];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const double tha = mc.Ra[a] * T;
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
            hE[a][dd] = 0.5 * (u[dd] * u[dd] + tha);
            const double xi = u[dd] + V[a][dd];
            xS[a][dd] = 0.5 * xi;
            hS[a][dd] = 0.5 * (xi * xi + tha);
        }
    }
    // extended equilibrium of the momentum lattice (eqs. feqmix, Pex)
    double hX[3];
    const double exf = (2.0 - omega) / (2.0 * rho * omega);
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) hX[dd] = 0.5 * (th + u[dd] * u[dd] + exf * d[dd]);
    GeqAxis gx, gy, gz;
    geq_axis(u[0], th, gx);
    geq_axis(u[1], th, gy);
    geq_axis(u[2], th, gz);
    const double hu[3] = {0.5 * u[0], 0.5 * u[1], 0.5 * u[2]};

#pragma unroll 1
    for (int i = 0; i < Q; ++i) {
        const int c0 = cx_of(i), c1 = cy_of(i), c2 = cz_of(i);
        // W_bi and W*_bi for all species
        double Wd[M], D[M];
#pragma unroll
        for (int a = 0; a < M; ++a) {
            const double e0 = c0 == 0 ? 1.0 - 2.0 * hE[a][0] : hE[a][0] + c0 * hu[0];
            const double e1 = c1 == 0 ? 1.0 - 2.0 * hE[a][1] : hE[a][1] + c1 * hu[1];
            const double e2 = c2 == 0 ? 1.0 - 2.0 * hE[a][2] : hE[a][2] + c2 * hu[2];
            const double s0 = c0 == 0 ? 1.0 - 2.0 * hS[a][0] : hS[a][0] + c0 * xS[a][0];
            const double s1 = c1 == 0 ? 1.0 - 2.0 * hS[a][1] : hS[a][1] + c1 * xS[a][1];
            const double s2 = c2 == 0 ? 1.0 - 2.0 * hS[a][2] : hS[a][2] + c2 * xS[a][2];
            Wd[a] = e0 * e1 * e2;
            D[a] = m.rho_a[a] * (Wd[a] - s0 * s1 * s2);
        }
        // species collision (eq. finalNumericalEquationsReactive, eq. fStar)
#pragma unroll
        for (int a = 0; a < M; ++a) {
            if (a == s) continue;
            const int l = lat_of<M>(a, s);
            double F = 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c)
                if (c != a) F += mc.Kab[a][c] * D[c];
            F *= common * Y[a];
            const double f = gather<S>(L, src, k, n, node, l, i);
            const double out = f + 2.0 * beta[a] * (m.rho_a[a] * Wd[a] - f) + (beta[a] - 1.0) * F + Wd[a] * drho[a];
            const int li = l * Q + i;
            Codec<S>::st(dst, (size_t)li * N + node, out, L.ref, li);
        }
        // momentum lattice with the extended equilibrium (eq. f)
        {
            const double e0 = c0 == 0 ? 1.0 - 2.0 * hX[0] : hX[0] + c0 * hu[0];
            const double e1 = c1 == 0 ? 1.0 - 2.0 * hX[1] : hX[1] + c1 * hu[1];
            const double e2 = c2 == 0 ? 1.0 - 2.0 * hX[2] : hX[2] + c2 * hu[2];
            const double f = gather<S>(L, src, k, n, node, M - 1, i);
            const double out = f + omega * (rho * e0 * e1 * e2 - f);
            const int li = (M - 1) * Q + i;
            Codec<S>::st(dst, (size_t)li * N + node, out, L.ref, li);
        }
        // energy lattice (eq. g)
        {
            const double g = gather<S>(L, src, k, n, node, M, i);
            double out = g + omega * (geq_i(i, rho, U, gx, gy, gz) - g);
            if (c2_of(i) == 1) out += 0.5 * (c0 * Qv[0] + c1 * Qv[1] + c2 * Qv[2]);
            const int li = M * Q + i;
            Codec<S>::st(dst, (size_t)li * N + node, out, L.ref, li);
        }
    }
}

// ---------------------------------------------------------------------------
// boundary reconstruction (section 4)
// ---------------------------------------------------------------------------
// Equilibrium of lattice l at velocity i for the state (rho, Y, u, T) with
// species velocities us (section 4.1, eqs. faEqGeneral, fEqGeneral,
// gEqGeneral).
template <int M>
struct EqState {
    double rho, th, U;
    double Y[M];
    double u[3];
    double us[M][3];
    GeqAxis gx, gy, gz;
};

template <int M>
__device__ __forceinline__ void eq_prepare(const MechDev& mc, EqState<M>& e, double T) {
    e.th = mc.R_univ * mix_inv_m<M>(mc, e.Y) * T;
    e.U = mix_U<M>(mc, e.Y, T);
    geq_axis(e.u[0], e.th, e.gx);
    geq_axis(e.u[1], e.th, e.gy);
    geq_axis(e.u[2], e.th, e.gz);
}

template <int M>
__device__ __forceinline__ double eq_value(const MechDev& mc, const EqState<M>& e, double T, int l, int slaved,
                                           int i) {
    const int c0 = cx_of(i), c1 = cy_of(i), c2 = cz_of(i);
    if (l == M) return geq_i(i, e.rho, e.U, e.gx, e.gy, e.gz);
    if (l == M - 1)
        return e.rho * psi(c0, e.u[0], e.u[0] * e.u[0] + e.th) * psi(c1, e.u[1], e.u[1] * e.u[1] + e.th) *
               psi(c2, e.u[2], e.u[2] * e.u[2] + e.th);
    const int a = l + (l >= slaved ? 1 : 0);
    double Ya = 0.0, tha = 0.0, w0 = 0.0, w1 = 0.0, w2 = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        if (c == a) {
            Ya = e.Y[c];
            tha = mc.Ra[c] * T;
            w0 = e.us[c][0]; w1 = e.us[c][1]; w2 = e.us[c][2];
        }
    }
    return e.rho * Ya * psi(c0, w0, w0 * w0 + tha) * psi(c1, w1, w1 * w1 + tha) * psi(c2, w2, w2 * w2 + tha);
}

template <int M, typename S>
__global__ __launch_bounds__(64) void k_boundary(const LatDev* __restrict__ lats, const int* __restrict__ blk,
                                                 int n_lat, long long t, int* __restrict__ flag) {
    const int b = blockIdx.x;
    const int lj = find_lattice(blk, n_lat, b);
    const LatDev& L = lats[lj];
    if (t >= L.t_end) return;
    const int k = (b - blk[lj]) * 64 + threadIdx.x;
    if (k >= L.n_if) return;
    const MechDev& mc = *L.mech;
    const void* src = L.pop[(L.parity0 + t) & 1];
    const long long node = L.if_node[k];
    const unsigned Dm = L.if_mask[k];
    const int type = L.if_type[k];
    const int s = L.slaved;
    const size_t N = (size_t)L.N;
    Nbr n;
    make_nbr(L, node, n);
    const int nL = M + 1;
    int fail = 0;

    auto streamed = [&](int l, int i) -> double {
        const int li = l * Q + i;
        return Codec<S>::ld(src, (size_t)li * N + pull_src(L, n, i), L.ref, li);
    };
    auto incoming = [&](int i) -> bool { return (Dm >> i) & 1u; };

    EqState<M> A;     // imposed equilibrium: target (wall), inlet or outlet state
    double T_A;
    if (type == RLBM_FACE_WALL) {
        // TMS step 1: bounce-back density and mass fractions (eqs. BBrho, BBY)
        double rb = 0.0, rY[M];
#pragma unroll
        for (int a = 0; a < M; ++a) rY[a] = 0.0;
        for (int l = 0; l < nL - 1; ++l) {
            double sum = 0.0;
            for (int i = 0; i < Q; ++i) {
                const int li = l * Q + i;
                sum += incoming(i) ? Codec<S>::ld(src, (size_t)(l * Q + (Q - 1 - i)) * N + node, L.ref,
                                                  l * Q + (Q - 1 - i))
                                   : streamed(l, i);
                (void)li;
            }
            if (l == M - 1) {
                rb = sum;
            } else {
                const int a = l + (l >= s ? 1 : 0);
#pragma unroll
                for (int c = 0; c < M; ++c)
                    if (c == a) rY[c] = sum;
            }
        }
        double rs = rb;
#pragma unroll
        for (int a = 0; a < M; ++a)
            if (a != s) rs -= rY[a];
#pragma unroll
        for (int a = 0; a < M; ++a) {
            if (a == s) rY[a] = rs;
            A.Y[a] = rY[a] / rb;
        }
        A.rho = rb;
        A.u[0] = A.u[1] = A.u[2] = 0.0;
#pragma unroll
        for (int a = 0; a < M; ++a) A.us[a][0] = A.us[a][1] = A.us[a][2] = 0.0;
        T_A = L.if_T[k];
    } else if (type == RLBM_FACE_INLET) {
        A.rho = L.rho_in;
        A.u[0] = L.u_in; A.u[1] = 0.0; A.u[2] = 0.0;
#pragma unroll
        for (int a = 0; a < M; ++a) {
            A.Y[a] = L.Y_in[a];
            A.us[a][0] = L.u_in; A.us[a][1] = 0.0; A.us[a][2] = 0.0;
        }
        T_A = L.T_in;
    } else {
        // outlet: LODI state from the previous outlet state and the previous
        // post-boundary moments of the first interior node (section 4.4)
        const int ko = L.if_out[k];
        const size_t No = (size_t)L.n_out;
        double* os = L.out_state;
        const double rho0 = os[0 * No + ko];
        const double u0[3] = {os[1 * No + ko], os[2 * No + ko], os[3 * No + ko]};
        const double T0 = os[4 * No + ko];
        double Y0[M], Y1[M];
        const size_t in = (size_t)node - 1;
#pragma unroll
        for (int a = 0; a < M; ++a) {
            Y0[a] = os[(5 + a) * No + ko];
            Y1[a] = L.aux[(AUX_Y + a) * N + in];
        }
        const double rho1 = L.aux[AUX_RHO * N + in];
        const double u1[3] = {L.aux[(AUX_U + 0) * N + in], L.aux[(AUX_U + 1) * N + in], L.aux[(AUX_U + 2) * N + in]};
        const double T1 = L.aux[AUX_T * N + in];
        const double R0 = mc.R_univ * mix_inv_m<M>(mc, Y0);
        const double P0 = rho0 * R0 * T0;
        const double P1 = rho1 * mc.R_univ * mix_inv_m<M>(mc, Y1) * T1;
        double Cv = 0.0;
#pragma unroll
        for (int a = 0; a < M; ++a) Cv += Y0[a] * species_cv(mc, a, T0);
        const double gam = (Cv + R0) / Cv;
        const double c = sqrt(gam * P0 / rho0);
        const double un = u0[0];
        const double Ma = un / c;
        const double L1 = L.sigma * (1.0 - Ma * Ma) * c / (double)L.nx * (P0 - L.P_inf);
        const double L2 = un * (c * c * (rho0 - rho1) - (P0 - P1));
        const double L3 = un * (u0[1] - u1[1]);
        const double L4 = un * (u0[2] - u1[2]);
        const double L5 = (un + c) * ((P0 - P1) + rho0 * c * (u0[0] - u1[0]));
        const double rho_o = rho0 - (L2 + 0.5 * (L5 + L1)) / (c * c);
        const double P_o = P0 - 0.5 * (L5 + L1);
        A.rho = rho_o;
        A.u[0] = un - (L5 - L1) / (2.0 * rho0 * c);
        A.u[1] = u0[1] - L3;
        A.u[2] = u0[2] - L4;
#pragma unroll
        for (int a = 0; a < M; ++a) {
            A.Y[a] = Y0[a] - un * (Y0[a] - Y1[a]);
            A.us[a][0] = A.u[0]; A.us[a][1] = A.u[1]; A.us[a][2] = A.u[2];
        }
        T_A = P_o / (rho_o * mc.R_univ * mix_inv_m<M>(mc, A.Y));
        os[0 * No + ko] = A.rho;
        os[1 * No + ko] = A.u[0]; os[2 * No + ko] = A.u[1]; os[3 * No + ko] = A.u[2];
        os[4 * No + ko] = T_A;
#pragma unroll
        for (int a = 0; a < M; ++a) os[(5 + a) * No + ko] = A.Y[a];
    }
    eq_prepare<M>(mc, A, T_A);

    // local state with the incoming links set to the imposed equilibrium
    // (eqs. locRho..locT, inletlocRho..inletlocT, outletlocRho..outletlocT)
    EqState<M> Lc;
    double rl = 0.0, jl[3] = {0.0, 0.0, 0.0}, El = 0.0, ra[M], ja[M][3];
#pragma unroll
    for (int a = 0; a < M; ++a) ra[a] = ja[a][0] = ja[a][1] = ja[a][2] = 0.0;
    for (int l = 0; l < nL; ++l) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int i = 0; i < Q; ++i) {
            const double v = incoming(i) ? eq_value<M>(mc, A, T_A, l, s, i) : streamed(l, i);
            s0 += v; s1 += v * cx_of(i); s2 += v * cy_of(i); s3 += v * cz_of(i);
        }
        if (l == M) {
            El = s0;
        } else if (l == M - 1) {
            rl = s0; jl[0] = s1; jl[1] = s2; jl[2] = s3;
        } else {
            const int a = l + (l >= s ? 1 : 0);
#pragma unroll
            for (int c = 0; c < M; ++c)
                if (c == a) { ra[c] = s0; ja[c][0] = s1; ja[c][1] = s2; ja[c][2] = s3; }
        }
    }
    {
        double rs = rl, j0 = jl[0], j1 = jl[1], j2 = jl[2];
#pragma unroll
        for (int a = 0; a < M; ++a)
            if (a != s) { rs -= ra[a]; j0 -= ja[a][0]; j1 -= ja[a][1]; j2 -= ja[a][2]; }
#pragma unroll
        for (int a = 0; a < M; ++a)
            if (a == s) { ra[a] = rs; ja[a][0] = j0; ja[a][1] = j1; ja[a][2] = j2; }
    }
    Lc.rho = rl;
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) Lc.u[dd] = jl[dd] / rl;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        Lc.Y[a] = ra[a] / rl;
        const bool small = ra[a] <= 1e-14 * rl;
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
            // TMS local species equilibria use the species velocities (eq. locua);
            // inlet and outlet local equilibria use the mixture velocity.
            Lc.us[a][dd] = (type == RLBM_FACE_WALL && !small) ? ja[a][dd] / ra[a] : Lc.u[dd];
        }
    }
    const double Ul = El / rl - 0.5 * (Lc.u[0] * Lc.u[0] + Lc.u[1] * Lc.u[1] + Lc.u[2] * Lc.u[2]);
    const double T_l = solve_T<M>(mc, Lc.Y, Ul, T_A, &fail);
    eq_prepare<M>(mc, Lc, T_l);

    // inlet target: local density and composition at the imposed u, T (eqs. in_tgt_*)
    EqState<M> Tg;
    const bool inlet = type == RLBM_FACE_INLET;
    if (inlet) {
        Tg.rho = Lc.rho;
        Tg.u[0] = L.u_in; Tg.u[1] = 0.0; Tg.u[2] = 0.0;
#pragma unroll
        for (int a = 0; a < M; ++a) {
            Tg.Y[a] = Lc.Y[a];
            Tg.us[a][0] = L.u_in; Tg.us[a][1] = 0.0; Tg.us[a][2] = 0.0;
        }
        eq_prepare<M>(mc, Tg, L.T_in);
    }

    // final populations (eqs. ftms/gtms/fatms, f_inlet/g_inlet/fa_inlet,
    // f_outlet/g_outlet/fa_outlet)
    for (int l = 0; l < nL; ++l) {
        for (int i = 0; i < Q; ++i) {
            const double a_eq = eq_value<M>(mc, A, T_A, l, s, i);
            const double l_eq = eq_value<M>(mc, Lc, T_l, l, s, i);
            double out;
            if (inlet) {
                const double t_eq = eq_value<M>(mc, Tg, L.T_in, l, s, i);
                out = incoming(i) ? t_eq + a_eq - l_eq : t_eq + streamed(l, i) - l_eq;
            } else {
                out = incoming(i) ? 2.0 * a_eq - l_eq : a_eq + streamed(l, i) - l_eq;
            }
            L.bcbuf[(size_t)(l * Q + i) * L.n_if + k] = out;
        }
    }
    if (fail) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// initial state, read-out, populations I/O, invariants
// ---------------------------------------------------------------------------
template <int M, typename S>
__global__ __launch_bounds__(256) void k_init(const LatDev* __restrict__ lat, const double* __restrict__ rho_in,
                                              const double* __restrict__ u_in, const double* __restrict__ T_in,
                                              const double* __restrict__ Y_in) {
    const LatDev& L = *lat;
    const long long node = (long long)blockIdx.x * 256 + threadIdx.x;
    if (node >= L.N) return;
    const MechDev& mc = *L.mech;
    const size_t N = (size_t)L.N;
    void* dst = L.pop[L.parity0];
    EqState<M> e;
    e.rho = rho_in[node];
    const double T = T_in[node];
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) e.u[dd] = u_in[dd * N + node];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        e.Y[a] = Y_in[a * N + node];
        e.us[a][0] = e.u[0]; e.us[a][1] = e.u[1]; e.us[a][2] = e.u[2];
    }
    eq_prepare<M>(mc, e, T);
    for (int l = 0; l <= M; ++l)
        for (int i = 0; i < Q; ++i) {
            const int li = l * Q + i;
            Codec<S>::st(dst, (size_t)li * N + node, eq_value<M>(mc, e, T, l, L.slaved, i), L.ref, li);
        }
    double* aux = L.aux;
    aux[AUX_RHO * N + node] = e.rho;
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) {
        aux[(AUX_U + dd) * N + node] = e.u[dd];
        aux[(AUX_PHI + dd) * N + node] = e.rho * e.u[dd] * (1.0 - 3.0 * e.th) - e.rho * e.u[dd] * e.u[dd] * e.u[dd];
    }
    aux[AUX_T * N + node] = T;
#pragma unroll
    for (int a = 0; a < M; ++a) aux[(AUX_Y + a) * N + node] = e.Y[a];
    if (L.n_if) {
        const int k = L.if_index[node];
        if (k >= 0 && L.if_out[k] >= 0) {
            const int ko = L.if_out[k];
            const size_t No = (size_t)L.n_out;
            L.out_state[0 * No + ko] = e.rho;
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) L.out_state[(1 + dd) * No + ko] = e.u[dd];
            L.out_state[4 * No + ko] = T;
#pragma unroll
            for (int a = 0; a < M; ++a) L.out_state[(5 + a) * No + ko] = e.Y[a];
        }
    }
}

// Reference populations for FP32 deviation storage: the zero-velocity
// equilibria of the domain-mean state.
template <int M>
__global__ void k_refs(const LatDev* __restrict__ lat, double* __restrict__ ref, double rho, double T,
                       const double* __restrict__ Y) {
    const LatDev& L = *lat;
    const int li = blockIdx.x * blockDim.x + threadIdx.x;
    if (li >= (M + 1) * Q) return;
    const MechDev& mc = *L.mech;
    EqState<M> e;
    e.rho = rho;
    e.u[0] = e.u[1] = e.u[2] = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        e.Y[a] = Y[a];
        e.us[a][0] = e.us[a][1] = e.us[a][2] = 0.0;
    }
    eq_prepare<M>(mc, e, T);
    ref[li] = eq_value<M>(mc, e, T, li / Q, L.slaved, li % Q);
}

template <int M, typename S>
__global__ __launch_bounds__(256) void k_fields(const LatDev* __restrict__ lat, long long t, double* rho_o,
                                                double* u_o, double* T_o, double* Y_o, double* P_o,
                                                int* __restrict__ flag) {
    const LatDev& L = *lat;
    const long long node = (long long)blockIdx.x * 256 + threadIdx.x;
    if (node >= L.N) return;
    const MechDev& mc = *L.mech;
    const size_t N = (size_t)L.N;
    const void* src = L.pop[(L.parity0 + t) & 1];
    const int s = L.slaved;
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, rE = 0.0, ra[M];
    for (int i = 0; i < Q; ++i) {
        const double f = Codec<S>::ld(src, (size_t)((M - 1) * Q + i) * N + node, L.ref, (M - 1) * Q + i);
        rho += f; j[0] += f * cx_of(i); j[1] += f * cy_of(i); j[2] += f * cz_of(i);
        rE += Codec<S>::ld(src, (size_t)(M * Q + i) * N + node, L.ref, M * Q + i);
    }
    double rs = rho;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        ra[a] = 0.0;
        if (a == s) continue;
        const int l = lat_of<M>(a, s);
        for (int i = 0; i < Q; ++i) ra[a] += Codec<S>::ld(src, (size_t)(l * Q + i) * N + node, L.ref, l * Q + i);
        rs -= ra[a];
    }
#pragma unroll
    for (int a = 0; a < M; ++a)
        if (a == s) ra[a] = rs;
    double Y[M];
#pragma unroll
    for (int a = 0; a < M; ++a) Y[a] = ra[a] / rho;
    const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    const double U = rE / rho - 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    int fail = 0;
    const double T = solve_T<M>(mc, Y, U, L.aux[AUX_T * N + node], &fail);
    if (fail) atomicOr(flag, 1);
    if (rho_o) rho_o[node] = rho;
    if (u_o)
        for (int dd = 0; dd < 3; ++dd) u_o[dd * N + node] = u[dd];
    if (T_o) T_o[node] = T;
    if (Y_o)
#pragma unroll
        for (int a = 0; a < M; ++a) Y_o[a * N + node] = Y[a];
    if (P_o) P_o[node] = rho * mc.R_univ * mix_inv_m<M>(mc, Y) * T;
}

template <typename S>
__global__ __launch_bounds__(256) void k_pops(const LatDev* __restrict__ lat, long long t, int nl, double* buf,
                                              int write) {
    const LatDev& L = *lat;
    const size_t total = (size_t)nl * Q * L.N;
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const int li = (int)(idx / L.N);
    void* p = L.pop[(L.parity0 + t) & 1];
    if (write) Codec<S>::st(p, idx, buf[idx], L.ref, li);
    else buf[idx] = Codec<S>::ld(p, idx, L.ref, li);
}

// Per-block partial sums of the invariants; nv = 6 + E values per block.
template <int M, typename S>
__global__ __launch_bounds__(256) void k_invariants(const LatDev* __restrict__ lat, long long t,
                                                    double* __restrict__ partial, int nv) {
    const LatDev& L = *lat;
    const MechDev& mc = *L.mech;
    const long long node = (long long)blockIdx.x * 256 + threadIdx.x;
    const size_t N = (size_t)L.N;
    const int s = L.slaved;
    double v[6 + MAXE];
    for (int q = 0; q < 6 + MAXE; ++q) v[q] = 0.0;
    if (node < L.N) {
        const void* src = L.pop[(L.parity0 + t) & 1];
        double bad = 0.0;
        double rho = 0.0;
        for (int i = 0; i < Q; ++i) {
            const double f = Codec<S>::ld(src, (size_t)((M - 1) * Q + i) * N + node, L.ref, (M - 1) * Q + i);
            const double g = Codec<S>::ld(src, (size_t)(M * Q + i) * N + node, L.ref, M * Q + i);
            if (!isfinite(f) || !isfinite(g)) bad = 1.0;
            rho += f;
            v[1] += f * cx_of(i); v[2] += f * cy_of(i); v[3] += f * cz_of(i);
            v[4] += g;
        }
        v[0] = rho;
        double ra[M];
        double rs = rho;
#pragma unroll
        for (int a = 0; a < M; ++a) {
            ra[a] = 0.0;
            if (a == s) continue;
            const int l = lat_of<M>(a, s);
            for (int i = 0; i < Q; ++i) {
                const double f = Codec<S>::ld(src, (size_t)(l * Q + i) * N + node, L.ref, l * Q + i);
                if (!isfinite(f)) bad = 1.0;
                ra[a] += f;
            }
            rs -= ra[a];
        }
#pragma unroll
        for (int a = 0; a < M; ++a)
            if (a == s) ra[a] = rs;
        for (int e = 0; e < mc.E; ++e) {
            double sum = 0.0;
#pragma unroll
            for (int a = 0; a < M; ++a) sum += ra[a] * mc.inv_m[a] * mc.comp[a][e];
            v[5 + e] = sum;
        }
        v[5 + mc.E] = bad;
    }
    __shared__ double red[256];
    for (int q = 0; q < nv; ++q) {
        red[threadIdx.x] = v[q];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                if (q == nv - 1) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
                else red[threadIdx.x] += red[threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * nv + q] = red[0];
        __syncthreads();
    }
}

__global__ void k_reduce_partials(const double* __restrict__ partial, int nblocks, int nv, double* __restrict__ out) {
    const int q = threadIdx.x;
    if (q >= nv) return;
    double acc = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        const double x = partial[(size_t)b * nv + q];
        acc = (q == nv - 1) ? fmax(acc, x) : acc + x;
    }
    out[q] = acc;
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
#define RLBM_DISPATCH(M_, ...)                            \
    switch (M_) {                                         \
        case 2: { constexpr int MM = 2; __VA_ARGS__; break; } \
        case 3: { constexpr int MM = 3; __VA_ARGS__; break; } \
        case 4: { constexpr int MM = 4; __VA_ARGS__; break; } \
        case 9: { constexpr int MM = 9; __VA_ARGS__; break; } \
        default: return hipErrorInvalidValue;             \
    }

template <typename S>
static hipError_t launch_step_phase(int phase, int M, const StepLaunch& a) {
    if (a.blocks <= 0) return hipSuccess;
    if (phase == 0) {
        RLBM_DISPATCH(M, hipLaunchKernelGGL((k_boundary<MM, S>), dim3(a.blocks), dim3(64), 0, a.stream, a.lats,
                                                a.blk, a.n_lat, a.t, a.flag))
    } else if (phase == 1) {
        RLBM_DISPATCH(M, hipLaunchKernelGGL((k_moments<MM, S>), dim3(a.blocks), dim3(256), 0, a.stream, a.lats,
                                                a.blk, a.n_lat, a.t, a.flag))
    } else {
        RLBM_DISPATCH(M, hipLaunchKernelGGL((k_collide<MM, S>), dim3(a.blocks), dim3(256), 0, a.stream, a.lats,
                                                a.blk, a.n_lat, a.t, a.flag))
    }
    return hipGetLastError();
}

hipError_t launch_phase(int phase, int M, int storage, const StepLaunch& a) {
    return storage == RLBM_STORAGE_F32_DEV ? launch_step_phase<float>(phase, M, a)
                                           : launch_step_phase<double>(phase, M, a);
}

template <typename S>
static hipError_t launch_init_t(int M, const LatDev* lat, long long N, const double* rho, const double* u,
                                const double* T, const double* Y, hipStream_t st) {
    const int blocks = (int)((N + 255) / 256);
    RLBM_DISPATCH(M, hipLaunchKernelGGL((k_init<MM, S>), dim3(blocks), dim3(256), 0, st, lat, rho, u, T, Y))
    return hipGetLastError();
}

hipError_t launch_init(int M, int storage, const LatDev* lat, long long N, const double* rho, const double* u,
                       const double* T, const double* Y, hipStream_t st) {
    return storage == RLBM_STORAGE_F32_DEV ? launch_init_t<float>(M, lat, N, rho, u, T, Y, st)
                                           : launch_init_t<double>(M, lat, N, rho, u, T, Y, st);
}

hipError_t launch_refs(int M, const LatDev* lat, double* ref, double rho, double T, const double* Y,
                       hipStream_t st) {
    const int n = (M + 1) * Q;
    RLBM_DISPATCH(M, hipLaunchKernelGGL((k_refs<MM>), dim3((n + 63) / 64), dim3(64), 0, st, lat, ref, rho,
                                                 T, Y))
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_fields_t(int M, const LatDev* lat, long long N, long long t, double* rho, double* u,
                                  double* T, double* Y, double* P, int* flag, hipStream_t st) {
    const int blocks = (int)((N + 255) / 256);
    RLBM_DISPATCH(M, hipLaunchKernelGGL((k_fields<MM, S>), dim3(blocks), dim3(256), 0, st, lat, t, rho, u, T,
                                            Y, P, flag))
    return hipGetLastError();
}

hipError_t launch_fields(int M, int storage, const LatDev* lat, long long N, long long t, double* rho, double* u,
                         double* T, double* Y, double* P, int* flag, hipStream_t st) {
    return storage == RLBM_STORAGE_F32_DEV ? launch_fields_t<float>(M, lat, N, t, rho, u, T, Y, P, flag, st)
                                           : launch_fields_t<double>(M, lat, N, t, rho, u, T, Y, P, flag, st);
}

hipError_t launch_pops(int storage, const LatDev* lat, long long N, int nl, long long t, double* buf, int write,
                       hipStream_t st) {
    const size_t total = (size_t)nl * Q * (size_t)N;
    const int blocks = (int)((total + 255) / 256);
    if (storage == RLBM_STORAGE_F32_DEV)
        hipLaunchKernelGGL((k_pops<float>), dim3(blocks), dim3(256), 0, st, lat, t, nl, buf, write);
    else
        hipLaunchKernelGGL((k_pops<double>), dim3(blocks), dim3(256), 0, st, lat, t, nl, buf, write);
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_inv_t(int M, const LatDev* lat, long long N, long long t, double* partial, int nv,
                               double* out, hipStream_t st) {
    const int blocks = (int)((N + 255) / 256);
    RLBM_DISPATCH(M, hipLaunchKernelGGL((k_invariants<MM, S>), dim3(blocks), dim3(256), 0, st, lat, t, partial,
                                            nv))
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(64), 0, st, partial, blocks, nv, out);
    return hipGetLastError();
}

hipError_t launch_invariants(int M, int storage, const LatDev* lat, long long N, long long t, double* partial,
                             int nv, double* out, hipStream_t st) {
    return storage == RLBM_STORAGE_F32_DEV ? launch_inv_t<float>(M, lat, N, t, partial, nv, out, st)
                                           : launch_inv_t<double>(M, lat, N, t, partial, nv, out, st);
}

bool species_supported(int M) { return M == 2 || M == 3 || M == 4 || M == 9; }

}  // namespace rlbm
