// HIP kernels of the reactive-mixture lattice Boltzmann step for gfx950.
//
// One time step is four launches over a (possibly batched) work list:
//   k_boundary   interface nodes: advection + wall / inlet / outlet
//                reconstruction (section 4) into a side buffer;
//   k_local      every node: advection, moments, temperature (eq.
//                temperature), relaxation rates, Stefan-Maxwell diffusion
//                velocities (eq. transform1) and the reaction increment by l
//                forward-Euler sub-steps (eq. R3); publishes rho, u, T, Y,
//                Phi_a and the enthalpy moments for the neighbours and writes
//                the per-node record read by k_update;
//   k_gradients  the same-time gradients of Phi_a and sum_b H_b Y_b
//                (k_chem_implicit instead for lattices with the linearly
//                implicit reaction update: its sub-steps, then the gradients);
//   k_update     every node: advection again and the collisions of all stored
//                lattices, written to the other population buffer.
// Populations are structure-of-arrays [L][27][N] (x fastest), pulled from the
// source buffer, so every load and store of a wavefront is coalesced.  The
// storage type S is double (FP64) or float (FP32 deviation from a reference
// population per lattice and velocity, decoded to FP64 on load).

#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

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
    static __device__ __forceinline__ double ld(const void* p, size_t idx, double) {
        return static_cast<const double*>(p)[idx];
    }
    static __device__ __forceinline__ void st(void* p, size_t idx, double v, double) {
        static_cast<double*>(p)[idx] = v;
    }
};

template <>
struct Codec<float> {
    static __device__ __forceinline__ double ld(const void* p, size_t idx, double ref) {
        return (double)static_cast<const float*>(p)[idx] + ref;
    }
    static __device__ __forceinline__ void st(void* p, size_t idx, double v, double ref) {
        static_cast<float*>(p)[idx] = __double2float_rn(v - ref);
    }
};

// FP32 deviation storage: population (l, i) is stored as its deviation from
// s_l(y) G_li, where G_li is the zero-velocity equilibrium shape of lattice l
// at the domain-mean initial state normalised to unit zeroth moment, and
// s_l(y) the zeroth moment of lattice l (rho_a, rho or rho E) at the node y
// that reads the population, as it was when the population was written.
// Both factors hold FP32 values, so their product is exact in FP64: every
// writer and reader forms the same reference however the compiler fuses it.
__device__ __forceinline__ double ref_of(float s, double G) { return (double)s * G; }

// The energy lattice's reference: at zero velocity its equilibrium is
// rho U W_i(theta) + rho K_i(theta) (eq. geq_i with u = 0: K carries the
// theta^2 terms and has zero sum), so its reference is s_g W_i + s_f K_i with
// s_g = rho E and s_f = rho of the reading node (both products exact).
__device__ __forceinline__ double ref_g(float sg, float sf, double W, double K) {
    return (double)sg * W + (double)sf * K;
}

// Stored lattices: the species lattices (M - 1 of them when one species is
// slaved, eq. strongest; all M in the weakly coupled storage, W = 1), then
// the momentum lattice f at LF and the energy lattice g at LG.
template <int M, int W>
struct Lat {
    static constexpr int NSP = M - 1 + W;
    static constexpr int LF = NSP;
    static constexpr int LG = NSP + 1;
    static constexpr int NL = NSP + 2;
};

// Layout of the reference table for NL stored lattices: shapes G[NL][Q] (the
// energy lattice's row is W), the zeroth moments sum_i G_li [NL],
// sum_i G_fi c_ix^2, the energy lattice's K[Q] and sum_i K_i.
template <int NL> constexpr int REF_M0 = NL * Q;
template <int NL> constexpr int REF_M2 = NL * Q + NL;
template <int NL> constexpr int REF_K = NL * Q + NL + 1;
template <int NL> constexpr int REF_K0 = NL * Q + NL + 1 + Q;

// Scales s_l of node n in buffer q: rss floats per node, lattices in order
// (stored species, rho, rho E).
__device__ __forceinline__ const RLBM_GLOBAL float* scale_at(const LatDev& L, int q, long long n) {
    return as_global(L.rscale[q]) + (size_t)n * L.rss;
}

// Block index -> work tile, XCD-aware.  Workgroups are dispatched to the
// eight XCDs round-robin (block b on XCD b mod 8), and each XCD has its own
// L2.  Remapping gives every XCD one contiguous range of tiles, so tiles that
// share cache lines (x-neighbours of the pull advection, the rows of a
// gradient stencil) are processed by the same L2 at about the same time.
// A bijection on [0, gridDim.x) for any grid size.
__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb >> 3, r = nb & 7, j = b & 7, i = b >> 3;
    return j * q + (j < r ? j : r) + i;
}

// Byte-offset addressing: a uniform base plus a 32-bit per-lane offset keeps
// every population access in the scalar-base form (no 64-bit address math).
template <typename S>
__device__ __forceinline__ S ld_at(const RLBM_GLOBAL S* base, int idx) {
    return *(const RLBM_GLOBAL S*)((const RLBM_GLOBAL char*)base + (unsigned)(idx * (int)sizeof(S)));
}
template <typename S>
__device__ __forceinline__ void st_at(RLBM_GLOBAL S* base, int idx, S v) {
    *(RLBM_GLOBAL S*)((RLBM_GLOBAL char*)base + (unsigned)(idx * (int)sizeof(S))) = v;
}

// A correction row of the per-node record: FP32 (rounded to nearest even)
// when F32, else FP64.
template <bool F32>
__device__ __forceinline__ void st_corr(RLBM_GLOBAL double* prm, int row, size_t N, int node, double v) {
    if constexpr (F32) st_at(reinterpret_cast<RLBM_GLOBAL float*>(prm + (size_t)row * N), node, (float)v);
    else st_at(prm + (size_t)row * N, node, v);
}
template <bool F32>
__device__ __forceinline__ double ld_corr(const RLBM_GLOBAL double* prm, int row, size_t N, int node) {
    if constexpr (F32) return (double)ld_at(reinterpret_cast<const RLBM_GLOBAL float*>(prm + (size_t)row * N), node);
    else return ld_at(prm + (size_t)row * N, node);
}

// ---------------------------------------------------------------------------
// work-list helpers
// ---------------------------------------------------------------------------
// Step counter of a launch: a device counter (batched steps replayed from a
// captured graph advance it with k_advance_time) plus the launch's offset.
__device__ __forceinline__ long long step_time(const long long* tp, long long toff) {
    return (tp ? *tp : 0) + toff;
}
__device__ __forceinline__ int find_lattice(const int* blk, int n_lat, int b) {
    int lo = 0, hi = n_lat - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blk[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// pull-advection addressing for the hot kernels
// ---------------------------------------------------------------------------
// Node offsets of the source x - c for c = -1, 0, +1 along each axis, with
// periodic wrap.  Along non-periodic axes only interface nodes would leave
// the box, and those read the boundary buffer instead, so the wrapped value
// is only ever an in-bounds placeholder.
struct PullOff {
    int x[3], y[3], z[3];   // index c + 1
};

__device__ __forceinline__ void pull_offsets(const LatDev& L, int x, int y, int z, PullOff& o) {
    const int nx = L.nx, ny = L.ny, nz = L.nz, sxy = nx * ny;
    o.x[0] = x == nx - 1 ? -(nx - 1) : 1;   // c = -1: source x + 1
    o.x[1] = 0;
    o.x[2] = x == 0 ? nx - 1 : -1;          // c = +1: source x - 1
    o.y[0] = y == ny - 1 ? -(ny - 1) * nx : nx;
    o.y[1] = 0;
    o.y[2] = y == 0 ? (ny - 1) * nx : -nx;
    o.z[0] = z == nz - 1 ? -(nz - 1) * sxy : sxy;
    o.z[1] = 0;
    o.z[2] = z == 0 ? (nz - 1) * sxy : -sxy;
}

__device__ __forceinline__ int sel3(int c, int m, int z, int p) { return c < 0 ? m : (c == 0 ? z : p); }
__device__ __forceinline__ double sel3d(int c, double m, double z, double p) { return c < 0 ? m : (c == 0 ? z : p); }

// Stored lattice of species a; a slaved index of M (the weakly coupled
// storage) stores every species at its own index.
__device__ __forceinline__ int lat_of(int a, int slaved) { return a - (a > slaved ? 1 : 0); }

// Per-thread LDS columns of k_local (stride LOC_T doubles between rows): the
// species densities rho_a [M] and velocity differences u_a - u [3 M], handed
// from the streaming part to the Stefan-Maxwell step without a trip to memory.
struct LocalLds {
    double* ra;   // &rho_a[0][tid]
    double* dv;   // &(u_a - u)[0][tid], row 3 a + d
};
constexpr int LOC_T = NODE_TILE;   // k_local threads per block

// ---------------------------------------------------------------------------
// Stefan-Maxwell diffusion velocities (section 2.3, eq. transform1)
// ---------------------------------------------------------------------------
// The system (dt = 1)
//   (1 + 1/(2 tau_a)) V_a - 1/2 sum_{b != a} Y_b V_b / tau_ab = u_a - u
// with 1/tau_ab = common K_ab and 1/tau_a = sum_{b != a} Y_b / tau_ab, for
// the three components at once.  Its matrix is strictly row diagonally
// dominant with margin 1 (the off-diagonal row sums are -1/(2 tau_a)), so
// Doolittle LU without pivoting is stable.  Rows are generated on the fly
// from cY_b = -common Y_b / 2 (A_ab = K_ab cY_b) and the forward substitution
// runs with the factorisation.  The velocity differences u_a - u and the
// densities rho_a come from k_local's LDS columns, the node's scalars from
// its registers; writes V_a and the energy flux base Qb plus
// omega1 sum_a H_a rho_a V_a to the per-node record.
template <int M, int W, bool F32>
__device__ __forceinline__ void stefan_maxwell(const LatDev& L, int node, const LocalLds& ls, double T, double rho,
                                               double common, double omega1, const double* Y, const double* Qb,
                                               double rho_over_rhoY) {
    MechC mc0 = *as_const(L.mech);
    const size_t N = (size_t)L.N;
    RLBM_GLOBAL double* prm = as_global(L.prm);
    double cY[M], V[M][3];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        cY[a] = -0.5 * common * Y[a];
#pragma unroll
        for (int d = 0; d < 3; ++d) V[a][d] = ls.dv[(3 * a + d) * LOC_T];
    }
    double Uu[M][M];
    double inv_diag[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        reload_barrier();
        MechC mc = in_loop(mc0);   // this row's K_ab as scalar loads, not hoisted
        double st = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c)
            if (c != i) st += mc.Kab[i][c] * cY[c];
        const double inv_tau = -2.0 * st;
        double lrow[M];
#pragma unroll
        for (int j = 0; j < i; ++j) {
            double a = mc.Kab[i][j] * cY[j];
#pragma unroll
            for (int kk = 0; kk < j; ++kk) a -= lrow[kk] * Uu[kk][j];
            lrow[j] = a * inv_diag[j];
        }
#pragma unroll
        for (int j = i; j < M; ++j) {
            double a = (i == j) ? 1.0 + 0.5 * inv_tau : mc.Kab[i][j] * cY[j];
#pragma unroll
            for (int kk = 0; kk < i; ++kk) a -= lrow[kk] * Uu[kk][j];
            Uu[i][j] = a;
        }
        inv_diag[i] = 1.0 / Uu[i][i];
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
            double yv = V[i][dd];
#pragma unroll
            for (int kk = 0; kk < i; ++kk) yv -= lrow[kk] * V[kk][dd];
            V[i][dd] = yv;
        }
    }
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
            double sm = V[i][dd];
#pragma unroll
            for (int j = i + 1; j < M; ++j) sm -= Uu[i][j] * V[j][dd];
            V[i][dd] = sm * inv_diag[i];
            st_corr<F32>(prm, PRM_SP + 6 * i + 1 + dd, N, node, V[i][dd]);
        }
    }
    // energy flux: Qb + omega1 sum_a H_a rho_a V_a
    MechC mc = mc0;
    double diff[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const double hy = (species_U(mc, a, T) + mc.Ra[a] * T) * ls.ra[a * LOC_T];
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) diff[dd] += hy * V[a][dd];
    }
    (void)rho;
    // rho Y_a = rho_a, except in the weakly coupled storage where Y_a is
    // normalised by sum_b rho_b
    if constexpr (W) {
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) diff[dd] *= rho_over_rhoY;
    } else {
        (void)rho_over_rhoY;
    }
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) st_corr<F32>(prm, PRM_QB + dd, N, node, Qb[dd] + omega1 * diff[dd]);
}

// Relaxation rates of a node (sections 2.3 and 3.4) from its temperature,
// pressure and mixture gas constant Rmix = R_univ sum_a Y_a / m_a: the
// factor `common` of 1/tau_ab = common K_ab (eqs. betaa, taua), and omega,
// omega_1 of the momentum and energy lattices.
__device__ __forceinline__ void relax_rates(MechC mc, double T, double P, double Rmix, double& common,
                                            double& omega, double& omega1) {
    const double lnr = log(T * mc.inv_T_ref);
    common = mc.R_univ * mc.R_univ * T / Rmix * P * mc.inv_P_ref * exp(-mc.D_exp * lnr);
    const double mu = mc.mu_ref * exp(mc.mu_exp * lnr);
    omega = 1.0 / (mu / P + 0.5);
    omega1 = 1.0 / (mu * mc.inv_Pr / P + 0.5);
}

// ---------------------------------------------------------------------------
// k_local: moments and everything else a node needs from its own populations
// ---------------------------------------------------------------------------
// Moments of the node's post-advection, post-boundary populations (eqs.
// density1, momentum1, fdensity, f1momMomentum, g0momTotalEnergy), the
// slaved species by difference (eq. strongest), then the temperature (eq.
// temperature), the relaxation rates and the local part of the energy flux.
// The momentum and energy lattices are summed first so the mixture velocity
// is known when each species lattice is summed: its velocity difference
// u_a - u is written out at once and only rho_a stays in registers.  In FP32
// deviation storage the sums run over the stored deviations and the
// reference's own moments are added in closed form (zeroth s_l sum_i G_li,
// second s_f sum_i G_fi c c, first zero by symmetry); the stored lattices'
// zeroth moments (rho_a, rho, rho E) become the scales of the references of
// the populations written this step.  The Stefan-Maxwell solve comes last,
// once the streaming part no longer holds registers.
template <int M>
struct LocalMoments {
    double rho, rhoE, j[3], q[3], Pd[3], Po[3];   // Pd: xx yy zz, Po: xy xz yz
    double u[3];
    double rho_a[M];
};


// Buffer-resource load: a wave-uniform base (scalar registers) plus a 32-bit
// per-lane byte offset (node counts are limited so that idx * sizeof(S) fits).
// An offset at or beyond nbytes reads zero instead of leaving the buffer.
template <typename S>
__device__ __forceinline__ S ldb(const RLBM_GLOBAL S* base, unsigned nbytes, int idx) {
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc((void*)(unsigned long long)base, 0, (int)nbytes, 0x00020000);
    if constexpr (sizeof(S) == 4)
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (unsigned)idx * 4u, 0, 0));
    else
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (unsigned)idx * 8u, 0, 0));
}
__device__ __forceinline__ unsigned plane_bytes(long long N, int s) {
    const unsigned long long b = (unsigned long long)N * (unsigned)s;
    return b > 0xffffffffull ? 0xffffffffu : (unsigned)b;
}

// Population loads through one resource per window of nine planes (the nine
// velocities of one c_z layer of one lattice): the plane within the window is
// a scalar offset, the node a per-lane offset.  Few resources stay live, so
// the scalar registers do not run out.  The host keeps 9 N sizeof(S) below
// 2^32.
template <typename S>
__device__ __forceinline__ S ld_win(const RLBM_GLOBAL S* win, unsigned plane, int iw, int idx) {
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc((void*)(unsigned long long)win, 0, (int)(9u * plane), 0x00020000);
    if constexpr (sizeof(S) == 4)
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (unsigned)idx * 4u, iw * plane, 0));
    else
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (unsigned)idx * 8u, iw * plane, 0));
}

// The moment sums of k_local.  IF = false: no lane of the wave is an
// interface node and every population is pulled from the source buffer;
// IF = true: interface lanes read their reconstructed populations from the
// planes' interface slots instead.
template <int M, typename S, int W, bool IF>
__device__ __forceinline__ void local_moments(const LatDev& L, int par, int k, int node, const PullOff& o,
                                              const LocalLds& ls, LocalMoments<M>& m) {
    constexpr int NSP = Lat<M, W>::NSP, LF = Lat<M, W>::LF, LG = Lat<M, W>::LG, NL = Lat<M, W>::NL;
    const size_t N = (size_t)L.N;
    const int s = W ? M : L.slaved;
    const RLBM_GLOBAL S* src = as_global(static_cast<const S*>(L.pop[par]));
    RLBM_GLOBAL double* prm = as_global(L.prm);
    auto off_of = [&](int i) { return node + o.x[cx_of(i) + 1] + o.y[cy_of(i) + 1] + o.z[cz_of(i) + 1]; };
    const size_t P = (size_t)L.P;
    const unsigned nb = plane_bytes(L.P, sizeof(S));
    // an interface lane reads its post-boundary population from the plane's
    // interface slot N + k instead of its pull source: the same load with
    // another index
    auto ld = [&](int l, int i) -> S {
        const int idx = IF ? (k >= 0 ? (int)N + k : off_of(i)) : off_of(i);
        return ld_win(src + (size_t)(l * Q + 9 * (i / 9)) * P, nb, i % 9, idx);
    };
    const RLBM_GLOBAL float* sc = nullptr;
    RLBM_GLOBAL float* so = nullptr;
    if constexpr (sizeof(S) == 4) {
        sc = scale_at(L, par, node);
        so = as_global(L.rscale[par ^ 1]) + (size_t)node * L.rss;
    }

    // the first species lattice's loads go out with the momentum and energy
    // lattices' (FP32 storage), so its sum does not wait for a round trip of
    // its own
    constexpr bool PF = sizeof(S) == 4;
    S cur[Q];
    if constexpr (PF) {
#pragma unroll
        for (int i = 0; i < Q; ++i) cur[i] = ld(0, i);
    }
    // momentum and energy lattices
    double rho = 0.0, rhoE = 0.0, j[3] = {0.0, 0.0, 0.0}, q[3] = {0.0, 0.0, 0.0};
    double Pd[3] = {0.0, 0.0, 0.0}, Po[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
        const double f = (double)ld(LF, i);
        const double g = (double)ld(LG, i);
        rho += f;
        rhoE += g;
        if (cx) { j[0] += cx > 0 ? f : -f; Pd[0] += f; q[0] += cx > 0 ? g : -g; }
        if (cy) { j[1] += cy > 0 ? f : -f; Pd[1] += f; q[1] += cy > 0 ? g : -g; }
        if (cz) { j[2] += cz > 0 ? f : -f; Pd[2] += f; q[2] += cz > 0 ? g : -g; }
        if (cx * cy) Po[0] += cx * cy > 0 ? f : -f;
        if (cx * cz) Po[1] += cx * cz > 0 ? f : -f;
        if (cy * cz) Po[2] += cy * cz > 0 ? f : -f;
    }
    if constexpr (sizeof(S) == 4) {
        const RLBM_CONST double* G = as_const(L.ref);
        const double sf = (double)sc[LF];
        rho += sf * G[REF_M0<NL> + LF];
        rhoE += (double)sc[LG] * G[REF_M0<NL> + LG] + sf * G[REF_K0<NL>];
        const double p2 = sf * G[REF_M2<NL>];
        Pd[0] += p2; Pd[1] += p2; Pd[2] += p2;
        so[LF] = __double2float_rn(rho);
        so[LG] = __double2float_rn(rhoE);
    }
    const double inv_rho = 1.0 / rho;
    const double u[3] = {j[0] * inv_rho, j[1] * inv_rho, j[2] * inv_rho};

    // species lattices, one at a time, the next one's loads in flight while
    // the current one is summed; rho_a goes to the record row PRM_SP + 6 a and
    // with u_a - u (zero for an absent species, u_a := u) to LDS
    double rs = rho, js[3] = {j[0], j[1], j[2]};
    auto put_species = [&](int a, double ra, double jx, double jy, double jz) {
        const bool small = ra <= 1e-14 * rho;
        const double inv = small ? 0.0 : 1.0 / ra;
        st_at(prm + (size_t)(PRM_SP + 6 * a) * N, node, ra);
        ls.ra[a * LOC_T] = ra;
        ls.dv[(3 * a + 0) * LOC_T] = small ? 0.0 : jx * inv - u[0];
        ls.dv[(3 * a + 1) * LOC_T] = small ? 0.0 : jy * inv - u[1];
        ls.dv[(3 * a + 2) * LOC_T] = small ? 0.0 : jz * inv - u[2];
    };
    // FP32 storage double-buffers the species loads (the first lattice's
    // were issued above); FP64 has no registers to spare for it
#pragma unroll 1
    for (int l = 0; l < NSP; ++l) {
        reload_barrier();
        S nxt[Q];
        if constexpr (PF) {
            if (l + 1 < NSP) {
#pragma unroll
                for (int i = 0; i < Q; ++i) nxt[i] = ld(l + 1, i);
            }
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) cur[i] = ld(l, i);
        }
        double ra = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
            const double v = (double)cur[i];
            ra += v;
            if (cx) jx += cx > 0 ? v : -v;
            if (cy) jy += cy > 0 ? v : -v;
            if (cz) jz += cz > 0 ? v : -v;
        }
        if constexpr (sizeof(S) == 4) {
            const RLBM_CONST double* rm = as_const(L.ref) + REF_M0<NL> + opaque_zero();
            ra += (double)sc[l] * rm[l];
            so[l] = __double2float_rn(ra);
        }
        const int a = W ? l : l + (l >= s ? 1 : 0);
        put_species(a, ra, jx, jy, jz);
        rs -= ra; js[0] -= jx; js[1] -= jy; js[2] -= jz;
        if constexpr (PF) {
#pragma unroll
            for (int i = 0; i < Q; ++i) cur[i] = nxt[i];
        }
    }
    if constexpr (!W) put_species(s, rs, js[0], js[1], js[2]);
    // the species densities come back from LDS rather than being held in
    // registers through the loop
#pragma unroll
    for (int c = 0; c < M; ++c) m.rho_a[c] = ls.ra[c * LOC_T];
    m.rho = rho;
    m.rhoE = rhoE;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        m.j[d] = j[d]; m.q[d] = q[d]; m.Pd[d] = Pd[d]; m.Po[d] = Po[d]; m.u[d] = u[d];
    }
}

template <int M, typename S, int W>
__global__ __launch_bounds__(NODE_TILE) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_local(const LatDev* __restrict__ lats, const int* __restrict__ blk,
                                               int n_lat, const long long* __restrict__ tp, long long toff) {
    const long long t = step_time(tp, toff);
    const int b = xcd_block();
    const int lj = find_lattice(blk, n_lat, b);
    const LatDev& L = lats[lj];
    if (t >= L.t_end) return;
    const int node = (b - blk[lj]) * NODE_TILE + threadIdx.x;
    if (node >= L.N) return;
    MechC mc = *as_const(L.mech);
    const int par = (L.parity0 + t) & 1;
    const int x = node % L.nx, r = node / L.nx, y = r % L.ny, z = r / L.ny;
    PullOff o;
    pull_offsets(L, x, y, z, o);
    const int k = L.n_if ? L.if_index[node] : -1;
    double* aux = L.aux;
    double* prm = L.prm;
    const size_t N = (size_t)L.N;

    __shared__ double s_ra[M][LOC_T], s_dv[3 * M][LOC_T];
    const LocalLds ls{&s_ra[0][threadIdx.x], &s_dv[0][threadIdx.x]};
    LocalMoments<M> m;
    if (__builtin_amdgcn_ballot_w64(k >= 0) != 0) local_moments<M, S, W, true>(L, par, k, node, o, ls, m);
    else local_moments<M, S, W, false>(L, par, k, node, o, ls, m);
    const double rho = m.rho, inv_rho = 1.0 / rho;
    const double u[3] = {m.u[0], m.u[1], m.u[2]};
    const double rhoE = m.rhoE;
    const double* rho_a = m.rho_a;
    const double* q = m.q;
    const double* Pd = m.Pd;
    const double* Po = m.Po;

    const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    // composition: Y_a = rho_a / rho, or rho_a / sum_b rho_b in the weakly
    // coupled storage, where the species supply the composition and the
    // momentum lattice rho
    double rhoY = rho;
    if constexpr (W) {
        rhoY = 0.0;
#pragma unroll
        for (int a = 0; a < M; ++a) rhoY += rho_a[a];
    }
    const double inv_rhoY = W ? 1.0 / rhoY : inv_rho;
    double Y[M];
#pragma unroll
    for (int a = 0; a < M; ++a) Y[a] = rho_a[a] * inv_rhoY;
    const double U = rhoE * inv_rho - 0.5 * usq;
    int fail = 0;
    // temperature (eq. temperature), Newton from the previous step's value
    const double T = solve_T<M>(mc, Y, U, aux[AUX_T * N + node], &fail);
    if (fail) atomicOr(L.flag, 1);
    const double Rmix = mc.R_univ * mix_inv_m<M>(mc, Y);
    const double th = Rmix * T;
    const double P = rho * th;

    // relaxation rates (sections 2.3 and 3.4); k_update derives the same
    // values again from the record rather than reading them
    double common, omega, omega1;
    relax_rates(mc, T, P, Rmix, common, omega, omega1);

    // enthalpy-weighted composition moments sum_a H_a(T') Y_a = sum_kk T'^kk Pk
    double Pk[6];
#pragma unroll
    for (int kk = 0; kk < 6; ++kk) {
        double pk = 0.0;
#pragma unroll
        for (int a = 0; a < M; ++a) pk += mc.hc[a][kk] * Y[a];
        Pk[kk] = pk;
    }
    // local part of the energy-lattice flux
    //   Qb = (omega - omega1)(q - u.(P - P^eq) - q^eq); the Stefan-Maxwell step adds
    //   omega1 rho sum_a H_a Y_a V_a
    double Qb[3];
    {
        const double H = Pk[0] + T * (Pk[1] + T * (Pk[2] + T * (Pk[3] + T * (Pk[4] + T * Pk[5]))));
        const double hq = rho * (H + 0.5 * usq);
        const double Pt[3][3] = {{Pd[0], Po[0], Po[1]}, {Po[0], Pd[1], Po[2]}, {Po[1], Po[2], Pd[2]}};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double uP = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) uP += u[c] * (Pt[c][a] - rho * ((a == c ? th : 0.0) + u[c] * u[a]));
            Qb[a] = (omega - omega1) * (q[a] - uP - hq * u[a]);
        }
    }

    // neighbour-facing fields: Phi and the enthalpy moments for the gradient
    // stencil, T for the next step's Newton start; rho, u and Y only where
    // an outlet reads them (the first interior node of the x+ face)
#pragma unroll
    for (int d = 0; d < 3; ++d)
        aux[(AUX_PHI + d) * N + node] = rho * u[d] * (1.0 - 3.0 * th) - rho * u[d] * u[d] * u[d];
    aux[AUX_T * N + node] = T;
#pragma unroll
    for (int kk = 0; kk < 6; ++kk) aux[(AUX_Y + M + kk) * N + node] = Pk[kk];
    if (L.n_out > 0 && x == L.nx - 2) {
        aux[AUX_RHO * N + node] = rho;
#pragma unroll
        for (int d = 0; d < 3; ++d) aux[(AUX_U + d) * N + node] = u[d];
#pragma unroll
        for (int a = 0; a < M; ++a) aux[(AUX_Y + a) * N + node] = Y[a];
    }

    prm[PRM_RHO * N + node] = rho;
#pragma unroll
    for (int d = 0; d < 3; ++d) prm[(PRM_U + d) * N + node] = u[d];
    prm[PRM_T * N + node] = T;
    prm[PRM_UINT * N + node] = U;
    stefan_maxwell<M, W, sizeof(S) == 4>(L, node, ls, T, rho, common, omega1, Y, Qb, rho * inv_rhoY);

    // reaction increment (eq. R3, forward Euler), with the LDS columns the
    // diffusion step has finished with; the arithmetic-bound chemistry then
    // runs under this kernel's memory traffic.  Lattices with the linearly
    // implicit update take it in k_chem_implicit.
    if (L.reaction == RLBM_REACTION_EXPLICIT) {
        reload_barrier();
        const ChemLds<LOC_T> cl{&s_dv[0][threadIdx.x], &s_dv[M][threadIdx.x], nullptr};
        double ra[M], fin[M];
#pragma unroll
        for (int a = 0; a < M; ++a) ra[a] = s_ra[a][threadIdx.x];
        double rY = rho;   // the density that normalises the composition
        if constexpr (W) {
            rY = 0.0;
#pragma unroll
            for (int a = 0; a < M; ++a) rY += ra[a];
        }
        int fail_r = 0;
        reaction_increment<M, LOC_T, false>(mc, ra, rY, U, T, L.substeps, cl, fin, &fail_r);
        if (fail_r) atomicOr(L.flag, 1);
        // Delta rho_a against the densities read again from LDS, so that they
        // need not stay in registers through the sub-steps
        reload_barrier();
#pragma unroll
        for (int a = 0; a < M; ++a)
            st_corr<sizeof(S) == 4>(as_global(prm), PRM_SP + 6 * a + 5, N, node, fin[a] - s_ra[a][threadIdx.x]);
    }
}

// ---------------------------------------------------------------------------
// same-time gradients with the isotropic D3Q27 stencil
//   d phi/dx_a = 3 sum_i w_i c_ia phi(x + c_i)
// of Phi_a (extension, eqs. Pex, qex) and of sum_b H_b Y_b with H_b at this
// node's temperature (Fourier correction, eq. corrFourier), from the fields
// k_local published.  Ghost values beyond a non-periodic face repeat the
// nearest node.  Writes rows PRM_GRAD..PRM_GRAD+5 of the per-node record.
// ---------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ void store_gradients(const LatDev& L, int node, const double (&acc)[6]) {
    const size_t N = (size_t)L.N;
    if (L.storage == RLBM_STORAGE_F32_DEV) {
#pragma unroll
        for (int q = 0; q < 6; ++q) st_corr<true>(as_global(L.prm), prm_grad(M) + q, N, node, acc[q]);
    } else {
#pragma unroll
        for (int q = 0; q < 6; ++q) st_corr<false>(as_global(L.prm), prm_grad(M) + q, N, node, acc[q]);
    }
}

// Any node: the 26 neighbours' fields, each at its own offset.
template <int M>
__device__ __forceinline__ void node_gradients(const LatDev& L, int node) {
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int x = node % nx, r = node / nx, y = r % ny, z = r / ny;
    const size_t N = (size_t)L.N;
    const double* aux = L.aux;
    const double T = L.prm[PRM_T * N + node];
    const double T2 = T * T, T3 = T2 * T, T4 = T3 * T, T5 = T4 * T;
    const bool px = L.per[0], py = L.per[1], pz = L.per[2];
    const int gx[3] = {x == 0 ? (px ? nx - 1 : 0) : x - 1, x, x == nx - 1 ? (px ? 0 : x) : x + 1};
    const int gy[3] = {y == 0 ? (py ? ny - 1 : 0) : y - 1, y, y == ny - 1 ? (py ? 0 : y) : y + 1};
    const int gz[3] = {z == 0 ? (pz ? nz - 1 : 0) : z - 1, z, z == nz - 1 ? (pz ? 0 : z) : z + 1};
    const double* Pk = aux + (size_t)(AUX_Y + M) * N;
    double acc[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll 1
    for (int czi = 0; czi < 3; ++czi) {
        const int cz = czi - 1;
        const size_t zrow = (size_t)sel3(cz, gz[0], gz[1], gz[2]) * ny;
        const double wz = cz ? 1.0 / 6.0 : 2.0 / 3.0;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int cx = j % 3 - 1, cy = j / 3 - 1;
            if (cx == 0 && cy == 0 && cz == 0) continue;
            const double w = 3.0 * (cx ? 1.0 / 6.0 : 2.0 / 3.0) * (cy ? 1.0 / 6.0 : 2.0 / 3.0) * wz;
            const size_t nb = (zrow + gy[cy + 1]) * nx + gx[cx + 1];
            const double hy = Pk[nb] + T * Pk[N + nb] + T2 * Pk[2 * N + nb] + T3 * Pk[3 * N + nb] +
                              T4 * Pk[4 * N + nb] + T5 * Pk[5 * N + nb];
            if (cx) { acc[0] += (cx * w) * aux[(AUX_PHI + 0) * N + nb]; acc[3] += (cx * w) * hy; }
            if (cy) { acc[1] += (cy * w) * aux[(AUX_PHI + 1) * N + nb]; acc[4] += (cy * w) * hy; }
            if (cz) { acc[2] += (cz * w) * aux[(AUX_PHI + 2) * N + nb]; acc[5] += (cz * w) * hy; }
        }
    }
    store_gradients<M>(L, node, acc);
}

// The weights factor per direction, w_i = w(c_ix) w(c_iy) w(c_iz) with
// w(0) = 2/3 and w(+-1) = 1/6.  With the sums over the 3x3 (y, z)
// neighbourhood of one column x
//   A(x) = sum w(cy) w(cz) phi,  B(x) = sum cy w(cz) phi,  C(x) = sum cz w(cy) phi
// the stencil is
//   d_x phi = (A(x+1) - A(x-1)) / 2,  d_y phi = sum_cx w(cx) B(x+cx) / 2,
//   d_z phi = sum_cx w(cx) C(x+cx) / 2.
// Column sums of one x: the six enthalpy coefficients (A, B, C each) and
// A of Phi_x, B of Phi_y, C of Phi_z.
struct ColSums {
    double a[6], b[6], c[6];
    double ax, by, cz;
};
template <int M>
__device__ __forceinline__ void column_sums(const LatDev& L, int xc, const int (&gy)[3], const int (&gz)[3],
                                            ColSums& o) {
    const size_t N = (size_t)L.N;
    const int nx = L.nx, ny = L.ny;
    const double* aux = L.aux;
    const double* Pk = aux + (size_t)(AUX_Y + M) * N;
#pragma unroll
    for (int k = 0; k < 6; ++k) o.a[k] = o.b[k] = o.c[k] = 0.0;
    o.ax = o.by = o.cz = 0.0;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const int cy = j % 3 - 1, cz = j / 3 - 1;
        const double wy = cy ? 1.0 / 6.0 : 2.0 / 3.0, wz = cz ? 1.0 / 6.0 : 2.0 / 3.0;
        const size_t nb = ((size_t)gz[cz + 1] * ny + gy[cy + 1]) * nx + xc;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double f = Pk[k * N + nb];
            o.a[k] += (wy * wz) * f;
            if (cy) o.b[k] += (cy * wz) * f;
            if (cz) o.c[k] += (cz * wy) * f;
        }
        o.ax += (wy * wz) * aux[(AUX_PHI + 0) * N + nb];
        if (cy) o.by += (cy * wz) * aux[(AUX_PHI + 1) * N + nb];
        if (cz) o.cz += (cz * wy) * aux[(AUX_PHI + 2) * N + nb];
    }
}

__device__ __forceinline__ double poly5(double t, const double (&v)[6]) {
    return v[0] + t * (v[1] + t * (v[2] + t * (v[3] + t * (v[4] + t * v[5]))));
}

// A wave whose 64 lanes are the consecutive nodes x0..x0+63 of one x-row
// (lane = x - x0): each lane loads its own column's 9 (y, z) neighbours and
// takes the column sums of x-1 and x+1 from the adjacent lanes; lane 0 and
// lane 63 load the ghost-aware column beyond the tile themselves.  The sum
// of H_b Y_b at this node's temperature is formed from the neighbour's
// coefficient sums, so a lane evaluates its sums at the temperature of the
// lane that receives them (the adjacent lane's T).  Every lane of the wave
// must reach this function.
template <int M>
__device__ __forceinline__ void row_tile_gradients(const LatDev& L, int node, int lane) {
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int x = node % nx, r = node / nx, y = r % ny, z = r / ny;
    const size_t N = (size_t)L.N;
    const double T = L.prm[PRM_T * N + node];
    const bool px = L.per[0], py = L.per[1], pz = L.per[2];
    const int gy[3] = {y == 0 ? (py ? ny - 1 : 0) : y - 1, y, y == ny - 1 ? (py ? 0 : y) : y + 1};
    const int gz[3] = {z == 0 ? (pz ? nz - 1 : 0) : z - 1, z, z == nz - 1 ? (pz ? 0 : z) : z + 1};
    // the adjacent lanes' temperatures (lane 0 and lane 63 keep their own;
    // what they would send across the tile edge is not used)
    const double Tl = __shfl_up(T, 1u), Tr = __shfl_down(T, 1u);
    // from x+1 (sums at this lane's T), from x-1, and this column's own
    double hp_a, hp_b, hp_c, hm_a, hm_b, hm_c, h0_b, h0_c, fp_ax, fp_by, fp_cz, fm_ax, fm_by, fm_cz, f0_by, f0_cz;
    {
        ColSums s;
        column_sums<M>(L, x, gy, gz, s);
        h0_b = poly5(T, s.b);
        h0_c = poly5(T, s.c);
        f0_by = s.by;
        f0_cz = s.cz;
        hp_a = __shfl_down(poly5(Tl, s.a), 1u);
        hp_b = __shfl_down(poly5(Tl, s.b), 1u);
        hp_c = __shfl_down(poly5(Tl, s.c), 1u);
        hm_a = __shfl_up(poly5(Tr, s.a), 1u);
        hm_b = __shfl_up(poly5(Tr, s.b), 1u);
        hm_c = __shfl_up(poly5(Tr, s.c), 1u);
        fp_ax = __shfl_down(s.ax, 1u);
        fp_by = __shfl_down(s.by, 1u);
        fp_cz = __shfl_down(s.cz, 1u);
        fm_ax = __shfl_up(s.ax, 1u);
        fm_by = __shfl_up(s.by, 1u);
        fm_cz = __shfl_up(s.cz, 1u);
    }
    if (lane == 0 || lane == NODE_TILE - 1) {
        const int xg = lane == 0 ? (x == 0 ? (px ? nx - 1 : 0) : x - 1) : (x == nx - 1 ? (px ? 0 : x) : x + 1);
        ColSums s;
        column_sums<M>(L, xg, gy, gz, s);
        const double ga = poly5(T, s.a), gb = poly5(T, s.b), gc = poly5(T, s.c);
        if (lane == 0) {
            hm_a = ga; hm_b = gb; hm_c = gc; fm_ax = s.ax; fm_by = s.by; fm_cz = s.cz;
        } else {
            hp_a = ga; hp_b = gb; hp_c = gc; fp_ax = s.ax; fp_by = s.by; fp_cz = s.cz;
        }
    }
    constexpr double w0 = 2.0 / 3.0, w1 = 1.0 / 6.0;
    const double acc[6] = {0.5 * (fp_ax - fm_ax),
                           0.5 * (w1 * fm_by + w0 * f0_by + w1 * fp_by),
                           0.5 * (w1 * fm_cz + w0 * f0_cz + w1 * fp_cz),
                           0.5 * (hp_a - hm_a),
                           0.5 * (w1 * hm_b + w0 * h0_b + w1 * hp_b),
                           0.5 * (w1 * hm_c + w0 * h0_c + w1 * hp_c)};
    store_gradients<M>(L, node, acc);
}

// ---------------------------------------------------------------------------
// k_gradients: the same-time gradients of every node of the lattices whose
// reaction increment k_local has written (the forward-Euler update).
// k_chem_implicit: for lattices with the linearly implicit update, that
// increment (reading rho_a, rho, U, T from the per-node record and writing
// Delta rho_a into it), then the gradients.  The stencil's neighbour loads
// are latency-bound and the implicit chemistry arithmetic-bound, so the two
// share one launch.  A launch serves the lattices of its scheme; the blocks of
// the others return at once.
// ---------------------------------------------------------------------------
template <int M, bool IMPL>
__device__ __forceinline__ void chem_body(const LatDev* __restrict__ lats, const int* __restrict__ blk, int n_lat,
                                          const long long* __restrict__ tp, long long toff, int b, int tid) {
    const long long t = step_time(tp, toff);
    const int lj = find_lattice(blk, n_lat, b);
    const LatDev& L = lats[lj];
    if (t >= L.t_end) return;
    if ((L.reaction == RLBM_REACTION_LINEARLY_IMPLICIT) != IMPL) return;
    const int node = (b - blk[lj]) * NODE_TILE + tid;
    if (node >= L.N) return;
    if constexpr (IMPL) {
        MechC mc = *as_const(L.mech);
        double* prm = L.prm;
        const size_t N = (size_t)L.N;
        __shared__ double s_c[M][NODE_TILE], s_g[M][NODE_TILE], s_q[M][NODE_TILE];
        const ChemLds<NODE_TILE> ls{&s_c[0][threadIdx.x], &s_g[0][threadIdx.x], &s_q[0][threadIdx.x]};
        double rho_a[M], fin[M];
#pragma unroll
        for (int a = 0; a < M; ++a) rho_a[a] = prm[(PRM_SP + 6 * a) * N + node];
        // the density that normalises the composition (sum_a rho_a in the
        // weakly coupled storage)
        double rho = prm[PRM_RHO * N + node];
        if (L.weak) {
            rho = 0.0;
#pragma unroll
            for (int a = 0; a < M; ++a) rho += rho_a[a];
        }
        const double U = prm[PRM_UINT * N + node];
        const double T = prm[PRM_T * N + node];
        int fail = 0;
        reaction_increment<M, NODE_TILE, true>(mc, rho_a, rho, U, T, L.substeps, ls, fin, &fail);
        if (fail) atomicOr(L.flag, 1);
        // Delta rho_a against the densities read again, so that they need not
        // stay in registers through the sub-steps
        reload_barrier();
        if (L.storage == RLBM_STORAGE_F32_DEV) {
#pragma unroll
            for (int a = 0; a < M; ++a)
                st_corr<true>(as_global(prm), PRM_SP + 6 * a + 5, N, node, fin[a] - prm[(PRM_SP + 6 * a) * N + node]);
        } else {
#pragma unroll
            for (int a = 0; a < M; ++a)
                st_corr<false>(as_global(prm), PRM_SP + 6 * a + 5, N, node, fin[a] - prm[(PRM_SP + 6 * a) * N + node]);
        }
    }
    // wave-uniform: the tile's 64 nodes lie in one x-row
    const int x0 = __builtin_amdgcn_readfirstlane((node - tid) % L.nx);
    if (x0 + NODE_TILE <= L.nx)
        row_tile_gradients<M>(L, node, tid);
    else
        node_gradients<M>(L, node);
}

// GRAD_TILES tiles per block, one wave each (the stencil shares nothing
// between waves): the lattice of each tile is looked up per wave, and tiles
// past the end of the list return.
constexpr int GRAD_TILES = 4;
static_assert(NODE_TILE == 64, "one wave per tile");
template <int M>
__global__ __launch_bounds__(GRAD_TILES * NODE_TILE) void k_gradients(const LatDev* __restrict__ lats,
                                                                      const int* __restrict__ blk, int n_lat,
                                                                      const long long* __restrict__ tp, long long toff) {
    const int tile = xcd_block() * GRAD_TILES + __builtin_amdgcn_readfirstlane((int)threadIdx.x / NODE_TILE);
    if (tile >= blk[n_lat]) return;
    chem_body<M, false>(lats, blk, n_lat, tp, toff, tile, (int)threadIdx.x % NODE_TILE);
}

// The linearly implicit variant holds an (M-1)^2 matrix in registers.
template <int M>
__global__ __launch_bounds__(NODE_TILE) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_chem_implicit(
    const LatDev* __restrict__ lats, const int* __restrict__ blk, int n_lat, const long long* __restrict__ tp, long long toff) {
    chem_body<M, true>(lats, blk, n_lat, tp, toff, xcd_block(), (int)threadIdx.x);
}


// ---------------------------------------------------------------------------
// k_update: the collision of every stored lattice (section 2.3 eq.
// finalNumericalEquationsReactive, section 3.2 eq. f, section 3.3 eq. g).
// A block of three waves covers 64 consecutive nodes; wave w takes the nine
// velocities with c_z = w - 1, one node per lane.  The per-node record is
// staged once in LDS with the species in slot order (the stored species in
// lattice order, then the slaved one), so every per-species quantity sits at
// a compile-time index.  Product-form factors along y and z are formed once
// per row of three velocities (fixed c_y, c_z); the x factor per velocity.
// ---------------------------------------------------------------------------
// Record rows k_update reads: rho, u, T, U (0..5), the energy-flux base
// (9..11), per species slot rho_a, V_a and Delta rho_a (c = 0..3, 5), and the
// six gradient rows.  theta, omega, the diffusion factor, omega - omega_1,
// (2 - omega_1) P / 2 and beta_a are derived in the kernel instead.
__host__ __device__ constexpr int upd_loaded_rows(int M) { return 9 + 5 * M + 6; }
__host__ __device__ constexpr int upd_loaded_row(int M, int idx) {
    return idx < 6 ? idx
                   : idx < 9 ? idx + 3
                             : idx < 9 + 5 * M ? PRM_SP + 6 * ((idx - 9) / 5) + ((idx - 9) % 5 < 4 ? (idx - 9) % 5 : 5)
                                               : prm_grad(M) + (idx - 9 - 5 * M);
}

constexpr int UPD_NODES = 64;
constexpr int UPD_WAVES = 3;
constexpr int UPD_THREADS = UPD_WAVES * UPD_NODES;

// Product-form factor with a compile-time velocity component C.
template <int C>
__device__ __forceinline__ double psi_c(double xi, double P) {
    if constexpr (C == 0) return 1.0 - P;
    else if constexpr (C > 0) return 0.5 * (P + xi);
    else return 0.5 * (P - xi);
}

// Product-form factor with a wave-uniform component c, as a + b xi + d P.
struct PsiCoef {
    double a, b, d;
};
__device__ __forceinline__ PsiCoef psi_coef(int c) {
    PsiCoef r;
    r.a = c == 0 ? 1.0 : 0.0;
    r.b = 0.5 * (double)c;
    r.d = c == 0 ? -1.0 : 0.5;
    return r;
}
__device__ __forceinline__ double psi_u(const PsiCoef& k, double xi, double P) {
    return fma(k.b, xi, fma(k.d, P, k.a));
}
// Energy-equilibrium axis factors (W, k) of eq. geq_i for a uniform c.
__device__ __forceinline__ void geq_wk(int c, double u, double th, double& W, double& k) {
    const double u2 = u * u;
    const double P = th + u2;
    const double o1 = th * u + 0.5 * u2 * u;
    const double o2 = th * th + 2.5 * th * u2 + 0.5 * u2 * u2;
    const PsiCoef pc = psi_coef(c);
    W = psi_u(pc, u, P);
    // k_0 = u^2/2 - o2, k_{+-1} = (o2 +- o1)/2
    k = c == 0 ? 0.5 * u2 - o2 : 0.5 * (o2 + (double)c * o1);
}


// The weakly coupled storage's extra lattice would otherwise take the
// kernel just past three waves per SIMD (the LDS allows three).
template <int M, typename S, int W>
__global__ __launch_bounds__(UPD_THREADS) __attribute__((amdgpu_waves_per_eu(W ? 3 : 1))) void k_update(const LatDev* __restrict__ lats, const int* __restrict__ blk,
                                                        int n_lat, const long long* __restrict__ tp, long long toff) {
    const long long t = step_time(tp, toff);
    constexpr int NR = prm_rows(M);
    constexpr int NSP = Lat<M, W>::NSP, LF = Lat<M, W>::LF, LG = Lat<M, W>::LG;
    constexpr int NL = Lat<M, W>::NL;   // stored lattices
    constexpr int NS = sizeof(S) == 4 ? NL : 1;
    __shared__ double sp[NR][UPD_NODES];
    __shared__ float ssc[NS][UPD_NODES];     // FP32 storage: this node's reference scales
    const int b = xcd_block();
    const int lj = find_lattice(blk, n_lat, b);
    const LatDev& L = lats[lj];
    if (t >= L.t_end) return;
    const int node0 = (b - blk[lj]) * UPD_NODES;
    const int lane = threadIdx.x % UPD_NODES;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / UPD_NODES);
    const int c2 = wave - 1;
    const int node = node0 + lane;
    const int N = (int)L.N;
    const bool valid = node < N;
    const int s = W ? M : L.slaved;
    const int par = (L.parity0 + t) & 1;
    const RLBM_GLOBAL S* src = as_global(static_cast<const S*>(L.pop[par]));
    RLBM_GLOBAL S* dst = as_global(static_cast<S*>(L.pop[par ^ 1]));
    const size_t P = (size_t)L.P;
    const RLBM_GLOBAL double* prm = as_global(L.prm);

    // stage the record's stored rows (species rows in slot order) and (FP32
    // storage) this node's reference scales: wave w takes stored rows w,
    // w + 3, ..., one node per lane; every load is in flight before the first
    // LDS write.  The rows derived below are not read.
    {
        constexpr int NLD = upd_loaded_rows(M);
        constexpr int RPW = (NLD + UPD_WAVES - 1) / UPD_WAVES;
        constexpr int LPW = (NS + UPD_WAVES - 1) / UPD_WAVES;
        const int nd = node0 + lane < N ? node0 + lane : 0;   // beyond the end: a placeholder node
        // one copy per wave, so that each load's row, and with it its width
        // (the correction rows are FP32 in FP32 storage), is a compile-time
        // constant: no branches between the loads
        auto stage = [&](auto wave_c) {
            constexpr int WV = decltype(wave_c)::value;
            double v[RPW];
            float vf[RPW];
            float w[LPW];
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const int idx = WV + UPD_WAVES * q;
                const int row = upd_loaded_row(M, idx < NLD ? idx : 0);
                int srow = row;
                if (row >= PRM_SP && row < prm_grad(M)) {
                    const int slot = (row - PRM_SP) / 6, c = (row - PRM_SP) % 6;
                    const int a = W ? slot : (slot < M - 1 ? slot + (slot >= s ? 1 : 0) : s);
                    srow = PRM_SP + 6 * a + c;
                }
                // unconditional: no waits between
                if (sizeof(S) == 4 && prm_is_corr(M, row))
                    vf[q] = ld_at(reinterpret_cast<const RLBM_GLOBAL float*>(prm + (size_t)srow * L.N), nd);
                else
                    v[q] = ld_at(prm + (size_t)srow * L.N, nd);
            }
            if constexpr (sizeof(S) == 4) {
                const RLBM_GLOBAL float* sc = scale_at(L, par, nd);
#pragma unroll
                for (int q = 0; q < LPW; ++q) {
                    const int l = WV + UPD_WAVES * q;
                    w[q] = sc[l < NS ? l : 0];
                }
            }
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const int idx = WV + UPD_WAVES * q;
                if (idx < NLD) {
                    const int row = upd_loaded_row(M, idx);
                    sp[row][lane] = (sizeof(S) == 4 && prm_is_corr(M, row)) ? (double)vf[q] : v[q];
                }
            }
            if constexpr (sizeof(S) == 4) {
#pragma unroll
                for (int q = 0; q < LPW; ++q) {
                    const int l = WV + UPD_WAVES * q;
                    if (l < NS) ssc[l][lane] = w[q];
                }
            }
        };
        static_assert(UPD_WAVES == 3, "one staging copy per wave");
        if (wave == 0) stage(std::integral_constant<int, 0>{});
        else if (wave == 1) stage(std::integral_constant<int, 1>{});
        else stage(std::integral_constant<int, 2>{});
    }

    int x = 0, y = 0, z = 0;
    if (valid) { x = node % L.nx; const int r = node / L.nx; y = r % L.ny; z = r / L.ny; }
    const int k = (L.n_if && valid) ? as_global(L.if_index)[node] : -1;
    const bool wave_if = __builtin_amdgcn_ballot_w64(k >= 0) != 0;   // uniform
    PullOff o;
    pull_offsets(L, x, y, z, o);
    const int offz = node + sel3(c2, o.z[0], 0, o.z[2]);

    // populations of velocity i at node offset off (after advection and
    // boundary reconstruction: an interface lane reads the plane's interface
    // slot N + k)
    auto load = [&](int i, int off, S* out) {
        const int idx = wave_if && k >= 0 ? N + k : off;
#pragma unroll
        for (int l = 0; l < NL; ++l) out[l] = ld_at(src + (size_t)(l * Q + i) * P, idx);
    };
    // FP32 deviation storage: reference scales of this node (decode) and of
    // the node that reads what is written for velocity (c0, c1, c2) (encode)
    constexpr int NS4 = (NS + 3) / 4;
    auto load_scales = [&](int q, int n, float* out) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const RLBM_GLOBAL f4* p4 = reinterpret_cast<const RLBM_GLOBAL f4*>(scale_at(L, q, n));
#pragma unroll
        for (int v = 0; v < NS4; ++v) {
            const f4 w = p4[v];
            if (4 * v + 0 < NS) out[4 * v + 0] = w.x;
            if (4 * v + 1 < NS) out[4 * v + 1] = w.y;
            if (4 * v + 2 < NS) out[4 * v + 2] = w.z;
            if (4 * v + 3 < NS) out[4 * v + 3] = w.w;
        }
    };
    auto reader = [&](int c0, int c1, int c2) {
        return node + sel3(c0, o.x[2], 0, o.x[0]) + sel3(c1, o.y[2], 0, o.y[0]) + sel3(c2, o.z[2], 0, o.z[0]);
    };

    S fin[NL];
    const int i_first = 9 * (c2 + 1);
    if (valid) load(i_first, offz + o.y[0] + o.x[0], fin);
    __syncthreads();
    // the derived rows, once per node by the first wave: theta, the
    // relaxation rates (as k_local computes them) and beta_a =
    // 1/(2 tau_a + 1) with 1/tau_a = common sum_{b != a} K_ab Y_b (eqs.
    // betaa, taua), Y in slot order
    if (wave == 0) {
        MechC mc = *as_const(L.mech);
        const RLBM_CONST double* slotc = as_const(L.slotc);
        const double T = sp[PRM_T][lane], rho = sp[PRM_RHO][lane];
        double ry = rho;   // Y_a = rho_a / rho, or rho_a / sum_b rho_b (weakly coupled)
        if constexpr (W) {
            ry = 0.0;
#pragma unroll
            for (int q = 0; q < M; ++q) ry += sp[PRM_SP + 6 * q][lane];
        }
        const double iry = 1.0 / ry;
        double Y[M];
        double Rmix = 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q) {
            Y[q] = sp[PRM_SP + 6 * q][lane] * iry;
            Rmix = fma(Y[q], slotc[q], Rmix);
        }
        const double th = Rmix * T, P = rho * th;
        double common, omega, omega1;
        relax_rates(mc, T, P, Rmix, common, omega, omega1);
        sp[PRM_TH][lane] = th;
        sp[PRM_OMEGA][lane] = omega;
        sp[PRM_COMMON][lane] = common;
        sp[PRM_WQ][lane] = omega - omega1;
        sp[PRM_CC][lane] = 0.5 * (2.0 - omega1) * P;
        const RLBM_CONST double* Ks = slotc + M;
#pragma unroll
        for (int j = 0; j < NSP; ++j) {
            double st = 0.0;
#pragma unroll
            for (int q = 0; q < M; ++q)
                if (q != j) st = fma(Ks[j * M + q], Y[q], st);
            const double inv_tau = common * st;
            sp[PRM_SP + 6 * j + 4][lane] = inv_tau / (2.0 + inv_tau);
        }
    }
    __syncthreads();
    if (!valid) return;

    const int GR = prm_grad(M);
    // per-node values used by every velocity are re-read from LDS where they
    // are needed; only the few derived ones stay in registers
    const double exf = [&] {
        const double w = sp[PRM_OMEGA][lane];
        return (2.0 - w) / (2.0 * sp[PRM_RHO][lane] * w);
    }();
    // F_ai = common Y_a sum_b K_ab D_bi with Y_a = rho_a / rho, or
    // rho_a / sum_b rho_b in the weakly coupled storage
    const double fcm = [&] {
        double ry = sp[PRM_RHO][lane];
        if constexpr (W) {
            ry = 0.0;
#pragma unroll
            for (int q = 0; q < M; ++q) ry += sp[PRM_SP + 6 * q][lane];
        }
        return sp[PRM_COMMON][lane] / ry;
    }();
    const PsiCoef pz = psi_coef(c2);

#pragma unroll 1
    for (int c1 = -1; c1 <= 1; ++c1) {
        reload_barrier();
        const RLBM_CONST double* Ra = as_const(L.slotc) + opaque_zero();   // [M] gas constants, slot order
        const PsiCoef py = psi_coef(c1);
        const int offyz = offz + sel3(c1, o.y[0], 0, o.y[2]);
        const double T = sp[PRM_T][lane], th = sp[PRM_TH][lane];
        const double uy = sp[PRM_U + 1][lane], uz = sp[PRM_U + 2][lane];
        // y/z factors of the species equilibria (xi = u) and quasi-equilibria
        // (xi = u + V_b, eq. xiPstar2)
        double YZe[M], YZs[M];
#pragma unroll
        for (int q = 0; q < M; ++q) {
            const double tq = Ra[q] * T;
            const double vy = uy + sp[PRM_SP + 6 * q + 2][lane], vz = uz + sp[PRM_SP + 6 * q + 3][lane];
            YZe[q] = psi_u(py, uy, fma(uy, uy, tq)) * psi_u(pz, uz, fma(uz, uz, tq));
            YZs[q] = psi_u(py, vy, fma(vy, vy, tq)) * psi_u(pz, vz, fma(vz, vz, tq));
        }
        // momentum lattice: y/z factors of the extended equilibrium (eq. Pex)
        const double Fyz = psi_u(py, uy, th + uy * uy + exf * sp[GR + 1][lane]) *
                           psi_u(pz, uz, th + uz * uz + exf * sp[GR + 2][lane]);
        // energy lattice: y/z factors of eq. geq_i
        double Wy, ky, Wz, kz;
        geq_wk(c1, uy, th, Wy, ky);
        geq_wk(c2, uz, th, Wz, kz);
        const double Wyz = Wy * Wz, kyz = ky * Wz + Wy * kz;
        const int cyz2 = c1 * c1 + c2 * c2;

        auto body = [&](auto c0t) {
            constexpr int c0 = decltype(c0t)::value;
            const int i = 9 * (c2 + 1) + 3 * (c1 + 1) + (c0 + 1);
            // per-velocity re-reads of LDS and constants (cheap) instead of
            // keeping them live across the three velocities
            reload_barrier();
            const RLBM_CONST double* slotc = as_const(L.slotc) + opaque_zero();
            const RLBM_CONST double* Ra = slotc;
            const RLBM_CONST double* Ks = slotc + M;
            const RLBM_CONST double* ref = as_const(L.ref) + opaque_zero();
            // scales of the node that reads what this velocity writes (L2 hits,
            // consumed after the species work below), issued before the
            // prefetch so that waiting for them leaves the prefetch in flight
            float srd[NS];
            if constexpr (sizeof(S) == 4) load_scales(par ^ 1, reader(c0, c1, c2), srd);
            // prefetch the next velocity of this thread
            S fnx[NL];
            if constexpr (c0 < 1) {
                load(i + 1, offyz + o.x[c0 + 2], fnx);
            } else {
                if (c1 < 1) load(i + 1, offyz + sel3(c1 + 1, o.y[0], 0, o.y[2]) - sel3(c1, o.y[0], 0, o.y[2]) + o.x[0], fnx);
            }
            const double T = sp[PRM_T][lane], ux = sp[PRM_U][lane];
            double D[M];
#pragma unroll
            for (int q = 0; q < M; ++q) {
                reload_barrier();   // keep each species' LDS reads next to their use
                const double tq = Ra[q] * T;
                const double vx = ux + sp[PRM_SP + 6 * q + 1][lane];
                const double Xe = psi_c<c0>(ux, fma(ux, ux, tq));
                const double Xs = psi_c<c0>(vx, fma(vx, vx, tq));
                D[q] = sp[PRM_SP + 6 * q][lane] * (Xe * YZe[q] - Xs * YZs[q]);
            }
            // species (eq. finalNumericalEquationsReactive with eq. fStar)
#pragma unroll
            for (int j = 0; j < NSP; ++j) {
                reload_barrier();
                double F = 0.0;
#pragma unroll
                for (int q = 0; q < M; ++q)
                    if (q != j) F = fma(Ks[j * M + q], D[q], F);
                const double ra = sp[PRM_SP + 6 * j][lane], be = sp[PRM_SP + 6 * j + 4][lane],
                             dr = sp[PRM_SP + 6 * j + 5][lane];
                const double Wj = psi_c<c0>(ux, fma(ux, ux, Ra[j] * T)) * YZe[j];   // W_ji, recomputed
                const int li = j * Q + i;
                double f = (double)fin[j];
                if constexpr (sizeof(S) == 4) f += ref_of(ssc[j][lane], ref[li]);
                const double out = f + 2.0 * be * (ra * Wj - f) + (be - 1.0) * (fcm * ra * F) + Wj * dr;
                if constexpr (sizeof(S) == 4)
                    st_at(dst + (size_t)li * P, node, __double2float_rn(out - ref_of(srd[j], ref[li])));
                else st_at(dst + (size_t)li * P, node, out);
            }
            const double rho = sp[PRM_RHO][lane], th = sp[PRM_TH][lane], omega = sp[PRM_OMEGA][lane];
            // momentum lattice, extended equilibrium (eqs. f, feqmix, Pex)
            {
                const int li = LF * Q + i;
                double f = (double)fin[LF];
                if constexpr (sizeof(S) == 4) f += ref_of(ssc[LF][lane], ref[li]);
                const double fe = rho * psi_c<c0>(ux, th + ux * ux + exf * sp[GR][lane]) * Fyz;
                const double out = f + omega * (fe - f);
                if constexpr (sizeof(S) == 4)
                    st_at(dst + (size_t)li * P, node, __double2float_rn(out - ref_of(srd[LF], ref[li])));
                else st_at(dst + (size_t)li * P, node, out);
            }
            // energy lattice (eqs. g, geq_i, gstar)
            {
                const int li = LG * Q + i;
                double g = (double)fin[LG];
                if constexpr (sizeof(S) == 4)
                    g += ref_g(ssc[LG][lane], ssc[LF][lane], ref[li], ref[REF_K<NL> + i]);
                const double ux2 = ux * ux;
                const double Wx = psi_c<c0>(ux, th + ux2);
                double kx;
                if constexpr (c0 == 0) {
                    kx = 0.5 * ux2 - (th * th + 2.5 * th * ux2 + 0.5 * ux2 * ux2);
                } else {
                    const double o1 = th * ux + 0.5 * ux2 * ux;
                    const double o2 = th * th + 2.5 * th * ux2 + 0.5 * ux2 * ux2;
                    kx = 0.5 * (o2 + (double)c0 * o1);
                }
                const double geq = rho * (Wyz * (sp[PRM_UINT][lane] * Wx + kx) + Wx * kyz);
                double out = g + omega * (geq - g);
                // the singularity-free flux term on the six |c| = 1 velocities
                const double wq = sp[PRM_WQ][lane], cc = sp[PRM_CC][lane];
                if constexpr (c0 != 0) {
                    if (cyz2 == 0)
                        out += 0.5 * (double)c0 *
                               (sp[PRM_QB][lane] - 0.5 * wq * ux * sp[GR][lane] + cc * sp[GR + 3][lane]);
                } else {
                    if (cyz2 == 1) {
                        const int ax = c1 != 0 ? 1 : 2;   // uniform
                        const double ua = sp[PRM_U + ax][lane];
                        const double Qa = sp[PRM_QB + ax][lane] - 0.5 * wq * ua * sp[GR + ax][lane] +
                                          cc * sp[GR + 3 + ax][lane];
                        out += 0.5 * (double)(c1 + c2) * Qa;
                    }
                }
                if constexpr (sizeof(S) == 4)
                    st_at(dst + (size_t)li * P, node,
                          __double2float_rn(out - ref_g(srd[LG], srd[LF], ref[li], ref[REF_K<NL> + i])));
                else st_at(dst + (size_t)li * P, node, out);
            }
#pragma unroll
            for (int l = 0; l < NL; ++l) fin[l] = fnx[l];
        };
        body(std::integral_constant<int, -1>{});
        body(std::integral_constant<int, 0>{});
        body(std::integral_constant<int, 1>{});
    }
}

// ---------------------------------------------------------------------------
// boundary reconstruction (section 4)
// ---------------------------------------------------------------------------
// Equilibrium of lattice l at velocity i for the state (rho, Y, u, T)
// (section 4.1, eqs. faEqGeneral, fEqGeneral, gEqGeneral).  With SPV the
// species equilibria use per-species velocities us (the wall's local state,
// eq. locua); otherwise the mixture velocity.
template <int M, bool SPV>
struct EqState {
    double rho, th, U, T;
    double u[3];
    double Y[M];
    double us[SPV ? M : 1][3];
};

template <int M, bool SPV>
__device__ __forceinline__ void eq_prepare(MechC mc, EqState<M, SPV>& e, double T) {
    e.T = T;
    e.th = mc.R_univ * mix_inv_m<M>(mc, e.Y) * T;
    e.U = mix_U<M>(mc, e.Y, T);
}

template <int M, int W, bool SPV>
__device__ __forceinline__ double eq_value(MechC mc, const EqState<M, SPV>& e, int l, int slaved, int i) {
    constexpr int LF = Lat<M, W>::LF, LG = Lat<M, W>::LG;
    const int c0 = cx_of(i), c1 = cy_of(i), c2 = cz_of(i);
    if (l == LG) {
        GeqAxis gx, gy, gz;
        geq_axis(e.u[0], e.th, gx);
        geq_axis(e.u[1], e.th, gy);
        geq_axis(e.u[2], e.th, gz);
        const double Wx = sel3d(c0, gx.W[0], gx.W[1], gx.W[2]), kx = sel3d(c0, gx.k[0], gx.k[1], gx.k[2]);
        const double Wy = sel3d(c1, gy.W[0], gy.W[1], gy.W[2]), ky = sel3d(c1, gy.k[0], gy.k[1], gy.k[2]);
        const double Wz = sel3d(c2, gz.W[0], gz.W[1], gz.W[2]), kz = sel3d(c2, gz.k[0], gz.k[1], gz.k[2]);
        return e.rho * (e.U * Wx * Wy * Wz + kx * Wy * Wz + Wx * (ky * Wz + Wy * kz));
    }
    if (l == LF)
        return e.rho * psi(c0, e.u[0], e.u[0] * e.u[0] + e.th) * psi(c1, e.u[1], e.u[1] * e.u[1] + e.th) *
               psi(c2, e.u[2], e.u[2] * e.u[2] + e.th);
    const int a = W ? l : l + (l >= slaved ? 1 : 0);
    double Ya = 0.0, tha = 0.0, w0 = e.u[0], w1 = e.u[1], w2 = e.u[2];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        if (c == a) {
            Ya = e.Y[c];
            tha = mc.Ra[c] * e.T;
            if constexpr (SPV) { w0 = e.us[c][0]; w1 = e.us[c][1]; w2 = e.us[c][2]; }
        }
    }
    return e.rho * Ya * psi(c0, w0, w0 * w0 + tha) * psi(c1, w1, w1 * w1 + tha) * psi(c2, w2, w2 * w2 + tha);
}

// ---------------------------------------------------------------------------
// k_boundary: reconstruction at interface nodes (section 4).  A block takes
// 64 consecutive entries of the interface list (grouped by boundary type and
// ordered by node within a type, so mostly a run of a wall row or plane),
// one lane per node, and one wave per stored lattice: every population load
// and store of a wave is coalesced and its lattice, with the lattice's
// constants, is the same for the whole wave.  Each wave loads its lattice's
// populations once, in one pass with all 27 loads in flight, and keeps them
// in LDS for the moments and the reconstruction (the pull reads of the
// interface list are scattered over the lattice, so a second pass over them
// costs as much as the first); lattices beyond what the LDS holds beside the
// node states read them again per pass.  The output goes to the interface
// slots N + k of the planes of the buffer the step reads.  The node's state goes between the waves
// through LDS: the lattices' moments, and the imposed and local states that
// the first wave forms from them (temperature by the bounded Newton
// iteration, the LODI outlet state).  All barriers are at the top level of
// the kernel, so every wave meets all of them.
// ---------------------------------------------------------------------------
static_assert(BC_NODES == 64, "one lane per node in a wave");

// An equilibrium of one lattice at velocity i: s (U Wx Wy Wz + kx Wy Wz +
// Wx (ky Wz + Wy kz)), with W[d][c + 1] the product-form factor of axis d.
// The species and momentum lattices have U = 1 and k = 0; the energy lattice
// has the factors of eq. geq_i (section 3.3) and U the internal energy.
struct LatEq {
    double s, U;
    double W[3][3], k[3][3];
};

__device__ __forceinline__ void eq_axis(double w, double th, bool energy, double* Wa, double* ka) {
    const double w2 = w * w;
    const double P = th + w2;
    Wa[0] = 0.5 * (P - w);
    Wa[1] = 1.0 - P;
    Wa[2] = 0.5 * (P + w);
    if (energy) {
        const double o1 = th * w + 0.5 * w2 * w;
        const double o2 = th * th + 2.5 * th * w2 + 0.5 * w2 * w2;
        ka[0] = 0.5 * (o2 - o1);
        ka[1] = 0.5 * w2 - o2;
        ka[2] = 0.5 * (o2 + o1);
    } else {
        ka[0] = ka[1] = ka[2] = 0.0;
    }
}

template <int C0, int C1, int C2>
__device__ __forceinline__ double lat_eq(const LatEq& e) {
    const double wx = e.W[0][C0 + 1], wy = e.W[1][C1 + 1], wz = e.W[2][C2 + 1];
    const double wyz = wy * wz;
    return e.s * (e.U * wx * wyz + e.k[0][C0 + 1] * wyz + wx * (e.k[1][C1 + 1] * wz + wy * e.k[2][C2 + 1]));
}

// Node state of an equilibrium (sections 4.1-4.4), one LDS column per node:
// density, temperature, mixture theta, internal energy, velocity, mass
// fractions.
constexpr int ST_RHO = 0, ST_T = 1, ST_TH = 2, ST_U = 3, ST_V = 4, ST_Y = 7;

template <int M>
__device__ __forceinline__ void state_store(MechC mc0, double (*st)[BC_NODES], int lane, double rho, const double* u,
                                            const double* Y, double T) {
    reload_barrier();
    MechC mc = in_loop(mc0);
    st[ST_RHO][lane] = rho;
    st[ST_T][lane] = T;
    st[ST_TH][lane] = mc.R_univ * mix_inv_m<M>(mc, Y) * T;
    st[ST_U][lane] = mix_U<M>(mc, Y, T);
#pragma unroll
    for (int d = 0; d < 3; ++d) st[ST_V + d][lane] = u[d];
#pragma unroll
    for (int c = 0; c < M; ++c) st[ST_Y + c][lane] = Y[c];
}

// Equilibrium factors of stored lattice l (the wave's) for the state in
// column `lane` of st; a species lattice takes the velocity w (its own in
// the wall's local state, eq. locua), the others the mixture velocity.
template <int M, int W>
__device__ __forceinline__ void lat_prepare(MechC mc0, const double (*st)[BC_NODES], int lane, int l, int slaved,
                                            bool spv, const double (&w)[3], LatEq& q) {
    constexpr int LF = Lat<M, W>::LF, LG = Lat<M, W>::LG;
    reload_barrier();
    MechC mc = in_loop(mc0);
    const bool lg = l == LG, sp = l < LF;
    const int a = sp ? (W ? l : l + (l >= slaved ? 1 : 0)) : 0;
    const double rho = st[ST_RHO][lane];
    const double th = sp ? mc.Ra[a] * st[ST_T][lane] : st[ST_TH][lane];
    q.s = sp ? rho * st[ST_Y + a][lane] : rho;
    q.U = lg ? st[ST_U][lane] : 1.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) eq_axis(sp && spv ? w[d] : st[ST_V + d][lane], th, lg, q.W[d], q.k[d]);
}

// Compile-time loop over the 27 velocities.
template <int I, typename F>
__device__ __forceinline__ void for_q(F&& f) {
    if constexpr (I < Q) {
        f(std::integral_constant<int, I>{});
        for_q<I + 1>(f);
    }
}

template <int M, int W>
constexpr int bc_threads() { return BC_NODES * Lat<M, W>::NL; }

// How many of a block's lattices keep their advected populations (27 * 64
// stored values each) in LDS beside the node states and moments, within the
// 160 KB of LDS per CU on gfx950.
template <int M, typename S, int W>
constexpr int bc_stash() {
    constexpr int NL = Lat<M, W>::NL;
    constexpr long state = (long)(NL * 4 + 3 * (ST_Y + M)) * BC_NODES * (long)sizeof(double) + BC_NODES * 4L;
    constexpr long n = (160L * 1024 - state) / ((long)Q * BC_NODES * (long)sizeof(S));
    return n < 0 ? 0 : (n < NL ? (int)n : NL);
}

template <int M, typename S, int W>
__global__ __launch_bounds__((bc_threads<M, W>())) void k_boundary(
    const LatDev* __restrict__ lats, const int* __restrict__ blk, int n_lat, const long long* __restrict__ tp,
    long long toff) {
    constexpr int LF = Lat<M, W>::LF, LG = Lat<M, W>::LG, NL = Lat<M, W>::NL;
    __shared__ double mom[NL][4][BC_NODES];             // moments per lattice and node
    __shared__ double stA[ST_Y + M][BC_NODES];          // imposed state
    __shared__ double stL[ST_Y + M][BC_NODES];          // local state
    __shared__ double stT[ST_Y + M][BC_NODES];          // the full inlet's target
    __shared__ int flg[BC_NODES];
    // the advected populations of the first NS lattices as stored, loaded
    // once and read by all three passes (NS = NL where they fit beside the
    // state; one block per CU runs anyway, as the kernel's registers allow no
    // second one)
    constexpr int NS = bc_stash<M, S, W>();
    __shared__ S stash[NS > 0 ? NS : 1][Q][BC_NODES];
    const long long t = step_time(tp, toff);
    // tiles in reverse list order, without the XCD remap: the list is sorted
    // by boundary type and starts with the TMS walls (the cheapest entries),
    // so the costlier inlet, outlet and bounce-back tiles start first and
    // wall tiles fill the tail; and consecutive tiles go to different XCDs,
    // so every XCD gets a share of each kind (L2 sharing between neighbouring
    // tiles matters little here)
    const int b = (int)(gridDim.x - 1 - blockIdx.x);
    const int lj = find_lattice(blk, n_lat, b);
    const LatDev& L = lats[lj];
    if (t >= L.t_end) return;                       // the whole block
    const int lane = (int)threadIdx.x % BC_NODES;
    const int l = __builtin_amdgcn_readfirstlane((int)threadIdx.x / BC_NODES);   // this wave's lattice
    const int k = (b - blk[lj]) * BC_NODES + lane;
    const bool live = k < L.n_if;
    const int kk = live ? k : 0;                    // nodes past the end mirror entry 0 and write nothing
    MechC mc0 = *as_const(L.mech);
    const int par = (L.parity0 + t) & 1;
    const RLBM_GLOBAL S* src = as_global(static_cast<const S*>(L.pop[par]));
    // the output: interface slot N + k of every plane of the same buffer,
    // disjoint from the node slots the pull reads
    RLBM_GLOBAL S* bc = as_global(static_cast<S*>(L.pop[par])) + L.N;
    const size_t N = (size_t)L.N;
    const size_t P = (size_t)L.P;
    const int node = L.if_node[kk];
    const unsigned Dm = L.if_mask[kk];
    const int type = L.if_type[kk];
    const int s = W ? M : L.slaved;
    const int x = node % L.nx, r = node / L.nx, y = r % L.ny, z = r / L.ny;
    PullOff o;
    pull_offsets(L, x, y, z, o);
    const bool wall = type == RLBM_FACE_WALL;
    const bool bback = type == RLBM_FACE_BOUNCEBACK;
    const bool outlet = type == RLBM_FACE_OUTLET;
    const bool inlet_full = type == RLBM_FACE_INLET;
    const RLBM_CONST double* G = as_const(L.ref);
    const double zero3[3] = {0.0, 0.0, 0.0};
    if (l == 0) flg[lane] = 0;

    // FP32 deviation storage: references belong to the node that reads a
    // value, this node for an advected value and for what is written to the
    // boundary buffer, the pull source x - c_i (wrapped) for a bounce-back
    // source f'_{opp(i)}(x)
    float sl = 0.0f, sf = 0.0f;
    if constexpr (sizeof(S) == 4) {
        const RLBM_GLOBAL float* sc = scale_at(L, par, node);
        sl = sc[l];
        sf = sc[LF];
    }
    // population (l, i) after advection, or with bb on an incoming link the
    // bounce-back source (every lattice at a bounce-back wall, species and
    // momentum at a TMS wall)
    auto pop = [&](auto ic, bool bb) -> double {
        constexpr int i = decltype(ic)::value;
        constexpr int c0 = cx_of(i), c1 = cy_of(i), c2 = cz_of(i), io = Q - 1 - i;
        const int off = node + sel3(c0, o.x[0], 0, o.x[2]) + sel3(c1, o.y[0], 0, o.y[2]) + sel3(c2, o.z[0], 0, o.z[2]);
        double v;
        if (bb && ((Dm >> i) & 1u)) {
            v = (double)ld_at(src + (size_t)(l * Q + io) * P, node);
            if constexpr (sizeof(S) == 4) {
                const RLBM_GLOBAL float* sc = scale_at(L, par, off);
                const float sb = sc[l], sfb = sc[LF];
                v += l == LG ? ref_g(sb, sfb, G[l * Q + io], G[REF_K<NL> + io]) : ref_of(sb, G[l * Q + io]);
            }
        } else {
            v = (double)ld_at(src + (size_t)(l * Q + i) * P, off);
            if constexpr (sizeof(S) == 4)
                v += l == LG ? ref_g(sl, sf, G[l * Q + i], G[REF_K<NL> + i]) : ref_of(sl, G[l * Q + i]);
        }
        return v;
    };
    const bool stashed = NS == NL || l < NS;   // wave-uniform
    // the advected population (l, i), from the stash where there is one
    auto adv = [&](auto ic) -> double {
        if (NS > 0 && stashed) {
            constexpr int i = decltype(ic)::value;
            double v = (double)stash[l][i][lane];
            if constexpr (sizeof(S) == 4)
                v += l == LG ? ref_g(sl, sf, G[l * Q + i], G[REF_K<NL> + i]) : ref_of(sl, G[l * Q + i]);
            return v;
        } else {
            return pop(ic, false);
        }
    };
    auto put = [&](auto ic, double v) {
        constexpr int i = decltype(ic)::value;
        if (!live) return;
        RLBM_GLOBAL S* pl = bc + (size_t)(l * Q + i) * P;
        if constexpr (sizeof(S) == 4) {
            const double ref = l == LG ? ref_g(sl, sf, G[l * Q + i], G[REF_K<NL> + i]) : ref_of(sl, G[l * Q + i]);
            st_at(pl, k, __double2float_rn(v - ref));
        } else {
            st_at(pl, k, v);
        }
    };

    // step 1.  Bounce-back wall (section 4.2.1, eq. bb): incoming links carry
    // the opposite population of the same node, outgoing links their own.
    // TMS wall (section 4.2.2): the bounce-back densities (eqs. BBrho, BBY),
    // zeroth moments with the bounce-back sources on D.
    if (bback) {
        for_q<0>([&](auto ic) { put(ic, pop(ic, true)); });
    } else if (NS > 0 && stashed) {
        // one pass of loads, every one issued before the first store to LDS:
        // the advected populations of outgoing links and, at a TMS wall, the
        // bounce-back sources of incoming ones (species and momentum); any
        // other incoming link loads this node's own slot, an in-range
        // stand-in that no pass reads
        const bool tms = wall && l <= LF;
        S raw[Q];
        float sbv[Q];
        for_q<0>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int c0 = cx_of(i), c1 = cy_of(i), c2 = cz_of(i), io = Q - 1 - i;
            const int off = node + sel3(c0, o.x[0], 0, o.x[2]) + sel3(c1, o.y[0], 0, o.y[2]) +
                            sel3(c2, o.z[0], 0, o.z[2]);
            const bool in = (Dm >> i) & 1u;
            const RLBM_GLOBAL S* pi = src + (size_t)(l * Q + i) * P;
            const RLBM_GLOBAL S* pio = src + (size_t)(l * Q + io) * P;
            raw[i] = ld_at(tms && in ? pio : pi, in ? node : off);
            if constexpr (sizeof(S) == 4) {
                sbv[i] = 0.0f;
                if (tms && in) sbv[i] = scale_at(L, par, off)[l];   // the reader's scale
            }
        });
        for_q<0>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            stash[l][i][lane] = raw[i];
        });
        if (tms) {
            // TMS wall (section 4.2.2): the bounce-back densities (eqs.
            // BBrho, BBY), zeroth moments with the bounce-back sources on D
            double m0 = 0.0;
            for_q<0>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int io = Q - 1 - i;
                double v = (double)raw[i];
                if constexpr (sizeof(S) == 4)
                    v += ((Dm >> i) & 1u) ? ref_of(sbv[i], G[l * Q + io]) : ref_of(sl, G[l * Q + i]);
                m0 += v;
            });
            mom[l][0][lane] = m0;
        }
    } else if (wall && l <= LF) {
        double m0 = 0.0;
        for_q<0>([&](auto ic) { m0 += pop(ic, true); });
        mom[l][0][lane] = m0;
    }
    __syncthreads();
    // step 2: the imposed state, formed by the first wave: the TMS target
    // (u = 0, T_w(x)), the LODI outlet state (section 4.4, from the previous
    // outlet state and the previous post-boundary moments of the first
    // interior node), or the inlet equilibrium (section 4.3, eqs. in_f, in_g,
    // in_fa)
    if (l == 0 && !bback) {
        double Y[M], u[3] = {0.0, 0.0, 0.0}, rho, T;
        if (wall) {
            double rs = 0.0;
            const double rb = mom[LF][0][lane];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const bool slv = !W && c == s;
                const double v = slv ? 0.0 : mom[slv ? 0 : (W ? c : c - (c > s ? 1 : 0))][0][lane];
                Y[c] = v;
                rs += v;
            }
            if constexpr (!W) {
#pragma unroll
                for (int c = 0; c < M; ++c)
                    if (c == s) Y[c] = rb - rs;
            }
            const double iry = 1.0 / (W ? rs : rb);   // the weakly coupled storage normalises Y by sum_a rho_a
#pragma unroll
            for (int c = 0; c < M; ++c) Y[c] *= iry;
            rho = rb;
            T = L.if_T[kk];
        } else if (outlet) {
            reload_barrier();
            MechC mc = in_loop(mc0);
            const int ko = L.if_out[kk];
            const size_t No = (size_t)L.n_out;
            double* os = L.out_state;
            const double rho0 = os[0 * No + ko];
            const double u0[3] = {os[1 * No + ko], os[2 * No + ko], os[3 * No + ko]};
            const double T0 = os[4 * No + ko];
            double Y0[M], Y1[M];
            const size_t inn = (size_t)node - 1;
#pragma unroll
            for (int c = 0; c < M; ++c) {
                Y0[c] = os[(5 + c) * No + ko];
                Y1[c] = L.aux[(AUX_Y + c) * N + inn];
            }
            const double rho1 = L.aux[AUX_RHO * N + inn];
            const double u1[3] = {L.aux[(AUX_U + 0) * N + inn], L.aux[(AUX_U + 1) * N + inn],
                                  L.aux[(AUX_U + 2) * N + inn]};
            const double T1 = L.aux[AUX_T * N + inn];
            const double R0 = mc.R_univ * mix_inv_m<M>(mc, Y0);
            const double P0 = rho0 * R0 * T0;
            const double P1 = rho1 * mc.R_univ * mix_inv_m<M>(mc, Y1) * T1;
            double Cv = 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) Cv += Y0[c] * species_cv(mc, c, T0);
            const double gam = (Cv + R0) / Cv;
            const double cs = sqrt(gam * P0 / rho0);
            const double un = u0[0];
            const double Ma = un / cs;
            const double L1 = L.sigma * (1.0 - Ma * Ma) * cs / (double)L.nx * (P0 - L.P_inf);
            const double L2 = un * (cs * cs * (rho0 - rho1) - (P0 - P1));
            const double L3 = un * (u0[1] - u1[1]);
            const double L4 = un * (u0[2] - u1[2]);
            const double L5 = (un + cs) * ((P0 - P1) + rho0 * cs * (u0[0] - u1[0]));
            rho = rho0 - (L2 + 0.5 * (L5 + L1)) / (cs * cs);
            const double P_o = P0 - 0.5 * (L5 + L1);
            u[0] = un - (L5 - L1) / (2.0 * rho0 * cs);
            u[1] = u0[1] - L3;
            u[2] = u0[2] - L4;
#pragma unroll
            for (int c = 0; c < M; ++c) Y[c] = Y0[c] - un * (Y0[c] - Y1[c]);   // eq. convectiveBC
            T = P_o / (rho * mc.R_univ * mix_inv_m<M>(mc, Y));
            if (live) {
                os[0 * No + ko] = rho;
                os[1 * No + ko] = u[0]; os[2 * No + ko] = u[1]; os[3 * No + ko] = u[2];
                os[4 * No + ko] = T;
#pragma unroll
                for (int c = 0; c < M; ++c) os[(5 + c) * No + ko] = Y[c];
            }
        } else {
            rho = L.rho_in;
            u[0] = L.u_in;
#pragma unroll
            for (int c = 0; c < M; ++c) Y[c] = L.Y_in[c];
            T = L.T_in;
        }
        state_store<M>(mc0, stA, lane, rho, u, Y, T);
    }
    __syncthreads();
    // step 3: moments of the mixed set, incoming links at the imposed
    // equilibria and outgoing ones advected (eqs. locRho .. locT and their
    // inlet and outlet counterparts)
    LatEq eA;
    if (!bback) {
        lat_prepare<M, W>(mc0, stA, lane, l, s, false, zero3, eA);
        double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
        for_q<0>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int c0 = cx_of(i), c1 = cy_of(i), c2 = cz_of(i);
            double v;
            if ((Dm >> i) & 1u) v = lat_eq<c0, c1, c2>(eA);
            else v = adv(ic);
            m0 += v;
            if (c0) m1 += c0 > 0 ? v : -v;
            if (c1) m2 += c1 > 0 ? v : -v;
            if (c2) m3 += c2 > 0 ? v : -v;
        });
        mom[l][0][lane] = m0; mom[l][1][lane] = m1; mom[l][2][lane] = m2; mom[l][3][lane] = m3;
    }
    __syncthreads();
    // the local state (first wave): rho and u from the momentum lattice, the
    // species densities (the slaved one by difference, eq. strongest), T by
    // Newton on the energy lattice's internal energy from the imposed T; and
    // the full inlet's target, the local density and composition at the
    // imposed u^in and T^in (eqs. in_tgt_*)
    if (l == 0 && !bback) {
        double Y[M], u[3];
        const double rl = mom[LF][0][lane];
        double rs = rl, ry = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const bool slv = !W && c == s;
            const double v = slv ? 0.0 : mom[slv ? 0 : (W ? c : c - (c > s ? 1 : 0))][0][lane];
            Y[c] = v;
            rs -= v;
            ry += v;
        }
        if constexpr (!W) {
#pragma unroll
            for (int c = 0; c < M; ++c)
                if (c == s) Y[c] = rs;
        }
        const double iry = 1.0 / (W ? ry : rl), irl = 1.0 / rl;   // weakly coupled: Y by sum_a rho_a
#pragma unroll
        for (int c = 0; c < M; ++c) Y[c] *= iry;
#pragma unroll
        for (int d = 0; d < 3; ++d) u[d] = mom[LF][1 + d][lane] * irl;
        const double Ul = mom[LG][0][lane] * irl - 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        int fail = 0;
        reload_barrier();
        const double Tl = solve_T<M>(in_loop(mc0), Y, Ul, stA[ST_T][lane], &fail);
        flg[lane] = fail;
        state_store<M>(mc0, stL, lane, rl, u, Y, Tl);
        if (inlet_full) {
            const double uin[3] = {L.u_in, 0.0, 0.0};
            state_store<M>(mc0, stT, lane, rl, uin, Y, L.T_in);
        }
    }
    __syncthreads();
    // step 4: reconstruction of this wave's lattice
    if (!bback) {
        // the wall's local species equilibria take the species' own velocity
        // u_a = j_a / rho_a (u where rho_a <= 1e-14 rho, eq. locua)
        double w[3] = {0.0, 0.0, 0.0};
        const bool spv = wall && l < LF;
        if (spv) {
            const double ra = mom[l][0][lane];
            const bool small = ra <= 1e-14 * stL[ST_RHO][lane];
            const double ir = small ? 0.0 : 1.0 / ra;
#pragma unroll
            for (int d = 0; d < 3; ++d) w[d] = small ? stL[ST_V + d][lane] : mom[l][1 + d][lane] * ir;
        }
        LatEq eL;
        lat_prepare<M, W>(mc0, stL, lane, l, s, spv, w, eL);
        if (type == RLBM_FACE_INLET_LOCAL) {
            // the simplified inlet: every population at the local equilibria
            // (eqs. in_loc_*)
            for_q<0>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                put(ic, lat_eq<cx_of(i), cy_of(i), cz_of(i)>(eL));
            });
        } else if (inlet_full) {
            // eqs. f_inlet, g_inlet, fa_inlet
            LatEq eT;
            lat_prepare<M, W>(mc0, stT, lane, l, s, false, zero3, eT);
            for_q<0>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int c0 = cx_of(i), c1 = cy_of(i), c2 = cz_of(i);
                double fi;
                if ((Dm >> i) & 1u) fi = lat_eq<c0, c1, c2>(eA);
                else fi = adv(ic);
                put(ic, lat_eq<c0, c1, c2>(eT) + fi - lat_eq<c0, c1, c2>(eL));
            });
        } else {
            // TMS wall (eqs. ftms, gtms, fatms) and outlet (eqs. f_outlet,
            // g_outlet, fa_outlet): 2 A - loc on incoming links, A + f - loc
            // on outgoing ones
            for_q<0>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int c0 = cx_of(i), c1 = cy_of(i), c2 = cz_of(i);
                const double ea = lat_eq<c0, c1, c2>(eA), el = lat_eq<c0, c1, c2>(eL);
                double fi;
                if ((Dm >> i) & 1u) fi = ea;
                else fi = adv(ic);
                put(ic, ea + fi - el);
            });
        }
    }
    if (l == 0 && live && flg[lane]) atomicOr(L.flag, 1);
}

// ---------------------------------------------------------------------------
// initial state, read-out, populations I/O, invariants
// ---------------------------------------------------------------------------
// Node that pulls the population stored at slot (node, i): node + c_i,
// wrapped on every axis (the placeholder rule of the pull offsets).
__device__ __forceinline__ long long reader_of(const LatDev& L, long long node, int i) {
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int x = (int)(node % nx);
    const long long r = node / nx;
    const int y = (int)(r % ny), z = (int)(r / ny);
    const int xr = (x + cx_of(i) + nx) % nx, yr = (y + cy_of(i) + ny) % ny, zr = (z + cz_of(i) + nz) % nz;
    return ((long long)zr * ny + yr) * nx + xr;
}

// Reference value of slot (node, i) of lattice l in buffer q (FP32 storage).
template <int M, typename S, int W>
__device__ __forceinline__ double slot_ref(const LatDev& L, int q, long long node, int l, int i) {
    if constexpr (sizeof(S) == 8) {
        return 0.0;
    } else {
        constexpr int LF = Lat<M, W>::LF, LG = Lat<M, W>::LG, NL = Lat<M, W>::NL;
        const RLBM_CONST double* G = as_const(L.ref);
        const RLBM_GLOBAL float* sc = scale_at(L, q, reader_of(L, node, i));
        if (l == LG) return ref_g(sc[LG], sc[LF], G[l * Q + i], G[REF_K<NL> + i]);
        return ref_of(sc[l], G[l * Q + i]);
    }
}

// Reference scales of the initial populations: the zeroth moments rho_a of
// the stored species, rho and rho E.
template <int M, int W>
__global__ __launch_bounds__(256) void k_scale_init(const LatDev* __restrict__ lat, const double* __restrict__ rho_in,
                                                    const double* __restrict__ u_in, const double* __restrict__ T_in,
                                                    const double* __restrict__ Y_in) {
    const LatDev& L = *lat;
    const long long node = (long long)blockIdx.x * 256 + threadIdx.x;
    if (node >= L.N) return;
    MechC mc = *as_const(L.mech);
    const size_t N = (size_t)L.N;
    constexpr int NSP = Lat<M, W>::NSP, LF = Lat<M, W>::LF, LG = Lat<M, W>::LG;
    const int s = W ? M : L.slaved;
    const double rho = rho_in[node];
    float* so = L.rscale[L.parity0] + (size_t)node * L.rss;
    double Y[M];
#pragma unroll
    for (int a = 0; a < M; ++a) Y[a] = Y_in[a * N + node];
    for (int l = 0; l < NSP; ++l) {
        const int a = W ? l : l + (l >= s ? 1 : 0);
        so[l] = __double2float_rn(rho * Y_in[a * N + node]);
    }
    so[LF] = __double2float_rn(rho);
    double usq = 0.0;
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) usq += u_in[dd * N + node] * u_in[dd * N + node];
    so[LG] = __double2float_rn(rho * (mix_U<M>(mc, Y, T_in[node]) + 0.5 * usq));
}

template <int M, typename S, int W>
__global__ __launch_bounds__(256) void k_init(const LatDev* __restrict__ lat, const double* __restrict__ rho_in,
                                              const double* __restrict__ u_in, const double* __restrict__ T_in,
                                              const double* __restrict__ Y_in) {
    const LatDev& L = *lat;
    const long long node = (long long)blockIdx.x * 256 + threadIdx.x;
    if (node >= L.N) return;
    MechC mc = *as_const(L.mech);
    const size_t N = (size_t)L.N;
    void* dst = L.pop[L.parity0];
    EqState<M, false> e;
    e.rho = rho_in[node];
    const double T = T_in[node];
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) e.u[dd] = u_in[dd * N + node];
#pragma unroll
    for (int a = 0; a < M; ++a) e.Y[a] = Y_in[a * N + node];
    eq_prepare<M, false>(mc, e, T);
    for (int l = 0; l < Lat<M, W>::NL; ++l)
        for (int i = 0; i < Q; ++i) {
            const int li = l * Q + i;
            Codec<S>::st(dst, (size_t)li * L.P + node, eq_value<M, W, false>(mc, e, l, L.slaved, i),
                         slot_ref<M, S, W>(L, L.parity0, node, l, i));
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

// Reference shapes for FP32 deviation storage (one block): for the stored
// species, the momentum lattice and the energy lattice's internal-energy part
// the zero-velocity equilibrium shape (unit zeroth moment) at the
// domain-mean temperature and composition, and the energy lattice's theta^2
// part K (eq. geq_i at u = 0 with rho = 1, U = 0); then the zeroth moments,
// the momentum shape's sum_i G c_x^2 and sum_i K_i.
template <int M, int W>
__global__ __launch_bounds__(512) void k_refs(const LatDev* __restrict__ lat, double* __restrict__ ref, double rho,
                                              double T, const double* __restrict__ Y) {
    constexpr int NSP = Lat<M, W>::NSP, LF = Lat<M, W>::LF, LG = Lat<M, W>::LG, NL = Lat<M, W>::NL;
    static_assert(NL * Q <= 512, "one thread per reference shape value");
    (void)rho;
    const LatDev& L = *lat;
    const int li = threadIdx.x;
    MechC mc = *as_const(L.mech);
    const double th_mix = mc.R_univ * mix_inv_m<M>(mc, Y) * T;
    if (li < NL * Q) {
        const int l = li / Q, i = li % Q;
        const int c0 = cx_of(i), c1 = cy_of(i), c2 = cz_of(i);
        double th = th_mix;
        if (l < NSP) th = mc.Ra[W ? l : l + (l >= L.slaved ? 1 : 0)] * T;
        // shapes are rounded to FP32 values (see ref_of)
        ref[li] = (double)(float)(psi(c0, 0.0, th) * psi(c1, 0.0, th) * psi(c2, 0.0, th));
        if (l == LG) {
            const double Wx = psi(c0, 0.0, th), Wy = psi(c1, 0.0, th), Wz = psi(c2, 0.0, th);
            const double k0 = -th * th, k1 = 0.5 * th * th;
            const double kx = c0 ? k1 : k0, ky = c1 ? k1 : k0, kz = c2 ? k1 : k0;
            ref[REF_K<NL> + i] = (double)(float)(kx * Wy * Wz + Wx * (ky * Wz + Wy * kz));
        }
    }
    __syncthreads();
    if (li < NL) {
        double m0 = 0.0;
        for (int i = 0; i < Q; ++i) m0 += ref[li * Q + i];
        ref[REF_M0<NL> + li] = m0;
    } else if (li == NL) {
        double m2 = 0.0;
        for (int i = 0; i < Q; ++i) m2 += ref[LF * Q + i] * (double)(cx_of(i) * cx_of(i));
        ref[REF_M2<NL>] = m2;
    } else if (li == NL + 1) {
        double k0 = 0.0;
        for (int i = 0; i < Q; ++i) k0 += ref[REF_K<NL> + i];
        ref[REF_K0<NL>] = k0;
    }
}

template <int M, typename S, int W>
__global__ __launch_bounds__(256) void k_fields(const LatDev* __restrict__ lat, long long t, double* rho_o,
                                                double* u_o, double* T_o, double* Y_o, double* P_o) {
    const LatDev& L = *lat;
    const long long node = (long long)blockIdx.x * 256 + threadIdx.x;
    if (node >= L.N) return;
    MechC mc = *as_const(L.mech);
    const size_t N = (size_t)L.N;
    const int q = (L.parity0 + t) & 1;
    const void* src = L.pop[q];
    constexpr int LF = Lat<M, W>::LF, LG = Lat<M, W>::LG;
    const int s = W ? M : L.slaved;
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, rE = 0.0, ra[M];
    for (int i = 0; i < Q; ++i) {
        const double f = Codec<S>::ld(src, (size_t)(LF * Q + i) * L.P + node, slot_ref<M, S, W>(L, q, node, LF, i));
        rho += f; j[0] += f * cx_of(i); j[1] += f * cy_of(i); j[2] += f * cz_of(i);
        rE += Codec<S>::ld(src, (size_t)(LG * Q + i) * L.P + node, slot_ref<M, S, W>(L, q, node, LG, i));
    }
    double rs = rho;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        ra[a] = 0.0;
        if (a == s) continue;
        const int l = lat_of(a, s);
        for (int i = 0; i < Q; ++i)
            ra[a] += Codec<S>::ld(src, (size_t)(l * Q + i) * L.P + node, slot_ref<M, S, W>(L, q, node, l, i));
        rs -= ra[a];
    }
#pragma unroll
    for (int a = 0; a < M; ++a)
        if (a == s) ra[a] = rs;
    double ry = rho;   // the weakly coupled storage normalises Y by sum_a rho_a
    if constexpr (W) {
        ry = 0.0;
#pragma unroll
        for (int a = 0; a < M; ++a) ry += ra[a];
    }
    double Y[M];
#pragma unroll
    for (int a = 0; a < M; ++a) Y[a] = ra[a] / ry;
    const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    const double U = rE / rho - 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    int fail = 0;
    const double T = solve_T<M>(mc, Y, U, L.aux[AUX_T * N + node], &fail);
    if (fail) atomicOr(L.flag, 1);
    if (rho_o) rho_o[node] = rho;
    if (u_o)
        for (int dd = 0; dd < 3; ++dd) u_o[dd * N + node] = u[dd];
    if (T_o) T_o[node] = T;
    if (Y_o)
#pragma unroll
        for (int a = 0; a < M; ++a) Y_o[a * N + node] = Y[a];
    if (P_o) P_o[node] = rho * mc.R_univ * mix_inv_m<M>(mc, Y) * T;
}

// FP64 copies of the stored lattices l0 .. l0 + nl - 1 from (write = 0) or
// into (write = 1) the current population buffer; buf holds [nl][27][N].
template <int M, typename S, int W>
__global__ __launch_bounds__(256) void k_pops(const LatDev* __restrict__ lat, long long t, int l0, int nl,
                                              double* buf, int write) {
    const LatDev& L = *lat;
    const size_t total = (size_t)nl * Q * L.N;
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const size_t gidx = (size_t)l0 * Q * L.N + idx;   // in the packed [L][27][N] order
    const int li = (int)(gidx / L.N);
    const long long node = (long long)(gidx % L.N);
    const size_t pidx = (size_t)li * L.P + node;      // in the buffer's planes
    const int q = (L.parity0 + t) & 1;
    void* p = L.pop[q];
    const double ref = slot_ref<M, S, W>(L, q, node, li / Q, li % Q);
    if (write) Codec<S>::st(p, pidx, buf[idx], ref);
    else buf[idx] = Codec<S>::ld(p, pidx, ref);
}

// Per-block partial sums of the invariants; nv = 6 + E values per block.
template <int M, typename S, int W>
__global__ __launch_bounds__(256) void k_invariants(const LatDev* __restrict__ lat, long long t,
                                                    double* __restrict__ partial, int nv) {
    const LatDev& L = *lat;
    MechC mc = *as_const(L.mech);
    const long long node = (long long)blockIdx.x * 256 + threadIdx.x;
    const size_t N = (size_t)L.N;
    constexpr int LF = Lat<M, W>::LF, LG = Lat<M, W>::LG;
    const int s = W ? M : L.slaved;
    double v[6 + MAXE];
    for (int q = 0; q < 6 + MAXE; ++q) v[q] = 0.0;
    if (node < L.N) {
        const int q = (L.parity0 + t) & 1;
        const void* src = L.pop[q];
        double bad = 0.0;
        double rho = 0.0;
        for (int i = 0; i < Q; ++i) {
            const double f =
                Codec<S>::ld(src, (size_t)(LF * Q + i) * L.P + node, slot_ref<M, S, W>(L, q, node, LF, i));
            const double g = Codec<S>::ld(src, (size_t)(LG * Q + i) * L.P + node, slot_ref<M, S, W>(L, q, node, LG, i));
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
            const int l = lat_of(a, s);
            for (int i = 0; i < Q; ++i) {
                const double f = Codec<S>::ld(src, (size_t)(l * Q + i) * L.P + node, slot_ref<M, S, W>(L, q, node, l, i));
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

// Advances the device step counter of a launch series by n (the last node
// of a captured chunk of batched steps).
__global__ void k_advance_time(long long* __restrict__ tp, long long n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *tp += n;
}

// Reads and clears the failure flags of k lattices: out[j] = *flags[j].
__global__ __launch_bounds__(256) void k_gather_flags(int* const* __restrict__ flags, int k, int* __restrict__ out) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < k) out[j] = atomicExch(flags[j], 0);
}

hipError_t launch_advance_time(long long* tp, long long n, hipStream_t st) {
    (void)hipGetLastError();   // report this launch's error only
    hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(64), 0, st, tp, n);
    return hipGetLastError();
}

hipError_t launch_gather_flags(int* const* flags, int k, int* out, hipStream_t st) {
    (void)hipGetLastError();   // report this launch's error only
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_flags, dim3((k + 255) / 256), dim3(256), 0, st, flags, k, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// allocation-free group steps: tables in a file-scope device array
// ---------------------------------------------------------------------------
// Each GPU holds its own copy until the process ends.  Host code never
// names it: it uses the device address that group_scratch() returns.
static __device__ __align__(256) unsigned char scratch[GROUP_SCRATCH_BYTES];

hipError_t group_scratch(int device, char** ptr) {
    // one address per device, looked up once with that device current
    static std::mutex mu;
    static char* addr[64] = {};
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = (char*)p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

// Entries base .. base + n - 1 of the group table: block j copies lattice
// j's device entry word by word, then sets its buffer parity and step
// count; block 0 writes the block prefixes of those entries (and of the
// entry after the last), and resets the step counter on the first chunk.
__global__ __launch_bounds__(64) void k_group_gather(char* __restrict__ sc, GroupChunk c) {
    const int j = blockIdx.x;
    LatDev* table = (LatDev*)(sc + GROUP_OFF_TABLE);
    int* blk = (int*)(sc + GROUP_OFF_BLK);
    static_assert(sizeof(LatDev) % 8 == 0, "the entry is copied in 8-byte words");
    const unsigned long long* src = (const unsigned long long*)c.src[j];
    unsigned long long* dst = (unsigned long long*)&table[c.base + j];
    for (int w = threadIdx.x; w < (int)(sizeof(LatDev) / 8); w += 64) dst[w] = src[w];
    __syncthreads();
    if (threadIdx.x == 0) {
        table[c.base + j].parity0 = c.parity[j];
        table[c.base + j].t_end = c.t_end[j];
    }
    if (j == 0) {
        for (int q = threadIdx.x; q < 3 * (c.n + 1); q += 64) {
            const int a = q / (c.n + 1), e = q % (c.n + 1);
            blk[a * (c.k + 1) + c.base + e] = c.blk[a][e];
        }
        if (c.base == 0 && threadIdx.x == 0) *(long long*)sc = 0;
    }
}

hipError_t launch_group_gather(char* sc, const GroupChunk& c, hipStream_t st) {
    (void)hipGetLastError();   // report this launch's error only
    if (c.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_group_gather, dim3(c.n), dim3(64), 0, st, sc, c);
    return hipGetLastError();
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
// species count and storage coupling (WW = 1: weakly coupled, all M species stored)
#define RLBM_DISPATCH_W(M_, W_, ...)                                                   \
    if (W_) {                                                                          \
        constexpr int WW = 1;                                                          \
        RLBM_DISPATCH(M_, __VA_ARGS__)                                                 \
    } else {                                                                           \
        constexpr int WW = 0;                                                          \
        RLBM_DISPATCH(M_, __VA_ARGS__)                                                 \
    }

template <typename S>
static hipError_t launch_step_phase(int phase, int M, int weak, const StepLaunch& a) {
    if (a.blocks <= 0) return hipSuccess;
    (void)hipGetLastError();   // report this launch's error only
    if (phase == 0) {
        RLBM_DISPATCH_W(M, weak, hipLaunchKernelGGL((k_boundary<MM, S, WW>), dim3(a.blocks), dim3(bc_threads<MM, WW>()), 0,
                                                    a.stream, a.lats, a.blk, a.n_lat, a.tp, a.toff))
    } else if (phase == 1) {
        RLBM_DISPATCH_W(M, weak, hipLaunchKernelGGL((k_local<MM, S, WW>), dim3(a.blocks), dim3(NODE_TILE), 0, a.stream,
                                                    a.lats, a.blk, a.n_lat, a.tp, a.toff))
    } else if (phase == 2) {
        if (a.schemes & (1u << RLBM_REACTION_EXPLICIT))
            RLBM_DISPATCH(M, hipLaunchKernelGGL((k_gradients<MM>), dim3((a.blocks + GRAD_TILES - 1) / GRAD_TILES), dim3(GRAD_TILES * NODE_TILE), 0, a.stream, a.lats,
                                                    a.blk, a.n_lat, a.tp, a.toff))
        if (a.schemes & (1u << RLBM_REACTION_LINEARLY_IMPLICIT))
            RLBM_DISPATCH(M, hipLaunchKernelGGL((k_chem_implicit<MM>), dim3(a.blocks), dim3(NODE_TILE), 0, a.stream, a.lats,
                                                    a.blk, a.n_lat, a.tp, a.toff))
    } else {
        RLBM_DISPATCH_W(M, weak, hipLaunchKernelGGL((k_update<MM, S, WW>), dim3(a.blocks), dim3(UPD_THREADS), 0,
                                                    a.stream, a.lats, a.blk, a.n_lat, a.tp, a.toff))
    }
    return hipGetLastError();
}

hipError_t launch_phase(int phase, int M, int storage, int weak, const StepLaunch& a) {
    return storage == RLBM_STORAGE_F32_DEV ? launch_step_phase<float>(phase, M, weak, a)
                                           : launch_step_phase<double>(phase, M, weak, a);
}

template <typename S>
static hipError_t launch_init_t(int M, int weak, const LatDev* lat, long long N, const double* rho,
                                const double* u, const double* T, const double* Y, hipStream_t st) {
    (void)hipGetLastError();   // report this launch's error only
    const int blocks = (int)((N + 255) / 256);
    if constexpr (sizeof(S) == 4) {
        RLBM_DISPATCH_W(M, weak, hipLaunchKernelGGL((k_scale_init<MM, WW>), dim3(blocks), dim3(256), 0, st, lat, rho,
                                                    u, T, Y))
    }
    RLBM_DISPATCH_W(M, weak, hipLaunchKernelGGL((k_init<MM, S, WW>), dim3(blocks), dim3(256), 0, st, lat, rho, u,
                                                T, Y))
    return hipGetLastError();
}

hipError_t launch_init(int M, int storage, int weak, const LatDev* lat, long long N, const double* rho,
                       const double* u, const double* T, const double* Y, hipStream_t st) {
    return storage == RLBM_STORAGE_F32_DEV ? launch_init_t<float>(M, weak, lat, N, rho, u, T, Y, st)
                                           : launch_init_t<double>(M, weak, lat, N, rho, u, T, Y, st);
}

hipError_t launch_refs(int M, int weak, const LatDev* lat, double* ref, double rho, double T, const double* Y,
                       hipStream_t st) {
    (void)hipGetLastError();   // report this launch's error only
    RLBM_DISPATCH_W(M, weak, hipLaunchKernelGGL((k_refs<MM, WW>), dim3(1), dim3(512), 0, st, lat, ref, rho, T, Y))
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_fields_t(int M, int weak, const LatDev* lat, long long N, long long t, double* rho,
                                  double* u, double* T, double* Y, double* P, hipStream_t st) {
    (void)hipGetLastError();   // report this launch's error only
    const int blocks = (int)((N + 255) / 256);
    RLBM_DISPATCH_W(M, weak, hipLaunchKernelGGL((k_fields<MM, S, WW>), dim3(blocks), dim3(256), 0, st, lat, t, rho,
                                                u, T, Y, P))
    return hipGetLastError();
}

hipError_t launch_fields(int M, int storage, int weak, const LatDev* lat, long long N, long long t, double* rho,
                         double* u, double* T, double* Y, double* P, hipStream_t st) {
    return storage == RLBM_STORAGE_F32_DEV ? launch_fields_t<float>(M, weak, lat, N, t, rho, u, T, Y, P, st)
                                           : launch_fields_t<double>(M, weak, lat, N, t, rho, u, T, Y, P, st);
}

hipError_t launch_pops(int M, int storage, int weak, const LatDev* lat, long long N, int l0, int nl, long long t,
                       double* buf, int write, hipStream_t st) {
    (void)hipGetLastError();   // report this launch's error only
    const size_t total = (size_t)nl * Q * (size_t)N;
    const int blocks = (int)((total + 255) / 256);
    if (storage == RLBM_STORAGE_F32_DEV)
        RLBM_DISPATCH_W(M, weak, hipLaunchKernelGGL((k_pops<MM, float, WW>), dim3(blocks), dim3(256), 0, st, lat, t,
                                                    l0, nl, buf, write))
    else
        RLBM_DISPATCH_W(M, weak, hipLaunchKernelGGL((k_pops<MM, double, WW>), dim3(blocks), dim3(256), 0, st, lat, t,
                                                    l0, nl, buf, write))
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_inv_t(int M, int weak, const LatDev* lat, long long N, long long t, double* partial,
                               int nv, double* out, hipStream_t st) {
    (void)hipGetLastError();   // report this launch's error only
    const int blocks = (int)((N + 255) / 256);
    RLBM_DISPATCH_W(M, weak, hipLaunchKernelGGL((k_invariants<MM, S, WW>), dim3(blocks), dim3(256), 0, st, lat, t,
                                                partial, nv))
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(64), 0, st, partial, blocks, nv, out);
    return hipGetLastError();
}

hipError_t launch_invariants(int M, int storage, int weak, const LatDev* lat, long long N, long long t,
                             double* partial, int nv, double* out, hipStream_t st) {
    return storage == RLBM_STORAGE_F32_DEV ? launch_inv_t<float>(M, weak, lat, N, t, partial, nv, out, st)
                                           : launch_inv_t<double>(M, weak, lat, N, t, partial, nv, out, st);
}

bool species_supported(int M) { return M == 2 || M == 3 || M == 4 || M == 9; }

}  // namespace rlbm
