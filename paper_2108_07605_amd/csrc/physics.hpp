// Device-side physics of the reactive-mixture lattice Boltzmann step
// (Sawant, Dorschner & Karlin, arXiv 2108.07605).  FP64 throughout; the
// population storage format is decided in the kernels only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rlbm.h"

namespace rlbm {

constexpr int Q = 27;
constexpr int MAXM = RLBM_MAX_SPECIES;
constexpr int MAXR = RLBM_MAX_REACTIONS;
constexpr int MAXE = RLBM_MAX_ELEMENTS;
constexpr int MAXO = RLBM_MAX_ORDER;   // molecules per side of a reaction

// D3Q27 velocity i = 9 (cz + 1) + 3 (cy + 1) + (cx + 1) (section 2.2, eq. d3q27vel).
__host__ __device__ constexpr int cx_of(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy_of(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz_of(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int c2_of(int i) {
    return cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i) + cz_of(i) * cz_of(i);
}

// One reaction: Arrhenius parameters, reversibility, each side as a list of
// factors (its species in ascending order, each repeated by its coefficient:
// the mass-action product) and the net coefficients nu'' - nu'.
struct RxnDev {
    double lnA, beta, Ta, dnu_sum;
    int rev, nf, nr, pad_;
    int fac_f[MAXO], fac_r[MAXO];   // species per molecule; entries past nf / nr hold 0
    double dnu[MAXM];
};

// Mechanism in the layout the kernels read (uniform addresses: scalar loads).
struct MechDev {
    int M, R, E, pad_;
    double m[MAXM];             // molar masses
    double inv_m[MAXM];
    double Ra[MAXM];            // R_univ / m_a
    double uc[MAXM][6];         // U_a(T) = sum_k uc[a][k] T^k
    double cvc[MAXM][5];        // C_{a,v}(T) = sum_k cvc[a][k] T^k  (= dU_a/dT)
    double hc[MAXM][6];         // H_a(T) = sum_k hc[a][k] T^k
    double nasa[MAXM][7];       // raw NASA-7 coefficients (Gibbs functions)
    double R_univ, ln_cstd;
    // reactions, one contiguous record each (one scalar base per reaction)
    RxnDev rx[MAXR];
    // transport
    double T_ref, inv_T_ref, P_ref, inv_P_ref, mu_ref, mu_exp, inv_Pr, D_exp;
    double Kab[MAXM][MAXM];     // 1 / (D_ref[a][b] m_a m_b)
    double comp[MAXM][MAXE];    // element atoms per molecule (invariants)
};

// Per-lattice parameters (device resident, one entry per lattice of a batch).
struct LatDev {
    int nx, ny, nz, pad0;
    int per[3];                 // periodic flags per axis
    int slaved, substeps, storage, reaction;
    int weak, pad3;             // weak: all M species stored (slaved = M), else one slaved species
    long long N;
    int n_if, n_out;
    const MechDev* mech;
    long long P;                // population plane stride: N nodes, then the n_if interface slots, rounded up to 64
    void* pop[2];               // ping-pong population buffers [L][27][P]; slot N + k of a plane in the buffer a
                                // step reads holds interface node k's post-boundary population (written by the
                                // boundary kernel of that step)
    double* aux;                // [14 + M][N]: rho, ux, uy, uz, T, Phi_x,y,z, Y_0..Y_{M-1}, P_0..P_5
    double* prm;                // [14 + 6 M + 6][N] per-node record for k_update
    const int* if_index;        // [N]: interface slot or -1 (NULL if n_if == 0)
    const int* if_node;         // [n_if]
    const unsigned* if_mask;    // [n_if] incoming set D as a 27-bit mask
    const int* if_type;         // [n_if] RLBM_FACE_WALL / INLET / OUTLET
    const double* if_T;         // [n_if] wall target temperature
    const int* if_out;          // [n_if] outlet slot or -1
    double* out_state;          // [5 + M][n_out]: rho, ux, uy, uz, T, Y
    const double* ref;          // [L * 27] reference shapes G_li, then [L] sum_i G_li, then sum_i G_fi c_ix^2 (FP32 storage)
    float* rscale[2];           // [N][rss] reference scales s_l of the populations in pop[q] (FP32 storage)
    int rss, pad2;              // floats per node in rscale (L rounded up to 4)
    const double* slotc;        // [M + M * M] R_a and 1/(D_ref m_a m_b) in slot order (slaved species last)
    double rho_in, u_in, T_in, P_inf, sigma;
    double Y_in[MAXM];
    int parity0;                // buffer holding the current populations at t = 0
    int pad1;
    long long t_end;            // batch: lattice active while t < t_end
    int* flag;                  // this lattice's failure flag (bit 0: a temperature iteration failed)
};

constexpr int AUX_RHO = 0, AUX_U = 1, AUX_T = 4, AUX_PHI = 5, AUX_Y = 8;

// Per-node record written by k_local (the reaction increment also by
// k_chem_implicit, the gradients by k_gradients) for k_update (structure of
// arrays, row r of node n at prm[r * N + n]).  The rows PRM_TH, PRM_OMEGA,
// PRM_COMMON, PRM_WQ, PRM_CC and the beta_a rows are not stored: k_update
// derives them once per node and keeps them in its LDS copy of the record.
constexpr int PRM_RHO = 0, PRM_U = 1, PRM_T = 4, PRM_UINT = 5, PRM_TH = 6, PRM_OMEGA = 7, PRM_COMMON = 8,
              PRM_QB = 9, PRM_WQ = 12, PRM_CC = 13, PRM_SP = 14;
// species rows: PRM_SP + 6 a + {0: rho_a, 1..3: V_a, 4: beta_a, 5: drho_a}
__host__ __device__ constexpr int prm_grad(int M) { return PRM_SP + 6 * M; }   // d (3), sum H grad Y (3)
__host__ __device__ constexpr int prm_rows(int M) { return PRM_SP + 6 * M + 6; }
// Correction rows: the energy flux base, the diffusion velocities V_a, the
// reaction increments drho_a and the gradients.  They enter the collision as
// small additive terms, so in FP32 deviation storage they are kept as FP32
// (the first half of the row's bytes, node n at ((float*)&prm[r * N])[n]);
// the conserved moments and state (rho, u, T, U, rho_a) stay FP64 in both
// storages.
__host__ __device__ constexpr bool prm_is_corr(int M, int r) {
    return (r >= PRM_QB && r < PRM_QB + 3) ||
           (r >= PRM_SP && r < prm_grad(M) && (r - PRM_SP) % 6 != 0 && (r - PRM_SP) % 6 != 4) ||
           (r >= prm_grad(M) && r < prm_rows(M));
}


// Compiler barrier: memory may have changed, so mechanism constants used after
// it are re-read (cheap scalar loads) rather than kept live in vector
// registers across loop iterations, which would cost occupancy.
__device__ __forceinline__ void reload_barrier() { asm volatile("" ::: "memory"); }

// Read-only kernel inputs (mechanism, reference populations) are accessed
// through the constant address space: the compiler may then always use
// scalar loads for them, also after a reload barrier.
#define RLBM_CONST __attribute__((address_space(4)))
// Device buffers reached through generic pointers in a struct are cast to the
// global address space so loads and stores take the scalar-base form.
#define RLBM_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ RLBM_GLOBAL T* as_global(T* p) {
    return (RLBM_GLOBAL T*)((unsigned long long)p);
}
template <typename T>
__device__ __forceinline__ const RLBM_GLOBAL T* as_global(const T* p) {
    return (const RLBM_GLOBAL T*)((unsigned long long)p);
}
using MechC = const RLBM_CONST MechDev&;
template <typename T>
__device__ __forceinline__ const RLBM_CONST T* as_const(const T* p) {
    return (const RLBM_CONST T*)((unsigned long long)p);
}

// A zero the compiler cannot see through, held in a scalar register.  Adding
// it to a constant-space pointer inside a loop keeps the loads through that
// pointer in the loop (scalar loads) instead of hoisting every constant into
// registers up front, which would cost occupancy.
__device__ __forceinline__ int opaque_zero() {
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return z;
}
template <typename T>
__device__ __forceinline__ const RLBM_CONST T& in_loop(const RLBM_CONST T& r) {
    return *(&r + opaque_zero());
}

// ---------------------------------------------------------------------------
// product form (section 2.2, eqs. phi0, phiPlus, phis, prod)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double psi(int c, double xi, double P) {
    return c == 0 ? 1.0 - P : 0.5 * (c > 0 ? (xi + P) : (P - xi));
}

// Energy equilibrium of one velocity (section 3.3, eq. geq_i).  With
// W_a = Psi_{c_a}(u_a, theta + u_a^2) the operator product form applied to
// E = U + u^2/2 reduces, since O_b acts as multiplication by u_b on
// functions independent of u_b, to
//   g_i = rho [U Wx Wy Wz + kx Wy Wz + Wx ky Wz + Wx Wy kz],
//   k_0(u) = u^2/2 - O^2[u^2/2],  k_{+-1}(u) = (+-O[u^2/2] + O^2[u^2/2]) / 2,
//   O[u^2/2] = theta u + u^3/2,  O^2[u^2/2] = theta^2 + 5/2 theta u^2 + u^4/2.
struct GeqAxis {
    double W[3];   // c = -1, 0, +1
    double k[3];
};

__device__ __forceinline__ void geq_axis(double u, double th, GeqAxis& a) {
    const double u2 = u * u;
    const double P = th + u2;
    a.W[0] = 0.5 * (P - u);
    a.W[1] = 1.0 - P;
    a.W[2] = 0.5 * (P + u);
    const double o1 = th * u + 0.5 * u2 * u;
    const double o2 = th * th + 2.5 * th * u2 + 0.5 * u2 * u2;
    a.k[0] = 0.5 * (o2 - o1);
    a.k[1] = 0.5 * u2 - o2;
    a.k[2] = 0.5 * (o2 + o1);
}

__device__ __forceinline__ double geq_i(int i, double rho, double U, const GeqAxis& X,
                                        const GeqAxis& Yy, const GeqAxis& Z) {
    const int a = cx_of(i) + 1, b = cy_of(i) + 1, c = cz_of(i) + 1;
    const double wyz = Yy.W[b] * Z.W[c];
    return rho * (U * X.W[a] * wyz + X.k[a] * wyz + X.W[a] * (Yy.k[b] * Z.W[c] + Yy.W[b] * Z.k[c]));
}

// ---------------------------------------------------------------------------
// thermochemistry (section 3.1, eqs. specUa, U, temperature)
// ---------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ double mix_inv_m(MechC mc, const double* Y) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) s += Y[a] * mc.inv_m[a];
    return s;
}

// Collapse sum_a Y_a U_a(T) into one quintic and solve for T by Newton.
template <int M>
__device__ __forceinline__ double solve_T(MechC mc, const double* Y, double U,
                                          double T, int* fail) {
    // species-major, so that one species' six coefficients are live at a
    // time (each c[k] still sums over a in order)
    double c[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const RLBM_CONST double* u = mc.uc[a];
#pragma unroll
        for (int k = 0; k < 6; ++k) c[k] += Y[a] * u[k];
    }
    c[0] -= U;
    for (int it = 0; it < 100; ++it) {
        const double F = c[0] + T * (c[1] + T * (c[2] + T * (c[3] + T * (c[4] + T * c[5]))));
        const double dF = c[1] + T * (2.0 * c[2] + T * (3.0 * c[3] + T * (4.0 * c[4] + T * 5.0 * c[5])));
        const double dT = F / dF;
        T -= dT;
        if (fabs(dT) <= 1e-12 * fabs(T)) return T;
    }
    *fail = 1;
    return T;
}

template <int M>
__device__ __forceinline__ double mix_U(MechC mc, const double* Y, double T) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const RLBM_CONST double* u = mc.uc[a];
        s += Y[a] * (u[0] + T * (u[1] + T * (u[2] + T * (u[3] + T * (u[4] + T * u[5])))));
    }
    return s;
}

__device__ __forceinline__ double species_U(MechC mc, int a, double T) {
    const RLBM_CONST double* u = mc.uc[a];
    return u[0] + T * (u[1] + T * (u[2] + T * (u[3] + T * (u[4] + T * u[5]))));
}

__device__ __forceinline__ double species_cv(MechC mc, int a, double T) {
    const RLBM_CONST double* c = mc.cvc[a];
    return c[0] + T * (c[1] + T * (c[2] + T * (c[3] + T * c[4])));
}

// g_a/(R_univ T) = h/(R T) - s/R for one species.
__device__ __forceinline__ double gibbs_RT(MechC mc, int a, double T, double lnT, double invT) {
    const RLBM_CONST double* n = mc.nasa[a];
    const double h = n[0] + T * (n[1] * 0.5 + T * (n[2] * (1.0 / 3.0) + T * (n[3] * 0.25 + T * n[4] * 0.2))) +
                     n[5] * invT;
    const double s = n[0] * lnT + T * (n[1] + T * (n[2] * 0.5 + T * (n[3] * (1.0 / 3.0) + T * n[4] * 0.25))) +
                     n[6];
    return h - s;
}

// ---------------------------------------------------------------------------
// chemistry (section 2.3, eq. R3): production rates and sub-steps
// ---------------------------------------------------------------------------
// Per-thread LDS columns: the concentrations c_a and the Gibbs functions
// g_a/(R_univ T) of one node, at stride NT doubles between species, so a
// reaction reads just its own factors at a wave-uniform species index.  The
// linearly implicit update adds a third column, dq_b = d q_r / d c_b of the
// current reaction, scattered by factor and gathered at compile-time indices.
template <int NT>
struct ChemLds {
    double* c;   // &c[0][tid]
    double* g;   // &g[0][tid]
    double* dq;  // &dq[0][tid], or nullptr without the Jacobian
};

// Adds k prod_{g != f} c[g] to dq[fac[f]] for every factor f < n (c[f] = 1
// and nothing added for f >= n).
template <int NT>
__device__ __forceinline__ void scatter_factor_derivs(const ChemLds<NT>& ls, const RLBM_CONST int* fac, int n,
                                                      const double* c, double k) {
    // prefix and suffix products of the factor list
    double pre[MAXO], suf[MAXO];
    pre[0] = k;
#pragma unroll
    for (int f = 1; f < MAXO; ++f) pre[f] = pre[f - 1] * c[f - 1];
    suf[MAXO - 1] = 1.0;
#pragma unroll
    for (int f = MAXO - 2; f >= 0; --f) suf[f] = suf[f + 1] * c[f + 1];
#pragma unroll
    for (int f = 0; f < MAXO; ++f) ls.dq[fac[f] * NT] += f < n ? pre[f] * suf[f] : 0.0;
}

// Production rates rho_dot_a and, with JAC, the Jacobian J[a][b] =
// d rho_dot_a / d rho_b at fixed T in the reduced form used by the linearly
// implicit step (K = M - 1 is the last species):
//   Jr[a][b] = J[a][b] - J[a][K],   a, b < K.
// Each mass-action product is a list of factors (one per molecule), so d/dc_b
// of the product is the sum, over the factors that are species b, of the
// product of the other factors; the clip max(c, 0) is differentiated as the
// identity.
template <int M, int NT, bool JAC>
__device__ __forceinline__ void rates_jac(MechC mc0, const double* rho_a, double T, const ChemLds<NT>& ls,
                                          double* wdot, double (*Jr)[M - 1]) {
    constexpr int K = M - 1;
    MechC mc = mc0;
#pragma unroll
    for (int a = 0; a < M; ++a) wdot[a] = 0.0;
    if constexpr (JAC) {
#pragma unroll
        for (int a = 0; a < M; ++a) ls.dq[a * NT] = 0.0;
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
            for (int b = 0; b < K; ++b) Jr[a][b] = 0.0;
    }
    const int R = mc.R;
    if (R == 0) return;
    const double lnT = log(T);
    const double invT = 1.0 / T;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        ls.c[a * NT] = fmax(rho_a[a], 0.0) * mc.inv_m[a];
        ls.g[a * NT] = gibbs_RT(mc, a, T, lnT, invT);
    }
    const double lnc = mc.ln_cstd - lnT;
    for (int r = 0; r < R; ++r) {
        MechC mc = in_loop(mc0);
        const RLBM_CONST RxnDev& x = mc.rx[r];
        const int nf = x.nf, nr = x.nr;
        const double lnkf = x.lnA + x.beta * lnT - x.Ta * invT;
        // forward rate k_f prod_b c_b^nu'_b
        // Every factor slot is read (unused slots name species 0) and masked
        // to 1 or 0, so the factor loops have no branches: the index loads
        // merge into wide scalar loads and the LDS reads issue together.
        double cf[MAXO];
#pragma unroll
        for (int f = 0; f < MAXO; ++f) {
            const double v = ls.c[x.fac_f[f] * NT];
            cf[f] = f < nf ? v : 1.0;
        }
        const double kf = exp(lnkf);
        double fwd = kf;
#pragma unroll
        for (int f = 0; f < MAXO; ++f) fwd *= cf[f];
        if constexpr (JAC) scatter_factor_derivs<NT>(ls, x.fac_f, nf, cf, kf);
        double q = fwd;
        if (x.rev) {
            // k_r = k_f / K_c, ln K_c = -sum_a dnu_a g_a/(R T) + (sum_a dnu_a) ln c_std
            double cr[MAXO], gr[MAXO], gf[MAXO];
#pragma unroll
            for (int f = 0; f < MAXO; ++f) {
                const double v = ls.c[x.fac_r[f] * NT];
                const double w = ls.g[x.fac_r[f] * NT];
                const double u = ls.g[x.fac_f[f] * NT];
                cr[f] = f < nr ? v : 1.0;
                gr[f] = f < nr ? w : 0.0;
                gf[f] = f < nf ? u : 0.0;
            }
            double sg = 0.0;
#pragma unroll
            for (int f = 0; f < MAXO; ++f) sg += gr[f];
#pragma unroll
            for (int f = 0; f < MAXO; ++f) sg -= gf[f];
            const double kr = exp(lnkf + sg - x.dnu_sum * lnc);
            double bwd = kr;
#pragma unroll
            for (int f = 0; f < MAXO; ++f) bwd *= cr[f];
            if constexpr (JAC) scatter_factor_derivs<NT>(ls, x.fac_r, nr, cr, -kr);
            q -= bwd;
        }
#pragma unroll
        for (int a = 0; a < M; ++a) wdot[a] = fma(x.dnu[a], q, wdot[a]);
        if constexpr (JAC) {
            // d rho_dot_a / d rho_b = m_a dnu_a dq_b / m_b summed over the
            // reactions; Jr[a][b] += dnu_a (dq_b / m_b - dq_K / m_K), m_a below
            const double dK = ls.dq[K * NT] * mc.inv_m[K];
            ls.dq[K * NT] = 0.0;
#pragma unroll
            for (int b = 0; b < K; ++b) {
                const double d = fma(ls.dq[b * NT], mc.inv_m[b], -dK);
                ls.dq[b * NT] = 0.0;
#pragma unroll
                for (int a = 0; a < K; ++a) Jr[a][b] = fma(x.dnu[a], d, Jr[a][b]);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < M; ++a) wdot[a] *= mc.m[a];
    if constexpr (JAC) {
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
            for (int b = 0; b < K; ++b) Jr[a][b] *= mc.m[a];
    }
}

template <int M, int NT>
__device__ __forceinline__ void production_rates(MechC mc, const double* rho_a, double T, const ChemLds<NT>& ls,
                                                 double* wdot) {
    rates_jac<M, NT, false>(mc, rho_a, T, ls, wdot, nullptr);
}

// Solves A x = b in place (x returned in b) by Gaussian elimination with
// partial pivoting.  Every index is a compile-time constant, so A stays in
// registers: the pivot search is a chain of compare-and-swap steps that
// leaves the largest |A[i][k]|, i >= k, in row k (the first one on ties).
template <int M>
__device__ __forceinline__ void solve_pivoted(double (*A)[M], double* b) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
#pragma unroll
        for (int i = k + 1; i < M; ++i) {
            const bool sw = fabs(A[i][k]) > fabs(A[k][k]);
#pragma unroll
            for (int j = k; j < M; ++j) {
                const double t = A[k][j];
                A[k][j] = sw ? A[i][j] : t;
                A[i][j] = sw ? t : A[i][j];
            }
            const double t = b[k];
            b[k] = sw ? b[i] : t;
            b[i] = sw ? t : b[i];
        }
        const double inv = 1.0 / A[k][k];
#pragma unroll
        for (int i = k + 1; i < M; ++i) {
            const double f = A[i][k] * inv;
#pragma unroll
            for (int j = k + 1; j < M; ++j) A[i][j] = fma(-f, A[k][j], A[i][j]);
            b[i] = fma(-f, b[k], b[i]);
        }
    }
#pragma unroll
    for (int k = M - 1; k >= 0; --k) {
        double s = b[k];
#pragma unroll
        for (int j = k + 1; j < M; ++j) s = fma(-A[k][j], b[j], s);
        b[k] = s / A[k][k];
    }
}

// Densities after one step of l sub-steps at frozen U: forward Euler
// (eq. R3) or, with IMPL, linearly implicit sub-steps
// (I - dt^r J) Delta = dt^r rho_dot.  Every reaction conserves mass (checked
// when the mechanism is created), so the columns of J sum to zero, and so do
// rho_dot and Delta: the last row of the system is the negative sum of the
// others.  It is dropped, with Delta_K = -sum_{a<K} Delta_a substituted, which
// leaves (I - dt^r Jr) Delta_{<K} = dt^r rho_dot_{<K} of size M - 1.
template <int M, int NT, bool IMPL>
__device__ __forceinline__ void reaction_increment(MechC mc0, const double* rho_a, double rho, double U, double T,
                                                   int l, const ChemLds<NT>& ls, double* out, int* fail) {
    constexpr int K = M - 1;
    double cur[M], w[M];
#pragma unroll
    for (int a = 0; a < M; ++a) cur[a] = rho_a[a];
    if (mc0.R == 0) {
#pragma unroll
        for (int a = 0; a < M; ++a) out[a] = cur[a];
        return;
    }
    const double inv_l = 1.0 / (double)l;
    const double inv_rho = 1.0 / rho;
    double Ts = T;
    for (int s = 0; s < l; ++s) {
        MechC mc = in_loop(mc0);
        if (s > 0) {
            double Y[M];
#pragma unroll
            for (int a = 0; a < M; ++a) Y[a] = cur[a] * inv_rho;
            Ts = solve_T<M>(mc, Y, U, Ts, fail);
        }
        if constexpr (IMPL) {
            double A[K][K];
            rates_jac<M, NT, true>(mc, cur, Ts, ls, w, A);
#pragma unroll
            for (int a = 0; a < K; ++a) {
#pragma unroll
                for (int b = 0; b < K; ++b) A[a][b] = (a == b ? 1.0 : 0.0) - inv_l * A[a][b];
                w[a] *= inv_l;
            }
            solve_pivoted<K>(A, w);
            double sum = 0.0;
#pragma unroll
            for (int a = 0; a < K; ++a) {
                cur[a] += w[a];
                sum += w[a];
            }
            cur[K] -= sum;
        } else {
            production_rates<M, NT>(mc, cur, Ts, ls, w);
#pragma unroll
            for (int a = 0; a < M; ++a) cur[a] += w[a] * inv_l;
        }
    }
#pragma unroll
    for (int a = 0; a < M; ++a) out[a] = cur[a];
}

}  // namespace rlbm
