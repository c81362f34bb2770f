/*
 * rlbm.h -- C ABI of the reactive-mixture lattice Boltzmann library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library advances the M+2 coupled lattice Boltzmann equations of
 * Sawant, Dorschner & Karlin, "Consistent lattice Boltzmann model for reactive
 * mixtures" (arXiv 2108.07605) on the D3Q27 lattice: M species equations with
 * Stefan-Maxwell diffusion and mass-action reaction sources (section 2), the
 * mixture momentum lattice f with the extended equilibrium and the energy
 * lattice g whose energy includes the energy of formation (section 3), with
 * the M-th (slaved) species implied by f - sum_a f_a (section 3.6, eq.
 * strongest), and the wall, inlet and outlet constructions of section 4.
 *
 * Conventions
 *  - Lattice units: dt = dx = 1; temperatures in kelvin.
 *  - Nodes are numbered n = (z * ny + y) * nx + x (x fastest).  Fields are
 *    structure-of-arrays: u is [3][N], Y is [M][N].
 *  - Discrete velocities: i = 9 (c_z + 1) + 3 (c_y + 1) + (c_x + 1); the rest
 *    velocity is i = 13 and the opposite of i is 26 - i.
 *  - Population buffers exchanged through this ABI are FP64, ordered
 *    [L][27][N] with L = M + 1 stored lattices: the M - 1 unslaved species in
 *    ascending species index, then f, then g.  In the weakly coupled storage
 *    (RLBM_SLAVED_NONE) L = M + 2: all M species, then f, then g.
 *  - Every call returns 0 on success or a negative RLBM_E* code; the message
 *    of the last failure on the calling thread is rlbm_last_error().  No call
 *    aborts or throws.
 *  - Pointers flagged on_device refer to device memory of the lattice's GPU;
 *    otherwise to host memory.  The library never frees caller memory.
 *  - Calls on one lattice must not overlap from several threads.
 */
#ifndef RLBM_H
#define RLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RLBM_OK 0
#define RLBM_EINVAL (-1)      /* invalid argument (dims, faces, species, state) */
#define RLBM_ENOSPC (-2)      /* caller buffer smaller than rlbm_lattice_bytes */
#define RLBM_EHIP (-3)        /* a HIP runtime call failed */
#define RLBM_EUNSUP (-4)      /* valid but unsupported configuration */
#define RLBM_ENONFINITE (-5)  /* state contains NaN/Inf or non-positive density */

#define RLBM_MAX_SPECIES 12
#define RLBM_MAX_REACTIONS 64
#define RLBM_MAX_ORDER 4        /* molecules on either side of one reaction */
#define RLBM_MAX_ELEMENTS 8

/* Mechanism: species thermochemistry, reactions and transport, all in
 * lattice units (section 3.6: the paper obtains these from a kinetics
 * package; here they are inputs).
 *
 * Thermo (one NASA-7 range per species, T in kelvin, R_a = R_univ/m_a):
 *   C_{a,p}/R_a = a0 + a1 T + a2 T^2 + a3 T^3 + a4 T^4
 *   H_a/(R_a T) = a0 + a1 T/2 + a2 T^2/3 + a3 T^3/4 + a4 T^4/5 + a5/T
 *   S_a/R_a     = a0 ln T + a1 T + a2 T^2/2 + a3 T^3/3 + a4 T^4/4 + a6
 *   U_a = H_a - R_a T  (eqs. specUa, specHa with the Mayer relation)
 * Reactions (mass action, production rates of section 2.3):
 *   c_b = max(rho_b, 0)/m_b,  k_f = exp(lnA) T^beta exp(-Ta/T),
 *   K_c = exp(-sum_a dnu_a g_a/(R_univ T)) (exp(ln_cstd)/T)^(sum_a dnu_a),
 *   q = k_f prod c^nu_f - reversible * k_f/K_c prod c^nu_r,
 *   rho_dot_a = m_a sum_r (nu_r - nu_f)_ar q_r.
 * Every reaction must conserve mass, sum_a m_a (nu_r - nu_f)_a = 0 to 1e-12
 * relative (eq. sumRhoDot), else RLBM_EINVAL.
 * Transport (synthetic laws standing in for mixture-averaged transport):
 *   mu = mu_ref (T/T_ref)^mu_exp, lambda = mu C_p / Pr,
 *   D_ab = D_ref[a][b] (T/T_ref)^D_exp (P_ref/P),
 *   1/tau_ab = m R_univ T / (D_ab m_a m_b)    (section 2.3, eqs. betaa, taua)
 * The library copies everything; the caller may free the descriptor after
 * rlbm_mech_create returns. */
typedef struct rlbm_mech_desc {
    int32_t M;                    /* species: kernels are compiled for M = 2, 3, 4 and 9
                                     (RLBM_EUNSUP for other M up to RLBM_MAX_SPECIES) */
    int32_t R;                    /* reactions, 0..RLBM_MAX_REACTIONS */
    int32_t E;                    /* elements, 0..RLBM_MAX_ELEMENTS */
    const double* molar_mass;     /* [M] > 0 */
    const double* nasa;           /* [M][7] */
    const int32_t* composition;   /* [M][E] atoms per molecule (invariants); NULL if E = 0 */
    double R_univ;                /* universal gas constant > 0 */
    double ln_cstd;               /* standard concentration c_std(T) = exp(ln_cstd)/T */
    const int32_t* nu_f;          /* [R][M] reactant coefficients, 0..3, sum <= RLBM_MAX_ORDER */
    const int32_t* nu_r;          /* [R][M] product coefficients, 0..3, sum <= RLBM_MAX_ORDER */
    const double* lnA;            /* [R] */
    const double* beta;           /* [R] */
    const double* Ta;             /* [R] activation temperatures Ea/R (K) */
    const int32_t* reversible;    /* [R] 0 or 1 */
    double T_ref, P_ref;          /* transport reference state */
    double mu_ref, mu_exp, Pr;    /* viscosity law and Prandtl number */
    double D_exp;                 /* exponent of the diffusivity law */
    const double* D_ref;          /* [M][M] symmetric, > 0 off the diagonal */
} rlbm_mech_desc;

typedef struct rlbm_mech rlbm_mech;
typedef struct rlbm_lattice rlbm_lattice;

#define RLBM_FACE_PERIODIC 0
#define RLBM_FACE_WALL 1      /* Tamm-Mott-Smith isothermal no-slip wall (section 4.2.2) */
#define RLBM_FACE_INLET 2     /* flux inlet (section 4.3); x- face only */
#define RLBM_FACE_OUTLET 3    /* LODI + convective outlet (section 4.4); x+ face only */
#define RLBM_FACE_BOUNCEBACK 4   /* bounce-back wall (section 4.2.1, eq. bb): no slip half-way, adiabatic */
#define RLBM_FACE_INLET_LOCAL 5  /* simplified flux inlet (end of section 4.3): the node takes the local
                                    equilibria, u and T are not imposed; x- face only, same data as
                                    RLBM_FACE_INLET */

/* One face of the box.  Faces are ordered x-, x+, y-, y+, z-, z+.  An axis is
 * periodic on both faces or on neither.  A node on several non-periodic faces
 * takes the union of their incoming links; wall faces take precedence over
 * the inlet and the outlet at such nodes. */
typedef struct rlbm_face {
    int32_t type;
    /* WALL: target temperature at node x,
     *   T_w(x) = T_lo + (T_hi - T_lo) (1 + tanh((x - x0)/width)) / 2,
     * target velocity 0 (impermeable, stationary). */
    double T_lo, T_hi, x0, width;
    /* INLET: imposed density, normal velocity (+x), temperature and mass
     * fractions of the incoming mixture (its mass flux is rho_in * u_in). */
    double rho_in, u_in, T_in;
    const double* Y_in;           /* [M], copied at rlbm_lattice_create */
    /* OUTLET: far-field pressure and relaxation factor of the partially
     * non-reflecting LODI condition, L1 = sigma (1 - Ma^2) c / nx (P - P_inf). */
    double P_inf, sigma;
} rlbm_face;

/* Reaction sub-step scheme (section 2.3, eq. R3).  EXPLICIT is the paper's
 * forward Euler.  LINEARLY_IMPLICIT solves (I - dt^r J) Delta = dt^r rho_dot
 * per sub-step, J = d rho_dot / d rho at the sub-step's temperature (T held
 * fixed in J, re-solved at frozen U between sub-steps; max(c, 0) in the rates
 * differentiated as the identity).  Mass conservation makes the last row of
 * the system the negative sum of the others, so the library solves the
 * (M-1)-species system that remains, by Gaussian elimination with partial
 * pivoting, and sets Delta of the last species to minus the sum of the rest.
 * It conserves mass and elements like EXPLICIT and is backward Euler for a
 * linear network, so stiff mechanisms need fewer sub-steps. */
#define RLBM_REACTION_EXPLICIT 0
#define RLBM_REACTION_LINEARLY_IMPLICIT 1

/* Weakly coupled storage (section 3.6 before eq. strongest): no species is
 * slaved; all M species lattices are stored beside f and g (L = M + 2) and
 * the two subsystems exchange fields only.  The species supply the
 * composition Y_a = rho_a / sum_b rho_b; f supplies rho and u, and with g the
 * temperature.  Species relax with their own rho_a, toward quasi-equilibria
 * at the velocity u of f; rho and sum_a rho_a are both conserved globally and
 * may drift apart locally, which is the redundancy the slaving removes. */
#define RLBM_SLAVED_NONE (-2)

#define RLBM_STORAGE_F64 0        /* populations stored in FP64 */
#define RLBM_STORAGE_F32_DEV 1    /* FP32 deviations from a per-(lattice, velocity) reference */

typedef struct rlbm_lattice_desc {
    int32_t nx, ny, nz;           /* >= 1 each, >= 2 along an axis with an inlet/outlet; N = nx ny nz
                                     with 9 (N + n_if) s < 2^32 for s = 4 (FP32) or 8 (FP64) bytes,
                                     n_if the number of interface nodes (RLBM_EUNSUP otherwise) */
    rlbm_face faces[6];
    int32_t storage;              /* RLBM_STORAGE_* */
    int32_t substeps;             /* reaction sub-steps l >= 1 (eq. R3) */
    int32_t slaved;               /* slaved species index, or -1: chosen at rlbm_set_state as
                                     the largest domain-mean mass fraction (lowest index on ties),
                                     or RLBM_SLAVED_NONE */
    int32_t reaction;             /* RLBM_REACTION_* */
} rlbm_lattice_desc;

/* Create / destroy a mechanism (host object; uploaded per lattice). */
int rlbm_mech_create(const rlbm_mech_desc* desc, rlbm_mech** out);
void rlbm_mech_destroy(rlbm_mech* mech);

/* Exact number of device bytes a lattice needs: two population buffers,
 * per-node auxiliary fields, interface-node tables and scratch. */
int rlbm_lattice_bytes(const rlbm_lattice_desc* desc, const rlbm_mech* mech, size_t* bytes);

/* Create a lattice in caller-owned device memory `dev_mem` of `bytes` bytes
 * (256-byte aligned), which must stay valid until rlbm_lattice_destroy.
 * `stream` is a hipStream_t (NULL = default stream) on which all work of
 * this lattice is enqueued; it is borrowed, not owned.  The device is the
 * current device at creation.  Synchronous (uploads tables). */
int rlbm_lattice_create(const rlbm_lattice_desc* desc, const rlbm_mech* mech, void* dev_mem,
                        size_t bytes, void* stream, rlbm_lattice** out);
void rlbm_lattice_destroy(rlbm_lattice* lat);

/* Set the state to the equilibria at the given fields (rho > 0, T > 0,
 * sum_a Y_a = 1): species f_a^eq, mixture f^eq and energy g^eq (sections 2.2,
 * 3.2, 3.3).  rho [N], u [3][N], T [N], Y [M][N].  Resets the outlet state
 * and, in FP32 storage, fixes the reference populations at the domain-mean
 * state.  Host inputs are copied synchronously; device inputs are read on the
 * lattice stream. */
int rlbm_set_state(rlbm_lattice* lat, const double* rho, const double* u, const double* T,
                   const double* Y, int on_device);

/* Enqueue n time steps (stream, boundaries, moments, gradients, collision)
 * on the lattice stream and return; n = 0 is a no-op. */
int rlbm_step(rlbm_lattice* lat, int64_t n);

/* Macroscopic fields of the current (post-collision) populations: rho [N],
 * u [3][N], T [N], Y [M][N], P [N]; any pointer may be NULL.  With on_device =
 * 0 the call synchronises the stream and copies to host. */
int rlbm_read_fields(rlbm_lattice* lat, double* rho, double* u, double* T, double* Y, double* P,
                     int on_device);

/* FP64 copies of all stored populations, [L][27][N] (checkpoint/resume and
 * parity).  Writing re-encodes into the lattice's storage format. */
int rlbm_read_populations(rlbm_lattice* lat, double* buf, int on_device);
int rlbm_write_populations(rlbm_lattice* lat, const double* buf, int on_device);

/* Raw state snapshot for bit-exact checkpoint and resume.  The snapshot holds
 * the current populations in their storage format together with everything
 * the next steps read besides them: the FP32 references (shapes and per-node
 * scales), the per-node fields carried between steps (the temperature that
 * starts the next Newton iteration, the interior moments the outlet reads),
 * the outlet state and the slaved-species index.  A lattice that loads it
 * continues bit-identically to the one that saved it.
 *   rlbm_state_bytes: size of the snapshot of this lattice.
 *   rlbm_save_state: writes the snapshot to buf (host or device memory of at
 *     least rlbm_state_bytes bytes); synchronises the lattice's stream.
 *   rlbm_load_state: replaces the lattice's state with the snapshot; the
 *     lattice must have the snapshot's dimensions, species count and storage
 *     (RLBM_EINVAL otherwise).  rlbm_set_state is not needed before it. */
int rlbm_state_bytes(const rlbm_lattice* lat, size_t* bytes);
int rlbm_save_state(rlbm_lattice* lat, void* buf, int on_device);
int rlbm_load_state(rlbm_lattice* lat, const void* buf, int on_device);

/* Global invariants of the current populations into host array out[n_out]:
 * [0] sum rho, [1..3] sum rho u, [4] sum rho E, [5..5+E) element totals
 * (moles), [5+E] 1 if any population is non-finite else 0.  Needs
 * n_out >= 6 + E.  Synchronises the stream. */
int rlbm_invariants(rlbm_lattice* lat, double* out, int n_out);

/* Failure detection (the per-lattice flag).  Every kernel that solves the
 * temperature equation (section 3.1, eq. temperature: moments, boundary
 * constructions, reaction sub-steps, read-out) sets bit 0 of its lattice's
 * flag when the bounded Newton iteration does not converge, which is how a
 * non-physical or non-finite state shows itself; the kernels still finish.
 * Lattices of a batch each keep their own flag.  rlbm_lattice_status
 * synchronises the lattice stream, returns the bits set since the last
 * call in *status (0: healthy) and clears them.  rlbm_read_fields also
 * reports a set flag, as RLBM_ENONFINITE, and clears it. */
int rlbm_lattice_status(rlbm_lattice* lat, int32_t* status);

/* Number of stored lattices L, nodes N and interface nodes, and the slaved
 * species (RLBM_SLAVED_NONE in the weakly coupled storage). */
int rlbm_lattice_shape(const rlbm_lattice* lat, int32_t* L, int64_t* N, int64_t* n_interface,
                       int32_t* slaved);

/* Per-kernel timing with HIP events recorded on the lattice stream around
 * the launches of the kernels selected by `enable`: bit k set times kernel k
 * in {0: boundary, 1: moments, diffusion and the forward-Euler reaction
 * increment, 2: gradients (with the linearly implicit reaction increment
 * before them where selected), 3: update}; 0 switches timing off.  Event pairs are pooled and reused.
 * rlbm_kernel_times synchronises and returns the accumulated milliseconds
 * ms[k] and launch counts counts[k] since the last reset. */
int rlbm_set_timing(rlbm_lattice* lat, int enable);
int rlbm_kernel_times(rlbm_lattice* lat, double* ms, int64_t* counts, int n);

/* Batches of independent lattices advanced together (the batched uneven
 * instances of one GPU).  Each kernel phase of a step is one launch over the
 * flattened (lattice, node-block) work list of all lattices of the batch, so
 * small and uneven instances share the GPU; a lattice with fewer steps in a
 * call returns from its blocks once they are done.  All lattices of a batch
 * must be on the same device, use the same species count, storage format and
 * coupling (a slaved species, or RLBM_SLAVED_NONE for all), and appear once
 * (RLBM_EINVAL otherwise).  They may differ in everything else, the reaction
 * scheme included.  A batch step is equivalent, bit for bit, to rlbm_step on
 * each lattice.
 *   rlbm_batch_bytes: device bytes of the batch's tables for k lattices.
 *   rlbm_batch_create: the batch keeps its tables in the caller-owned device
 *     memory dev_mem (rlbm_batch_bytes(k) bytes, 256-byte aligned), which must
 *     stay valid until rlbm_batch_destroy; the lattices must stay valid while
 *     the batch is stepped or queried.  It also
 *     holds a little pinned host memory, events and a private stream.
 *     Synchronous. */
typedef struct rlbm_batch rlbm_batch;
int rlbm_batch_bytes(int32_t k, size_t* bytes);
int rlbm_batch_create(rlbm_lattice* const* lats, int32_t k, void* dev_mem, size_t bytes,
                      rlbm_batch** out);
/* Advance lattice j by steps[j] >= 0 steps.  Asynchronous: the work is
 * enqueued on the first lattice's stream, after the work already queued on
 * the other lattices' streams, and those streams wait for it, so later calls
 * on any lattice of the batch see its result.  Whole chunks of 16 steps are
 * enqueued as replays of one captured HIP graph (kernel nodes only), the
 * rest as direct launches.  Returns at once unless the host staging of the
 * call before last is still in flight. */
int rlbm_batch_step(rlbm_batch* batch, const int64_t* steps);
/* Failure flags of every lattice, status[k] (see rlbm_lattice_status), read
 * and cleared by one gather on the batch stream; synchronises that stream. */
int rlbm_batch_status(rlbm_batch* batch, int32_t* status);
/* Waits for the batch's enqueued work, then frees the batch (not the
 * lattices, which may already have been destroyed). */
void rlbm_batch_destroy(rlbm_batch* batch);

/* Group step without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Advances lattice j by steps[j] >= 0 steps, with the same
 * kernels and results as a batch of these lattices (bit for bit), but keeps
 * the work list in a file-scope device array of the library instead of
 * caller memory: no allocation, no batch object, no pinned staging, no graph.
 * Limits: 1 <= k <= RLBM_GROUP_MAX_LATTICES (RLBM_EINVAL beyond); all
 * lattices on one device and one stream (RLBM_EINVAL otherwise), with the
 * batch's other requirements.  Asynchronous on that stream.  Every call on a
 * GPU shares that GPU's array (about 100 KB, held until the process ends):
 * calls that overlap on one GPU, from several threads or on several streams,
 * race and must be ordered by the caller. */
#define RLBM_GROUP_MAX_LATTICES 256
int rlbm_step_group(rlbm_lattice* const* lats, int32_t k, const int64_t* steps);

const char* rlbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RLBM_H */
