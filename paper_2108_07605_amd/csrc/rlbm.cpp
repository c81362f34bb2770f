// Host side of the C ABI (include/rlbm.h): validation, device memory plan,
// interface-node tables, launches and timing.  No exception crosses the ABI.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "launch.hpp"
#include "physics.hpp"
#include "rlbm.h"

using namespace rlbm;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(RLBM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                       \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int NPHASE = 4;   // boundary, moments + diffusion, chemistry + gradients, update

struct Plan {
    size_t off_lat, off_mech, off_blk, off_flag, off_ref, off_pop0, off_pop1, off_aux, off_prm, off_ifindex, off_ifnode,
        off_ifmask, off_iftype, off_ifT, off_ifout, off_out, off_partial, off_invout, off_slot,
        off_rscale0, off_rscale1, total;
};

struct Geometry {
    long long N = 0;
    std::vector<int> if_index, if_node, if_type, if_out;
    std::vector<unsigned> if_mask;
    std::vector<double> if_T;
    int n_out = 0;
};

bool face_valid(int t) { return t >= RLBM_FACE_PERIODIC && t <= RLBM_FACE_INLET_LOCAL; }
bool is_inlet(int t) { return t == RLBM_FACE_INLET || t == RLBM_FACE_INLET_LOCAL; }

int validate_desc(const rlbm_lattice_desc* d, int M) {
    if (!d) return fail(RLBM_EINVAL, "null lattice descriptor");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(RLBM_EINVAL, "lattice dimensions must be >= 1");
    // kernels address nine population planes with 32-bit byte offsets
    const long long n_nodes = (long long)d->nx * d->ny * d->nz;
    const long long s_bytes = d->storage == RLBM_STORAGE_F32_DEV ? 4 : 8;
    if (9 * s_bytes * n_nodes >= (1LL << 32))
        return fail(RLBM_EUNSUP, "too many nodes: 9 N sizeof(storage) must stay below 2^32");
    for (int f = 0; f < 6; ++f)
        if (!face_valid(d->faces[f].type)) return fail(RLBM_EINVAL, "unknown face type");
    const int n[3] = {d->nx, d->ny, d->nz};
    for (int ax = 0; ax < 3; ++ax) {
        const bool p0 = d->faces[2 * ax].type == RLBM_FACE_PERIODIC;
        const bool p1 = d->faces[2 * ax + 1].type == RLBM_FACE_PERIODIC;
        if (p0 != p1) return fail(RLBM_EINVAL, "an axis must be periodic on both faces or on neither");
        if (!p0 && n[ax] < 2) return fail(RLBM_EINVAL, "a non-periodic axis needs at least 2 nodes");
    }
    for (int f = 0; f < 6; ++f) {
        const rlbm_face& fc = d->faces[f];
        if (is_inlet(fc.type)) {
            if (f != 0) return fail(RLBM_EUNSUP, "inlets are supported on the x- face only");
            if (!(fc.rho_in > 0) || !(fc.T_in > 0) || !fc.Y_in)
                return fail(RLBM_EINVAL, "inlet needs rho_in > 0, T_in > 0 and Y_in");
            double s = 0;
            for (int a = 0; a < M; ++a) {
                if (!(fc.Y_in[a] >= 0)) return fail(RLBM_EINVAL, "inlet mass fractions must be >= 0");
                s += fc.Y_in[a];
            }
            if (std::fabs(s - 1.0) > 1e-10) return fail(RLBM_EINVAL, "inlet mass fractions must sum to 1");
        }
        if (fc.type == RLBM_FACE_OUTLET) {
            if (f != 1) return fail(RLBM_EUNSUP, "outlets are supported on the x+ face only");
            if (!(fc.P_inf > 0) || !(fc.sigma >= 0)) return fail(RLBM_EINVAL, "outlet needs P_inf > 0, sigma >= 0");
        }
        if (fc.type == RLBM_FACE_WALL) {
            if (!(fc.T_lo > 0) || !(fc.T_hi > 0) || !(fc.width > 0))
                return fail(RLBM_EINVAL, "wall needs T_lo, T_hi, width > 0");
        }
    }
    if (d->storage != RLBM_STORAGE_F64 && d->storage != RLBM_STORAGE_F32_DEV)
        return fail(RLBM_EINVAL, "unknown storage format");
    if (d->substeps < 1) return fail(RLBM_EINVAL, "substeps must be >= 1");
    if (d->reaction != RLBM_REACTION_EXPLICIT && d->reaction != RLBM_REACTION_LINEARLY_IMPLICIT)
        return fail(RLBM_EINVAL, "unknown reaction scheme");
    if (d->slaved < RLBM_SLAVED_NONE || d->slaved >= M) return fail(RLBM_EINVAL, "slaved species index out of range");
    return RLBM_OK;
}

// Interface nodes: incoming sets D (velocities whose source lies outside the
// box through a non-periodic face) and the boundary type of every node.
void build_geometry(const rlbm_lattice_desc* d, Geometry& g) {
    const int nx = d->nx, ny = d->ny, nz = d->nz;
    g.N = (long long)nx * ny * nz;
    const int n[3] = {nx, ny, nz};
    bool per[3];
    for (int ax = 0; ax < 3; ++ax) per[ax] = d->faces[2 * ax].type == RLBM_FACE_PERIODIC;
    bool any = !(per[0] && per[1] && per[2]);
    g.if_index.assign(any ? (size_t)g.N : 0, -1);
    if (!any) return;
    // wall target temperature: first wall face touched in y-, y+, z-, z+, x-, x+
    const int prio[6] = {2, 3, 4, 5, 0, 1};
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int c[3] = {x, y, z};
                bool on[6];
                bool touches = false;
                for (int ax = 0; ax < 3; ++ax) {
                    on[2 * ax] = !per[ax] && c[ax] == 0;
                    on[2 * ax + 1] = !per[ax] && c[ax] == n[ax] - 1;
                    touches |= on[2 * ax] || on[2 * ax + 1];
                }
                if (!touches) continue;
                unsigned mask = 0;
                for (int i = 0; i < Q; ++i) {
                    const int ci[3] = {cx_of(i), cy_of(i), cz_of(i)};
                    bool out = false;
                    for (int ax = 0; ax < 3; ++ax) {
                        if (per[ax]) continue;
                        const int src = c[ax] - ci[ax];
                        out |= src < 0 || src >= n[ax];
                    }
                    if (out) mask |= 1u << i;
                }
                int type = 0;
                double Tw = 0.0;
                for (int q = 0; q < 6 && type == 0; ++q) {
                    const int f = prio[q];
                    if (on[f] && d->faces[f].type == RLBM_FACE_WALL) {
                        type = RLBM_FACE_WALL;
                        const rlbm_face& fc = d->faces[f];
                        Tw = fc.T_lo + (fc.T_hi - fc.T_lo) * 0.5 * (1.0 + std::tanh((x - fc.x0) / fc.width));
                    }
                }
                // bounce-back walls after Tamm-Mott-Smith walls, before inlet and outlet
                for (int q = 0; q < 6 && type == 0; ++q)
                    if (on[prio[q]] && d->faces[prio[q]].type == RLBM_FACE_BOUNCEBACK) type = RLBM_FACE_BOUNCEBACK;
                if (type == 0 && on[0] && is_inlet(d->faces[0].type)) type = d->faces[0].type;
                if (type == 0 && on[1] && d->faces[1].type == RLBM_FACE_OUTLET) type = RLBM_FACE_OUTLET;
                if (type == 0) continue;   // cannot happen: every non-periodic face has a type
                const long long node = ((long long)z * ny + y) * nx + x;
                g.if_index[node] = (int)g.if_node.size();
                g.if_node.push_back((int)node);
                g.if_mask.push_back(mask);
                g.if_type.push_back(type);
                g.if_T.push_back(Tw);
                g.if_out.push_back(type == RLBM_FACE_OUTLET ? g.n_out++ : -1);
            }
    // group the interface nodes by boundary type (stable): the boundary
    // kernel's waves then hold nodes of one type and take one branch
    const size_t nif = g.if_node.size();
    std::vector<size_t> ord(nif);
    for (size_t j = 0; j < nif; ++j) ord[j] = j;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return g.if_type[a] < g.if_type[b]; });
    Geometry s;
    s.N = g.N;
    s.if_index.assign(g.if_index.size(), -1);
    for (size_t j = 0; j < nif; ++j) {
        const size_t o = ord[j];
        s.if_index[g.if_node[o]] = (int)j;
        s.if_node.push_back(g.if_node[o]);
        s.if_mask.push_back(g.if_mask[o]);
        s.if_type.push_back(g.if_type[o]);
        s.if_T.push_back(g.if_T[o]);
        s.if_out.push_back(g.if_type[o] == RLBM_FACE_OUTLET ? s.n_out++ : -1);
    }
    g = std::move(s);
}

// Stored lattices: M - 1 species (one slaved), or all M in the weakly coupled
// storage, plus f and g.
int stored_lattices(const rlbm_lattice_desc* d, int M) { return d->slaved == RLBM_SLAVED_NONE ? M + 2 : M + 1; }

// Population plane stride: the nodes, then one slot per interface node for its
// post-boundary population, rounded up to 64 entries.
size_t plane_stride(const Geometry& g) {
    const size_t nif = g.if_node.size();
    return nif ? ((size_t)g.N + nif + 63) / 64 * 64 : (size_t)g.N;
}

// Kernels address nine population planes with 32-bit byte offsets.
int check_planes(const rlbm_lattice_desc* d, const Geometry& g) {
    const size_t s_bytes = d->storage == RLBM_STORAGE_F32_DEV ? 4 : 8;
    if (9 * s_bytes * plane_stride(g) >= (1ull << 32))
        return fail(RLBM_EUNSUP, "too many nodes: 9 (N + interface nodes) sizeof(storage) must stay below 2^32");
    return RLBM_OK;
}

Plan make_plan(const rlbm_lattice_desc* d, int M, int E, const Geometry& g) {
    Plan p{};
    const int L = stored_lattices(d, M);
    const size_t N = (size_t)g.N;
    const size_t s = d->storage == RLBM_STORAGE_F32_DEV ? 4 : 8;
    const size_t nif = g.if_node.size();
    const size_t nblocks = (N + 255) / 256;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
    p.off_lat = take(sizeof(LatDev));
    p.off_mech = take(sizeof(MechDev));
    p.off_blk = take(6 * sizeof(int));
    p.off_flag = take(sizeof(int));
    p.off_ref = take(((size_t)L * Q + L + Q + 2) * sizeof(double));
    p.off_slot = take((size_t)(M + M * M) * sizeof(double));
    const size_t P = plane_stride(g);
    p.off_pop0 = take((size_t)L * Q * P * s);
    p.off_pop1 = take((size_t)L * Q * P * s);
    p.off_aux = take((size_t)(AUX_Y + M + 6) * N * sizeof(double));
    p.off_prm = take((size_t)prm_rows(M) * N * sizeof(double));
    p.off_ifindex = take(nif ? N * sizeof(int) : 0);
    p.off_ifnode = take(nif * sizeof(int));
    p.off_ifmask = take(nif * sizeof(unsigned));
    p.off_iftype = take(nif * sizeof(int));
    p.off_ifT = take(nif * sizeof(double));
    p.off_ifout = take(nif * sizeof(int));
    p.off_out = take((size_t)(5 + M) * g.n_out * sizeof(double));
    p.off_partial = take(nblocks * (6 + E) * sizeof(double));
    p.off_invout = take((6 + E) * sizeof(double));
    const size_t rss = d->storage == RLBM_STORAGE_F32_DEV ? (size_t)((L + 3) / 4 * 4) : 0;
    p.off_rscale0 = take(rss * N * sizeof(float));
    p.off_rscale1 = take(rss * N * sizeof(float));
    p.total = o;
    return p;
}

struct Timing {
    int kernel;
    hipEvent_t a, b;
};

}  // namespace

struct rlbm_mech {
    MechDev dev;
};

struct rlbm_lattice {
    int device = 0;
    hipStream_t stream = nullptr;
    rlbm_lattice_desc desc{};
    std::vector<double> Y_in;
    int M = 0, L = 0, E = 0, storage = 0;
    Geometry geo;
    Plan plan{};
    char* base = nullptr;
    MechDev mech{};           // host copy of the mechanism (slot tables at rlbm_set_state)
    LatDev host{};            // mirror of the device entry
    LatDev* d_lat = nullptr;
    int* d_blk = nullptr;     // [0, node blocks] and [0, interface blocks]
    int* d_flag = nullptr;
    double* d_ref = nullptr;
    double* d_partial = nullptr;
    double* d_invout = nullptr;
    long long steps_done = 0;
    bool state_set = false;
    unsigned timing = 0;           // bit k: time kernel k
    std::vector<Timing> events;    // pool of event pairs; the first n_events are recorded
    size_t n_events = 0;
    double ms[NPHASE] = {0, 0, 0, 0};
    long long counts[NPHASE] = {0, 0, 0, 0};
};

extern "C" {

const char* rlbm_last_error(void) { return g_last_error.c_str(); }

int rlbm_mech_create(const rlbm_mech_desc* d, rlbm_mech** out) {
    if (!d || !out) return fail(RLBM_EINVAL, "null argument");
    *out = nullptr;
    const int M = d->M, R = d->R, E = d->E;
    if (M < 2 || M > RLBM_MAX_SPECIES) return fail(RLBM_EINVAL, "species count out of range");
    if (!species_supported(M)) return fail(RLBM_EUNSUP, "species count has no compiled kernel (2, 3, 4, 9)");
    if (R < 0 || R > RLBM_MAX_REACTIONS) return fail(RLBM_EINVAL, "reaction count out of range");
    if (E < 0 || E > RLBM_MAX_ELEMENTS) return fail(RLBM_EINVAL, "element count out of range");
    if (!d->molar_mass || !d->nasa || !d->D_ref) return fail(RLBM_EINVAL, "missing species data");
    if (E > 0 && !d->composition) return fail(RLBM_EINVAL, "missing composition");
    if (R > 0 && (!d->nu_f || !d->nu_r || !d->lnA || !d->beta || !d->Ta || !d->reversible))
        return fail(RLBM_EINVAL, "missing reaction data");
    if (!(d->R_univ > 0) || !(d->T_ref > 0) || !(d->P_ref > 0) || !(d->mu_ref > 0) || !(d->Pr > 0))
        return fail(RLBM_EINVAL, "R_univ, T_ref, P_ref, mu_ref and Pr must be > 0");
    rlbm_mech* m = new (std::nothrow) rlbm_mech();
    if (!m) return fail(RLBM_EINVAL, "out of host memory");
    MechDev& md = m->dev;
    std::memset(&md, 0, sizeof(md));
    md.M = M; md.R = R; md.E = E;
    md.R_univ = d->R_univ;
    md.ln_cstd = d->ln_cstd;
    for (int a = 0; a < M; ++a) {
        const double ma = d->molar_mass[a];
        if (!(ma > 0)) { delete m; return fail(RLBM_EINVAL, "molar masses must be > 0"); }
        md.m[a] = ma;
        md.inv_m[a] = 1.0 / ma;
        md.Ra[a] = d->R_univ / ma;
        const double* n = d->nasa + 7 * a;
        for (int k = 0; k < 7; ++k) md.nasa[a][k] = n[k];
        const double R_a = md.Ra[a];
        md.uc[a][0] = R_a * n[5];
        md.uc[a][1] = R_a * (n[0] - 1.0);
        md.uc[a][2] = R_a * n[1] / 2.0;
        md.uc[a][3] = R_a * n[2] / 3.0;
        md.uc[a][4] = R_a * n[3] / 4.0;
        md.uc[a][5] = R_a * n[4] / 5.0;
        md.cvc[a][0] = R_a * (n[0] - 1.0);
        for (int k = 1; k < 5; ++k) md.cvc[a][k] = R_a * n[k];
        for (int k = 0; k < 6; ++k) md.hc[a][k] = md.uc[a][k];
        md.hc[a][1] += R_a;   // H_a = U_a + R_a T
        for (int b = 0; b < M; ++b) {
            if (b == a) continue;
            const double D = d->D_ref[a * M + b];
            if (!(D > 0) || D != d->D_ref[b * M + a]) {
                delete m;
                return fail(RLBM_EINVAL, "D_ref must be symmetric and > 0 off the diagonal");
            }
            md.Kab[a][b] = 1.0 / (D * ma * d->molar_mass[b]);
        }
        for (int e = 0; e < E; ++e) md.comp[a][e] = (double)d->composition[a * E + e];
    }
    for (int r = 0; r < R; ++r) {
        RxnDev& x = md.rx[r];
        x.lnA = d->lnA[r];
        x.beta = d->beta[r];
        x.Ta = d->Ta[r];
        x.rev = d->reversible[r] ? 1 : 0;
        double s = 0;
        for (int a = 0; a < M; ++a) {
            const int f = d->nu_f[r * M + a], b = d->nu_r[r * M + a];
            if (f < 0 || f > 3 || b < 0 || b > 3) {
                delete m;
                return fail(RLBM_EUNSUP, "stoichiometric coefficients must be 0..3");
            }
            x.dnu[a] = (double)(b - f);
            s += (double)(b - f);
            if (x.nf + f > RLBM_MAX_ORDER || x.nr + b > RLBM_MAX_ORDER) {
                delete m;
                return fail(RLBM_EUNSUP, "more than RLBM_MAX_ORDER molecules on one side of a reaction");
            }
            for (int k = 0; k < f; ++k) x.fac_f[x.nf++] = a;
            for (int k = 0; k < b; ++k) x.fac_r[x.nr++] = a;
        }
        x.dnu_sum = s;
        // sum_a m_a dnu_a = 0: the rates conserve mass (eq. sumRhoDot)
        double net = 0.0, gross = 0.0;
        for (int a = 0; a < M; ++a) {
            net += d->molar_mass[a] * x.dnu[a];
            gross += d->molar_mass[a] * std::fabs(x.dnu[a]);
        }
        if (std::fabs(net) > 1e-12 * gross) {
            delete m;
            return fail(RLBM_EINVAL, "a reaction does not conserve mass (sum_a m_a dnu_a != 0)");
        }
    }
    md.T_ref = d->T_ref;
    md.inv_T_ref = 1.0 / d->T_ref;
    md.P_ref = d->P_ref;
    md.inv_P_ref = 1.0 / d->P_ref;
    md.mu_ref = d->mu_ref;
    md.mu_exp = d->mu_exp;
    md.inv_Pr = 1.0 / d->Pr;
    md.D_exp = d->D_exp;
    *out = m;
    return RLBM_OK;
}

void rlbm_mech_destroy(rlbm_mech* m) { delete m; }

int rlbm_lattice_bytes(const rlbm_lattice_desc* d, const rlbm_mech* mech, size_t* bytes) {
    if (!mech || !bytes) return fail(RLBM_EINVAL, "null argument");
    const int rc = validate_desc(d, mech->dev.M);
    if (rc) return rc;
    Geometry g;
    build_geometry(d, g);
    const int rp = check_planes(d, g);
    if (rp) return rp;
    *bytes = make_plan(d, mech->dev.M, mech->dev.E, g).total;
    return RLBM_OK;
}

int rlbm_lattice_create(const rlbm_lattice_desc* d, const rlbm_mech* mech, void* dev_mem, size_t bytes,
                        void* stream, rlbm_lattice** out) {
    if (!mech || !out || !dev_mem) return fail(RLBM_EINVAL, "null argument");
    *out = nullptr;
    const int M = mech->dev.M;
    int rc = validate_desc(d, M);
    if (rc) return rc;
    if (((uintptr_t)dev_mem & 255) != 0) return fail(RLBM_EINVAL, "device memory must be 256-byte aligned");
    rlbm_lattice* lat = new (std::nothrow) rlbm_lattice();
    if (!lat) return fail(RLBM_EINVAL, "out of host memory");
    lat->desc = *d;
    lat->M = M;
    lat->mech = mech->dev;
    lat->L = stored_lattices(d, M);
    lat->E = mech->dev.E;
    lat->storage = d->storage;
    lat->stream = (hipStream_t)stream;
    build_geometry(d, lat->geo);
    rc = check_planes(d, lat->geo);
    if (rc) {
        delete lat;
        return rc;
    }
    lat->plan = make_plan(d, M, lat->E, lat->geo);
    if (bytes < lat->plan.total) {
        delete lat;
        return fail(RLBM_ENOSPC, "device buffer smaller than rlbm_lattice_bytes");
    }
    if (hipGetDevice(&lat->device) != hipSuccess) {
        delete lat;
        return fail(RLBM_EHIP, "hipGetDevice failed");
    }
    char* base = (char*)dev_mem;
    lat->base = base;
    const Plan& p = lat->plan;
    const Geometry& g = lat->geo;
    const size_t nif = g.if_node.size();
    LatDev& h = lat->host;
    std::memset(&h, 0, sizeof(h));
    h.nx = d->nx; h.ny = d->ny; h.nz = d->nz;
    for (int ax = 0; ax < 3; ++ax) h.per[ax] = d->faces[2 * ax].type == RLBM_FACE_PERIODIC;
    // the weakly coupled storage marks "no slaved species" with the index M
    h.weak = d->slaved == RLBM_SLAVED_NONE ? 1 : 0;
    h.slaved = h.weak ? M : (d->slaved < 0 ? M - 1 : d->slaved);
    h.substeps = d->substeps;
    h.storage = d->storage;
    h.reaction = d->reaction;
    h.N = g.N;
    h.P = (long long)plane_stride(g);
    h.n_if = (int)nif;
    h.n_out = g.n_out;
    h.mech = (const MechDev*)(base + p.off_mech);
    h.slotc = (const double*)(base + p.off_slot);
    h.pop[0] = base + p.off_pop0;
    h.pop[1] = base + p.off_pop1;
    h.aux = (double*)(base + p.off_aux);
    h.prm = (double*)(base + p.off_prm);
    h.if_index = nif ? (const int*)(base + p.off_ifindex) : nullptr;
    h.if_node = (const int*)(base + p.off_ifnode);
    h.if_mask = (const unsigned*)(base + p.off_ifmask);
    h.if_type = (const int*)(base + p.off_iftype);
    h.if_T = (const double*)(base + p.off_ifT);
    h.if_out = (const int*)(base + p.off_ifout);
    h.out_state = (double*)(base + p.off_out);
    h.ref = d->storage == RLBM_STORAGE_F32_DEV ? (const double*)(base + p.off_ref) : nullptr;
    h.rss = d->storage == RLBM_STORAGE_F32_DEV ? (lat->L + 3) / 4 * 4 : 0;
    h.rscale[0] = d->storage == RLBM_STORAGE_F32_DEV ? (float*)(base + p.off_rscale0) : nullptr;
    h.rscale[1] = d->storage == RLBM_STORAGE_F32_DEV ? (float*)(base + p.off_rscale1) : nullptr;
    const rlbm_face& fi = d->faces[0];
    if (is_inlet(fi.type)) {
        h.rho_in = fi.rho_in; h.u_in = fi.u_in; h.T_in = fi.T_in;
        for (int a = 0; a < M; ++a) h.Y_in[a] = fi.Y_in[a];
    }
    const rlbm_face& fo = d->faces[1];
    if (fo.type == RLBM_FACE_OUTLET) { h.P_inf = fo.P_inf; h.sigma = fo.sigma; }
    h.parity0 = 0;
    h.t_end = LLONG_MAX;
    h.flag = (int*)(base + p.off_flag);
    lat->d_lat = (LatDev*)(base + p.off_lat);
    lat->d_blk = (int*)(base + p.off_blk);
    lat->d_flag = (int*)(base + p.off_flag);
    lat->d_ref = (double*)(base + p.off_ref);
    lat->d_partial = (double*)(base + p.off_partial);
    lat->d_invout = (double*)(base + p.off_invout);
    const int nb_nodes = (int)((g.N + NODE_TILE - 1) / NODE_TILE);
    const int nb_if = (int)((nif + BC_NODES - 1) / BC_NODES);
    const int nb64 = (int)((g.N + 63) / 64);
    const int blk[6] = {0, nb_nodes, 0, nb_if, 0, nb64};
    const int zero = 0;
#define UP(dst, src, n)                                                              \
    do {                                                                             \
        hipError_t e_ = hipMemcpy((dst), (src), (n), hipMemcpyHostToDevice);        \
        if (e_ != hipSuccess) { delete lat; return hip_fail(e_, "upload"); }        \
    } while (0)
    UP(base + p.off_mech, &mech->dev, sizeof(MechDev));
    UP(lat->d_lat, &h, sizeof(LatDev));
    UP(lat->d_blk, blk, sizeof(blk));
    UP(lat->d_flag, &zero, sizeof(int));
    if (nif) {
        UP(base + p.off_ifindex, g.if_index.data(), (size_t)g.N * sizeof(int));
        UP(base + p.off_ifnode, g.if_node.data(), nif * sizeof(int));
        UP(base + p.off_ifmask, g.if_mask.data(), nif * sizeof(unsigned));
        UP(base + p.off_iftype, g.if_type.data(), nif * sizeof(int));
        UP(base + p.off_ifT, g.if_T.data(), nif * sizeof(double));
        UP(base + p.off_ifout, g.if_out.data(), nif * sizeof(int));
    }
#undef UP
    if (is_inlet(fi.type)) lat->Y_in.assign(fi.Y_in, fi.Y_in + M);
    *out = lat;
    return RLBM_OK;
}

void rlbm_lattice_destroy(rlbm_lattice* lat) {
    if (!lat) return;
    for (auto& e : lat->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    delete lat;
}

int rlbm_lattice_shape(const rlbm_lattice* lat, int32_t* L, int64_t* N, int64_t* n_interface, int32_t* slaved) {
    if (!lat) return fail(RLBM_EINVAL, "null lattice");
    if (L) *L = lat->L;
    if (N) *N = lat->geo.N;
    if (n_interface) *n_interface = (int64_t)lat->geo.if_node.size();
    if (slaved) *slaved = lat->host.weak ? RLBM_SLAVED_NONE : lat->host.slaved;
    return RLBM_OK;
}

// Slot order for the collision: stored species in lattice order, then the
// slaved one (species order in the weakly coupled storage); gas constants R_a
// and couplings 1/(D_ref m_a m_b) permuted.
// The host vector is synchronised before it goes out of scope.
static int upload_slot_table(rlbm_lattice* lat) {
    const int M = lat->M;
    std::vector<double> slot((size_t)M + (size_t)M * M);
    const int sl = lat->host.slaved;
    const bool weak = lat->host.weak != 0;
    auto spc = [&](int j) { return weak ? j : (j < M - 1 ? j + (j >= sl ? 1 : 0) : sl); };
    for (int j = 0; j < M; ++j) {
        slot[j] = lat->mech.Ra[spc(j)];
        for (int q = 0; q < M; ++q) slot[M + (size_t)j * M + q] = lat->mech.Kab[spc(j)][spc(q)];
    }
    HIP_TRY(hipMemcpyAsync((void*)lat->host.slotc, slot.data(), slot.size() * sizeof(double), hipMemcpyHostToDevice,
                           lat->stream),
            "upload");
    HIP_TRY(hipStreamSynchronize(lat->stream), "hipStreamSynchronize");
    return RLBM_OK;
}

int rlbm_set_state(rlbm_lattice* lat, const double* rho, const double* u, const double* T, const double* Y,
                   int on_device) {
    if (!lat || !rho || !u || !T || !Y) return fail(RLBM_EINVAL, "null argument");
    HIP_TRY(hipSetDevice(lat->device), "hipSetDevice");
    const int M = lat->M;
    const size_t N = (size_t)lat->geo.N;
    const size_t nf = (5 + (size_t)M) * N;   // rho, u(3), T, Y(M)
    std::vector<double> hf(nf);
    double* hr = hf.data();
    double* hu = hr + N;
    double* hT = hu + 3 * N;
    double* hY = hT + N;
    if (on_device) {
        HIP_TRY(hipStreamSynchronize(lat->stream), "hipStreamSynchronize");
        HIP_TRY(hipMemcpy(hr, rho, N * sizeof(double), hipMemcpyDeviceToHost), "copy rho");
        HIP_TRY(hipMemcpy(hu, u, 3 * N * sizeof(double), hipMemcpyDeviceToHost), "copy u");
        HIP_TRY(hipMemcpy(hT, T, N * sizeof(double), hipMemcpyDeviceToHost), "copy T");
        HIP_TRY(hipMemcpy(hY, Y, (size_t)M * N * sizeof(double), hipMemcpyDeviceToHost), "copy Y");
    } else {
        std::memcpy(hr, rho, N * sizeof(double));
        std::memcpy(hu, u, 3 * N * sizeof(double));
        std::memcpy(hT, T, N * sizeof(double));
        std::memcpy(hY, Y, (size_t)M * N * sizeof(double));
    }
    double mean_rho = 0, mean_T = 0;
    std::vector<double> mean_Y(M, 0.0);
    for (size_t n = 0; n < N; ++n) {
        if (!(hr[n] > 0) || !(hT[n] > 0) || !std::isfinite(hr[n]) || !std::isfinite(hT[n]))
            return fail(RLBM_EINVAL, "rho and T must be finite and > 0");
        double s = 0;
        for (int a = 0; a < M; ++a) {
            const double y = hY[(size_t)a * N + n];
            if (!std::isfinite(y)) return fail(RLBM_EINVAL, "mass fractions must be finite");
            s += y;
            mean_Y[a] += y;
        }
        if (std::fabs(s - 1.0) > 1e-10) return fail(RLBM_EINVAL, "mass fractions must sum to 1 at every node");
        for (int dd = 0; dd < 3; ++dd)
            if (!std::isfinite(hu[dd * N + n])) return fail(RLBM_EINVAL, "velocity must be finite");
        mean_rho += hr[n];
        mean_T += hT[n];
    }
    mean_rho /= (double)N;
    mean_T /= (double)N;
    for (int a = 0; a < M; ++a) mean_Y[a] /= (double)N;
    if (lat->desc.slaved == -1) {
        int best = 0;
        for (int a = 1; a < M; ++a)
            if (mean_Y[a] > mean_Y[best]) best = a;
        lat->host.slaved = best;
    }
    lat->steps_done = 0;
    lat->host.parity0 = 0;
    HIP_TRY(hipMemcpyAsync(lat->d_lat, &lat->host, sizeof(LatDev), hipMemcpyHostToDevice, lat->stream), "upload");
    {
        const int rc = upload_slot_table(lat);
        if (rc) return rc;
    }
    // device staging for the fields: the second population buffer is idle now
    double* stage = (double*)lat->host.pop[1];
    HIP_TRY(hipMemcpyAsync(stage, hf.data(), nf * sizeof(double), hipMemcpyHostToDevice, lat->stream), "upload");
    double* dmeanY = stage + nf;
    HIP_TRY(hipMemcpyAsync(dmeanY, mean_Y.data(), M * sizeof(double), hipMemcpyHostToDevice, lat->stream),
            "upload");
    if (lat->storage == RLBM_STORAGE_F32_DEV)
        HIP_TRY(launch_refs(M, lat->host.weak, lat->d_lat, lat->d_ref, mean_rho, mean_T, dmeanY, lat->stream),
                "refs kernel");
    HIP_TRY(launch_init(M, lat->storage, lat->host.weak, lat->d_lat, (long long)N, stage, stage + N, stage + 4 * N,
                        stage + 5 * N, lat->stream),
            "init kernel");
    HIP_TRY(hipStreamSynchronize(lat->stream), "hipStreamSynchronize");
    lat->state_set = true;
    return RLBM_OK;
}

static int step_one(rlbm_lattice* lat, long long t) {
    const int nb_nodes = (int)((lat->geo.N + NODE_TILE - 1) / NODE_TILE);
    const int nb_if = (int)((lat->geo.if_node.size() + BC_NODES - 1) / BC_NODES);
    const int nb64 = (int)((lat->geo.N + 63) / 64);
    for (int phase = 0; phase < NPHASE; ++phase) {
        StepLaunch a;
        a.lats = lat->d_lat;
        a.blk = phase == 0 ? lat->d_blk + 2 : (phase == NPHASE - 1 ? lat->d_blk + 4 : lat->d_blk);
        a.n_lat = 1;
        a.blocks = phase == 0 ? nb_if : (phase == NPHASE - 1 ? nb64 : nb_nodes);
        a.tp = nullptr;
        a.toff = t;
        a.stream = lat->stream;
        a.schemes = 1u << lat->host.reaction;
        if (a.blocks == 0) continue;
        Timing* ev = nullptr;
        if (lat->timing >> phase & 1u) {
            if (lat->n_events == lat->events.size()) {
                Timing e{};
                HIP_TRY(hipEventCreate(&e.a), "hipEventCreate");
                if (hipEventCreate(&e.b) != hipSuccess) {
                    (void)hipEventDestroy(e.a);
                    return fail(RLBM_EHIP, "hipEventCreate failed");
                }
                lat->events.push_back(e);
            }
            ev = &lat->events[lat->n_events++];
            ev->kernel = phase;
            HIP_TRY(hipEventRecord(ev->a, lat->stream), "hipEventRecord");
        }
        HIP_TRY(launch_phase(phase, lat->M, lat->storage, lat->host.weak, a), "step kernel launch");
        if (ev) HIP_TRY(hipEventRecord(ev->b, lat->stream), "hipEventRecord");
    }
    return RLBM_OK;
}

int rlbm_step(rlbm_lattice* lat, int64_t n) {
    if (!lat) return fail(RLBM_EINVAL, "null lattice");
    if (n < 0) return fail(RLBM_EINVAL, "negative step count");
    if (!lat->state_set) return fail(RLBM_EINVAL, "rlbm_set_state has not been called");
    if (n == 0) return RLBM_OK;
    HIP_TRY(hipSetDevice(lat->device), "hipSetDevice");
    for (int64_t s = 0; s < n; ++s) {
        const int rc = step_one(lat, lat->steps_done);
        if (rc) return rc;
        lat->steps_done++;
    }
    return RLBM_OK;
}

static int check_flag(rlbm_lattice* lat) {
    int flag = 0;
    HIP_TRY(hipMemcpy(&flag, lat->d_flag, sizeof(int), hipMemcpyDeviceToHost), "read flag");
    if (flag) {
        const int zero = 0;
        HIP_TRY(hipMemcpy(lat->d_flag, &zero, sizeof(int), hipMemcpyHostToDevice), "clear flag");
        return fail(RLBM_ENONFINITE, "temperature iteration did not converge (non-physical state)");
    }
    return RLBM_OK;
}

// The population buffer the next step writes: idle between steps, so the
// host read and write paths stage through it instead of allocating.
static double* idle_buffer(const rlbm_lattice* lat) {
    return (double*)lat->host.pop[(lat->host.parity0 + lat->steps_done + 1) & 1];
}

int rlbm_read_fields(rlbm_lattice* lat, double* rho, double* u, double* T, double* Y, double* P, int on_device) {
    if (!lat) return fail(RLBM_EINVAL, "null lattice");
    if (!lat->state_set) return fail(RLBM_EINVAL, "rlbm_set_state has not been called");
    HIP_TRY(hipSetDevice(lat->device), "hipSetDevice");
    const int M = lat->M;
    const size_t N = (size_t)lat->geo.N;
    if (on_device) {
        HIP_TRY(launch_fields(M, lat->storage, lat->host.weak, lat->d_lat, (long long)N, lat->steps_done, rho, u, T, Y, P,
                              lat->stream),
                "fields kernel");
        HIP_TRY(hipStreamSynchronize(lat->stream), "hipStreamSynchronize");
        return check_flag(lat);
    }
    // (6 + M) N doubles staged in the idle population buffer, which holds
    // 27 L N s >= 27 * 3 * 4 N bytes
    double* stage = idle_buffer(lat);
    double *dr = stage, *du = dr + N, *dT = du + 3 * N, *dY = dT + N, *dP = dY + (size_t)M * N;
    hipError_t e = launch_fields(M, lat->storage, lat->host.weak, lat->d_lat, (long long)N, lat->steps_done,
                                 rho ? dr : nullptr, u ? du : nullptr, T ? dT : nullptr, Y ? dY : nullptr,
                                 P ? dP : nullptr, lat->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(lat->stream);
    if (e == hipSuccess && rho) e = hipMemcpy(rho, dr, N * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && u) e = hipMemcpy(u, du, 3 * N * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && T) e = hipMemcpy(T, dT, N * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && Y) e = hipMemcpy(Y, dY, (size_t)M * N * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && P) e = hipMemcpy(P, dP, N * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read fields");
    return check_flag(lat);
}

static int pops_io(rlbm_lattice* lat, double* buf, int on_device, int write) {
    if (!lat || !buf) return fail(RLBM_EINVAL, "null argument");
    if (!lat->state_set) return fail(RLBM_EINVAL, "rlbm_set_state has not been called");
    HIP_TRY(hipSetDevice(lat->device), "hipSetDevice");
    const size_t N = (size_t)lat->geo.N;
    if (on_device) {
        HIP_TRY(launch_pops(lat->M, lat->storage, lat->host.weak, lat->d_lat, (long long)N, 0, lat->L, lat->steps_done,
                            buf, write, lat->stream),
                "populations kernel");
        HIP_TRY(hipStreamSynchronize(lat->stream), "hipStreamSynchronize");
        return RLBM_OK;
    }
    // one stored lattice at a time (27 N doubles) through the idle
    // population buffer, which holds 27 L N s >= 27 N * 8 bytes
    double* stage = idle_buffer(lat);
    const size_t n = (size_t)Q * N;
    for (int l = 0; l < lat->L; ++l) {
        double* hb = buf + (size_t)l * n;
        hipError_t e = hipSuccess;
        if (write) e = hipMemcpyAsync(stage, hb, n * sizeof(double), hipMemcpyHostToDevice, lat->stream);
        if (e == hipSuccess)
            e = launch_pops(lat->M, lat->storage, lat->host.weak, lat->d_lat, (long long)N, l, 1, lat->steps_done, stage,
                            write, lat->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(lat->stream);
        if (e == hipSuccess && !write) e = hipMemcpy(hb, stage, n * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "populations transfer");
    }
    return RLBM_OK;
}

int rlbm_read_populations(rlbm_lattice* lat, double* buf, int on_device) { return pops_io(lat, buf, on_device, 0); }

int rlbm_write_populations(rlbm_lattice* lat, const double* buf, int on_device) {
    return pops_io(lat, const_cast<double*>(buf), on_device, 1);
}

// ---------------------------------------------------------------------------
// raw state snapshots
// ---------------------------------------------------------------------------
namespace {
constexpr uint32_t STATE_MAGIC = 0x4d424c52u;   // "RLBM"
struct StateHeader {
    uint32_t magic, version;
    int32_t M, L, storage, slaved, rss, pad;
    int64_t N, n_out;
};
struct StateLayout {
    size_t ref, pops, scale, aux, out, total;
    size_t n_ref, n_pops, n_scale, n_aux, n_out;   // bytes of each section
};
StateLayout state_layout(const rlbm_lattice* lat) {
    StateLayout s{};
    const size_t N = (size_t)lat->geo.N, L = (size_t)lat->L, M = (size_t)lat->M;
    const bool f32 = lat->storage == RLBM_STORAGE_F32_DEV;
    s.n_ref = f32 ? (L * Q + L + Q + 2) * sizeof(double) : 0;
    s.n_pops = L * Q * (size_t)lat->host.P * (f32 ? 4 : 8);
    s.n_scale = f32 ? (size_t)lat->host.rss * N * sizeof(float) : 0;
    s.n_aux = ((size_t)AUX_Y + M + 6) * N * sizeof(double);
    s.n_out = (5 + M) * (size_t)lat->geo.n_out * sizeof(double);
    size_t o = align256(sizeof(StateHeader));
    s.ref = o; o = align256(o + s.n_ref);
    s.pops = o; o = align256(o + s.n_pops);
    s.scale = o; o = align256(o + s.n_scale);
    s.aux = o; o = align256(o + s.n_aux);
    s.out = o; o = align256(o + s.n_out);
    s.total = o;
    return s;
}
}  // namespace

int rlbm_state_bytes(const rlbm_lattice* lat, size_t* bytes) {
    if (!lat || !bytes) return fail(RLBM_EINVAL, "null argument");
    *bytes = state_layout(lat).total;
    return RLBM_OK;
}

int rlbm_save_state(rlbm_lattice* lat, void* buf, int on_device) {
    if (!lat || !buf) return fail(RLBM_EINVAL, "null argument");
    if (!lat->state_set) return fail(RLBM_EINVAL, "rlbm_set_state has not been called");
    HIP_TRY(hipSetDevice(lat->device), "hipSetDevice");
    HIP_TRY(hipStreamSynchronize(lat->stream), "hipStreamSynchronize");
    (void)on_device;   // hipMemcpyDefault resolves host or device pointers
    const StateLayout sl = state_layout(lat);
    const int q = (int)((lat->host.parity0 + lat->steps_done) & 1);
    StateHeader h{STATE_MAGIC, 1u, lat->M, lat->L, lat->storage, lat->host.slaved, lat->host.rss, 0,
                  lat->geo.N, lat->geo.n_out};
    char* b = (char*)buf;
    HIP_TRY(hipMemcpy(b, &h, sizeof(h), hipMemcpyDefault), "save state");
    if (sl.n_ref) HIP_TRY(hipMemcpy(b + sl.ref, lat->d_ref, sl.n_ref, hipMemcpyDefault), "save state");
    HIP_TRY(hipMemcpy(b + sl.pops, lat->host.pop[q], sl.n_pops, hipMemcpyDefault), "save state");
    if (sl.n_scale) HIP_TRY(hipMemcpy(b + sl.scale, lat->host.rscale[q], sl.n_scale, hipMemcpyDefault), "save state");
    HIP_TRY(hipMemcpy(b + sl.aux, lat->host.aux, sl.n_aux, hipMemcpyDefault), "save state");
    if (sl.n_out) HIP_TRY(hipMemcpy(b + sl.out, lat->host.out_state, sl.n_out, hipMemcpyDefault), "save state");
    return RLBM_OK;
}

int rlbm_load_state(rlbm_lattice* lat, const void* buf, int on_device) {
    if (!lat || !buf) return fail(RLBM_EINVAL, "null argument");
    HIP_TRY(hipSetDevice(lat->device), "hipSetDevice");
    HIP_TRY(hipStreamSynchronize(lat->stream), "hipStreamSynchronize");
    (void)on_device;
    const StateLayout sl = state_layout(lat);
    const char* b = (const char*)buf;
    StateHeader h{};
    HIP_TRY(hipMemcpy(&h, b, sizeof(h), hipMemcpyDefault), "load state");
    if (h.magic != STATE_MAGIC || h.version != 1u) return fail(RLBM_EINVAL, "not a lattice state snapshot");
    if (h.M != lat->M || h.L != lat->L || h.storage != lat->storage || h.N != lat->geo.N ||
        h.n_out != lat->geo.n_out || h.rss != lat->host.rss || h.slaved < 0 || h.slaved >= lat->M + lat->host.weak ||
        (lat->host.weak && h.slaved != lat->M))
        return fail(RLBM_EINVAL, "snapshot taken on a lattice of another shape, species count or storage");
    lat->host.slaved = h.slaved;
    HIP_TRY(hipMemcpy(lat->d_lat, &lat->host, sizeof(LatDev), hipMemcpyHostToDevice), "load state");
    {
        const int rc = upload_slot_table(lat);
        if (rc) return rc;
    }
    const int q = (int)((lat->host.parity0 + lat->steps_done) & 1);
    if (sl.n_ref) HIP_TRY(hipMemcpy(lat->d_ref, b + sl.ref, sl.n_ref, hipMemcpyDefault), "load state");
    HIP_TRY(hipMemcpy(lat->host.pop[q], b + sl.pops, sl.n_pops, hipMemcpyDefault), "load state");
    if (sl.n_scale) HIP_TRY(hipMemcpy(lat->host.rscale[q], b + sl.scale, sl.n_scale, hipMemcpyDefault), "load state");
    HIP_TRY(hipMemcpy(lat->host.aux, b + sl.aux, sl.n_aux, hipMemcpyDefault), "load state");
    if (sl.n_out) HIP_TRY(hipMemcpy(lat->host.out_state, b + sl.out, sl.n_out, hipMemcpyDefault), "load state");
    lat->state_set = true;
    return RLBM_OK;
}

int rlbm_invariants(rlbm_lattice* lat, double* out, int n_out) {
    if (!lat || !out) return fail(RLBM_EINVAL, "null argument");
    if (!lat->state_set) return fail(RLBM_EINVAL, "rlbm_set_state has not been called");
    const int nv = 6 + lat->E;
    if (n_out < nv) return fail(RLBM_EINVAL, "output array too small (needs 6 + E)");
    HIP_TRY(hipSetDevice(lat->device), "hipSetDevice");
    HIP_TRY(launch_invariants(lat->M, lat->storage, lat->host.weak, lat->d_lat, lat->geo.N, lat->steps_done,
                              lat->d_partial, nv,
                              lat->d_invout, lat->stream),
            "invariants kernel");
    HIP_TRY(hipStreamSynchronize(lat->stream), "hipStreamSynchronize");
    HIP_TRY(hipMemcpy(out, lat->d_invout, nv * sizeof(double), hipMemcpyDeviceToHost), "read invariants");
    return RLBM_OK;
}

int rlbm_set_timing(rlbm_lattice* lat, int enable) {
    if (!lat) return fail(RLBM_EINVAL, "null lattice");
    lat->timing = (unsigned)enable & ((1u << NPHASE) - 1u);
    return RLBM_OK;
}

int rlbm_kernel_times(rlbm_lattice* lat, double* ms, int64_t* counts, int n) {
    if (!lat) return fail(RLBM_EINVAL, "null lattice");
    HIP_TRY(hipStreamSynchronize(lat->stream), "hipStreamSynchronize");
    for (size_t j = 0; j < lat->n_events; ++j) {
        const Timing& e = lat->events[j];
        float t = 0;
        HIP_TRY(hipEventElapsedTime(&t, e.a, e.b), "hipEventElapsedTime");
        lat->ms[e.kernel] += t;
        lat->counts[e.kernel] += 1;
    }
    lat->n_events = 0;
    for (int k = 0; k < n && k < NPHASE; ++k) {
        if (ms) ms[k] = lat->ms[k];
        if (counts) counts[k] = lat->counts[k];
        lat->ms[k] = 0;
        lat->counts[k] = 0;
    }
    return RLBM_OK;
}

int rlbm_lattice_status(rlbm_lattice* lat, int32_t* status) {
    if (!lat || !status) return fail(RLBM_EINVAL, "null argument");
    HIP_TRY(hipSetDevice(lat->device), "hipSetDevice");
    HIP_TRY(hipStreamSynchronize(lat->stream), "hipStreamSynchronize");
    int flag = 0;
    HIP_TRY(hipMemcpy(&flag, lat->d_flag, sizeof(int), hipMemcpyDeviceToHost), "read flag");
    if (flag) {
        const int zero = 0;
        HIP_TRY(hipMemcpy(lat->d_flag, &zero, sizeof(int), hipMemcpyHostToDevice), "clear flag");
    }
    *status = flag;
    return RLBM_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
namespace {
// Device memory of a batch: the step counter of the launch series, the
// lattice table and the block prefixes (uploaded together at every step
// call), then the lattices' flag pointers (uploaded once) and the gathered
// flags.
struct BatchPlan {
    size_t off_t, off_table, off_blk, upload, off_flagp, off_status, total;
};
BatchPlan batch_plan(int k) {
    BatchPlan p{};
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
    p.off_t = take(sizeof(long long));
    p.off_table = take((size_t)k * sizeof(LatDev));
    p.off_blk = take(3 * (size_t)(k + 1) * sizeof(int));
    p.upload = o;
    p.off_flagp = take((size_t)k * sizeof(int*));
    p.off_status = take((size_t)k * sizeof(int));
    p.total = o;
    return p;
}
// Steps per captured chunk of a batch.
constexpr int BATCH_CHUNK = 16;
constexpr int BATCH_RING = 2;
}  // namespace

}  // extern "C"

struct rlbm_batch {
    std::vector<rlbm_lattice*> lats;
    BatchPlan plan{};
    char* base = nullptr;
    int device = 0;
    bool stepped = false;                       // `done` has been recorded
    hipStream_t stream = nullptr;               // the first lattice's stream
    std::vector<hipStream_t> others;            // the other lattices' distinct streams
    std::vector<hipEvent_t> other_ev;           // their work before a batch step
    hipEvent_t done = nullptr;                  // the batch step's work, for the other streams
    char* pinned[BATCH_RING] = {nullptr, nullptr};   // host staging of the per-call upload
    hipEvent_t slot_ev[BATCH_RING] = {nullptr, nullptr};
    bool slot_used[BATCH_RING] = {false, false};
    int next_slot = 0;
    int* pinned_status = nullptr;
    int nb[3] = {0, 0, 0};                      // node, interface and 64-node blocks of all lattices
    unsigned schemes = 0;
    std::vector<int> host_blk;
    bool graphs = true;
    hipStream_t cap = nullptr;                  // private stream for graph capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void batch_free(rlbm_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (auto e : b->other_ev) (void)hipEventDestroy(e);
    if (b->done) (void)hipEventDestroy(b->done);
    for (int r = 0; r < BATCH_RING; ++r) {
        if (b->slot_ev[r]) (void)hipEventDestroy(b->slot_ev[r]);
        if (b->pinned[r]) (void)hipHostFree(b->pinned[r]);
    }
    if (b->pinned_status) (void)hipHostFree(b->pinned_status);
    delete b;
}

// Launches of steps t = *tp + toff0 .. *tp + toff0 + n - 1 of every lattice
// of the batch (a lattice is active while t < its t_end).
static hipError_t batch_launch(rlbm_batch* b, hipStream_t st, long long toff0, long long n) {
    const int k = (int)b->lats.size();
    rlbm_lattice* l0 = b->lats[0];
    const long long* tp = (const long long*)(b->base + b->plan.off_t);
    const LatDev* table = (const LatDev*)(b->base + b->plan.off_table);
    const int* blk = (const int*)(b->base + b->plan.off_blk);
    for (long long t = toff0; t < toff0 + n; ++t) {
        for (int phase = 0; phase < NPHASE; ++phase) {
            StepLaunch a;
            a.lats = table;
            a.blk = phase == 0 ? blk + (k + 1) : (phase == NPHASE - 1 ? blk + 2 * (k + 1) : blk);
            a.n_lat = k;
            a.blocks = phase == 0 ? b->nb[1] : (phase == NPHASE - 1 ? b->nb[2] : b->nb[0]);
            a.tp = tp;
            a.toff = t;
            a.stream = st;
            a.schemes = b->schemes;
            if (a.blocks == 0) continue;
            const hipError_t e = launch_phase(phase, l0->M, l0->storage, l0->host.weak, a);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// Captures BATCH_CHUNK steps and the counter advance as one graph.
static int batch_capture(rlbm_batch* b) {
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
    hipError_t e = batch_launch(b, b->cap, 0, BATCH_CHUNK);
    if (e == hipSuccess) e = launch_advance_time((long long*)(b->base + b->plan.off_t), BATCH_CHUNK, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e, "batch capture");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    b->graph = g;
    b->exec = x;
    return RLBM_OK;
}

extern "C" {

int rlbm_batch_bytes(int32_t k, size_t* bytes) {
    if (k < 1 || !bytes) return fail(RLBM_EINVAL, "batch needs k >= 1");
    *bytes = batch_plan(k).total;
    return RLBM_OK;
}

int rlbm_batch_create(rlbm_lattice* const* lats, int32_t k, void* dev_mem, size_t bytes, rlbm_batch** out) {
    if (!lats || k < 1 || !dev_mem || !out) return fail(RLBM_EINVAL, "null argument or k < 1");
    *out = nullptr;
    const BatchPlan plan = batch_plan(k);
    if (bytes < plan.total) return fail(RLBM_ENOSPC, "device buffer smaller than rlbm_batch_bytes");
    if (((uintptr_t)dev_mem & 255) != 0) return fail(RLBM_EINVAL, "device memory must be 256-byte aligned");
    for (int j = 0; j < k; ++j) {
        if (!lats[j]) return fail(RLBM_EINVAL, "null lattice in batch");
        if (lats[j]->M != lats[0]->M || lats[j]->storage != lats[0]->storage || lats[j]->device != lats[0]->device ||
            lats[j]->host.weak != lats[0]->host.weak)
            return fail(RLBM_EINVAL, "batched lattices need the same species count, storage and device");
        for (int i = 0; i < j; ++i)
            if (lats[i] == lats[j]) return fail(RLBM_EINVAL, "a lattice appears twice in the batch");
    }
    HIP_TRY(hipSetDevice(lats[0]->device), "hipSetDevice");
    rlbm_batch* b = new (std::nothrow) rlbm_batch();
    if (!b) return fail(RLBM_EINVAL, "out of host memory");
    b->lats.assign(lats, lats + k);
    b->plan = plan;
    b->base = (char*)dev_mem;
    b->device = lats[0]->device;
    b->stream = lats[0]->stream;
    auto bail = [&](hipError_t e, const char* what) {
        batch_free(b);
        return hip_fail(e, what);
    };
    hipError_t e;
    for (int j = 1; j < k; ++j) {
        const hipStream_t sj = lats[j]->stream;
        if (sj == b->stream || std::find(b->others.begin(), b->others.end(), sj) != b->others.end()) continue;
        hipEvent_t ev = nullptr;
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return bail(e, "hipEventCreate");
        b->others.push_back(sj);
        b->other_ev.push_back(ev);
    }
    if ((e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming)) != hipSuccess) return bail(e, "hipEventCreate");
    for (int r = 0; r < BATCH_RING; ++r) {
        if ((e = hipEventCreateWithFlags(&b->slot_ev[r], hipEventDisableTiming)) != hipSuccess)
            return bail(e, "hipEventCreate");
        if ((e = hipHostMalloc((void**)&b->pinned[r], plan.upload, hipHostMallocDefault)) != hipSuccess)
            return bail(e, "hipHostMalloc");
    }
    if ((e = hipHostMalloc((void**)&b->pinned_status, (size_t)k * sizeof(int), hipHostMallocDefault)) != hipSuccess)
        return bail(e, "hipHostMalloc");
    if ((e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess) return bail(e, "hipStreamCreate");
    // every lattice takes part in every launch (a lattice without steps in a
    // call returns at once), so the grids, and with them a captured chunk,
    // stay the same from call to call
    b->host_blk.assign(3 * (k + 1), 0);
    std::vector<int*> flagp(k);
    for (int j = 0; j < k; ++j) {
        const rlbm_lattice* lat = lats[j];
        b->schemes |= 1u << lat->host.reaction;
        b->host_blk[j + 1] = b->host_blk[j] + (int)((lat->geo.N + NODE_TILE - 1) / NODE_TILE);
        b->host_blk[(k + 1) + j + 1] =
            b->host_blk[(k + 1) + j] + (int)((lat->geo.if_node.size() + BC_NODES - 1) / BC_NODES);
        b->host_blk[2 * (k + 1) + j + 1] = b->host_blk[2 * (k + 1) + j] + (int)((lat->geo.N + 63) / 64);
        flagp[j] = lat->d_flag;
    }
    b->nb[0] = b->host_blk[k];
    b->nb[1] = b->host_blk[2 * (k + 1) - 1];
    b->nb[2] = b->host_blk[3 * (k + 1) - 1];
    if ((e = hipMemcpy(b->base + plan.off_flagp, flagp.data(), (size_t)k * sizeof(int*), hipMemcpyHostToDevice)) !=
        hipSuccess)
        return bail(e, "upload batch table");
    *out = b;
    return RLBM_OK;
}

int rlbm_batch_step(rlbm_batch* b, const int64_t* steps) {
    if (!b || !steps) return fail(RLBM_EINVAL, "null argument");
    const int k = (int)b->lats.size();
    long long tmax = 0;
    for (int j = 0; j < k; ++j) {
        if (steps[j] < 0) return fail(RLBM_EINVAL, "negative step count");
        if (!b->lats[j]->state_set) return fail(RLBM_EINVAL, "rlbm_set_state has not been called");
        tmax = std::max<long long>(tmax, steps[j]);
    }
    if (tmax == 0) return RLBM_OK;
    HIP_TRY(hipSetDevice(b->device), "hipSetDevice");
    // host staging slot: free once the copy that last read it has run
    const int r = b->next_slot;
    if (b->slot_used[r]) HIP_TRY(hipEventSynchronize(b->slot_ev[r]), "hipEventSynchronize");
    char* up = b->pinned[r];
    *(long long*)(up + b->plan.off_t) = 0;
    LatDev* tab = (LatDev*)(up + b->plan.off_table);
    for (int j = 0; j < k; ++j) {
        const rlbm_lattice* lat = b->lats[j];
        LatDev e = lat->host;
        e.parity0 = (int)((lat->host.parity0 + lat->steps_done) & 1);
        e.t_end = steps[j];
        tab[j] = e;
    }
    std::memcpy(up + b->plan.off_blk, b->host_blk.data(), b->host_blk.size() * sizeof(int));
    // order after the work already queued on the lattices' own streams
    for (size_t q = 0; q < b->others.size(); ++q) {
        HIP_TRY(hipEventRecord(b->other_ev[q], b->others[q]), "hipEventRecord");
        HIP_TRY(hipStreamWaitEvent(b->stream, b->other_ev[q], 0), "hipStreamWaitEvent");
    }
    HIP_TRY(hipMemcpyAsync(b->base, up, b->plan.upload, hipMemcpyHostToDevice, b->stream), "upload batch table");
    HIP_TRY(hipEventRecord(b->slot_ev[r], b->stream), "hipEventRecord");
    b->slot_used[r] = true;
    b->next_slot = (r + 1) % BATCH_RING;
    // whole chunks replay the captured graph; the rest are direct launches
    long long full = b->graphs ? tmax / BATCH_CHUNK : 0;
    if (full > 0 && !b->exec) {
        const int rc = batch_capture(b);
        if (rc) return rc;
    }
    for (long long c = 0; c < full; ++c) HIP_TRY(hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
    HIP_TRY(batch_launch(b, b->stream, 0, tmax - full * BATCH_CHUNK), "batch kernel launch");
    HIP_TRY(hipEventRecord(b->done, b->stream), "hipEventRecord");
    b->stepped = true;
    for (size_t q = 0; q < b->others.size(); ++q)
        HIP_TRY(hipStreamWaitEvent(b->others[q], b->done, 0), "hipStreamWaitEvent");
    for (int j = 0; j < k; ++j) b->lats[j]->steps_done += steps[j];
    return RLBM_OK;
}

int rlbm_batch_status(rlbm_batch* b, int32_t* status) {
    if (!b || !status) return fail(RLBM_EINVAL, "null argument");
    const int k = (int)b->lats.size();
    HIP_TRY(hipSetDevice(b->device), "hipSetDevice");
    // the lattices' own streams may hold work of their own
    for (size_t q = 0; q < b->others.size(); ++q) {
        HIP_TRY(hipEventRecord(b->other_ev[q], b->others[q]), "hipEventRecord");
        HIP_TRY(hipStreamWaitEvent(b->stream, b->other_ev[q], 0), "hipStreamWaitEvent");
    }
    int* d_status = (int*)(b->base + b->plan.off_status);
    HIP_TRY(launch_gather_flags((int* const*)(b->base + b->plan.off_flagp), k, d_status, b->stream), "flags kernel");
    HIP_TRY(hipMemcpyAsync(b->pinned_status, d_status, (size_t)k * sizeof(int), hipMemcpyDeviceToHost, b->stream),
            "read flags");
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    for (int j = 0; j < k; ++j) status[j] = b->pinned_status[j];
    return RLBM_OK;
}

int rlbm_step_group(rlbm_lattice* const* lats, int32_t k, const int64_t* steps) {
    if (!lats || !steps) return fail(RLBM_EINVAL, "null argument");
    if (k < 1 || k > RLBM_GROUP_MAX_LATTICES)
        return fail(RLBM_EINVAL, "group needs 1 <= k <= RLBM_GROUP_MAX_LATTICES lattices");
    long long tmax = 0;
    for (int j = 0; j < k; ++j) {
        const rlbm_lattice* lat = lats[j];
        if (!lat) return fail(RLBM_EINVAL, "null lattice in group");
        if (!lat->state_set) return fail(RLBM_EINVAL, "rlbm_set_state has not been called");
        if (lat->M != lats[0]->M || lat->storage != lats[0]->storage || lat->device != lats[0]->device ||
            lat->host.weak != lats[0]->host.weak || lat->stream != lats[0]->stream)
            return fail(RLBM_EINVAL, "grouped lattices need the same species count, storage, device and stream");
        for (int i = 0; i < j; ++i)
            if (lats[i] == lat) return fail(RLBM_EINVAL, "a lattice appears twice in the group");
        if (steps[j] < 0) return fail(RLBM_EINVAL, "negative step count");
        tmax = std::max<long long>(tmax, steps[j]);
    }
    if (tmax == 0) return RLBM_OK;
    rlbm_lattice* l0 = lats[0];
    HIP_TRY(hipSetDevice(l0->device), "hipSetDevice");
    char* sc = nullptr;
    HIP_TRY(group_scratch(l0->device, &sc), "hipGetSymbolAddress");
    // the table, filled on the device from the lattices' own entries in
    // chunks whose data travel as kernel arguments
    int pre[3] = {0, 0, 0};
    unsigned schemes = 0;
    for (int base = 0; base < k; base += GROUP_CHUNK) {
        GroupChunk c;
        std::memset(&c, 0, sizeof(c));
        c.base = base;
        c.n = std::min(GROUP_CHUNK, k - base);
        c.k = k;
        for (int j = 0; j <= c.n; ++j) {
            for (int a = 0; a < 3; ++a) c.blk[a][j] = pre[a];
            if (j == c.n) break;
            const rlbm_lattice* lat = lats[base + j];
            c.src[j] = lat->d_lat;
            c.t_end[j] = steps[base + j];
            c.parity[j] = (int)((lat->host.parity0 + lat->steps_done) & 1);
            schemes |= 1u << lat->host.reaction;
            pre[0] += (int)((lat->geo.N + NODE_TILE - 1) / NODE_TILE);
            pre[1] += (int)((lat->geo.if_node.size() + BC_NODES - 1) / BC_NODES);
            pre[2] += (int)((lat->geo.N + 63) / 64);
        }
        HIP_TRY(launch_group_gather(sc, c, l0->stream), "group table kernel");
    }
    const LatDev* table = (const LatDev*)(sc + GROUP_OFF_TABLE);
    const int* blk = (const int*)(sc + GROUP_OFF_BLK);
    for (long long t = 0; t < tmax; ++t) {
        for (int phase = 0; phase < NPHASE; ++phase) {
            StepLaunch a;
            a.lats = table;
            a.blk = phase == 0 ? blk + (k + 1) : (phase == NPHASE - 1 ? blk + 2 * (k + 1) : blk);
            a.n_lat = k;
            a.blocks = phase == 0 ? pre[1] : (phase == NPHASE - 1 ? pre[2] : pre[0]);
            a.tp = (const long long*)sc;
            a.toff = t;
            a.stream = l0->stream;
            a.schemes = schemes;
            if (a.blocks == 0) continue;
            HIP_TRY(launch_phase(phase, l0->M, l0->storage, l0->host.weak, a), "group kernel launch");
        }
    }
    for (int j = 0; j < k; ++j) lats[j]->steps_done += steps[j];
    return RLBM_OK;
}

void rlbm_batch_destroy(rlbm_batch* b) {
    if (!b) return;
    // the batch's last launches read its tables and the pinned staging its
    // copies: wait for them through the batch's own events (the lattices
    // and their streams may already be gone)
    if (hipSetDevice(b->device) == hipSuccess) {
        if (b->stepped) (void)hipEventSynchronize(b->done);
        for (int r = 0; r < BATCH_RING; ++r)
            if (b->slot_used[r]) (void)hipEventSynchronize(b->slot_ev[r]);
    }
    batch_free(b);
    (void)hipGetLastError();   // leave no error of this teardown for the next call
}

}  // extern "C"
