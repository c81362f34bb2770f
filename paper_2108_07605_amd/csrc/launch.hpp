// Kernel launchers shared by the host library (kernels.hip implements them).
#pragma once

#include <hip/hip_runtime.h>

#include "physics.hpp"

namespace rlbm {

// One launch of a step phase over a work list of n_lat lattices.
struct StepLaunch {
    const LatDev* lats;   // device table [n_lat]
    const int* blk;       // device prefix of blocks per lattice [n_lat + 1]
    int n_lat;
    int blocks;           // total blocks (blk[n_lat])
    const long long* tp;  // device step counter of the launch series, or NULL (counter 0)
    long long toff;       // step of this launch: *tp + toff
    hipStream_t stream;
    unsigned schemes;     // bit r set if a lattice uses RLBM_REACTION r (phase 2 launches one kernel per scheme)
};

// Interface nodes per boundary block (one wave, one lane per node).
constexpr int BC_NODES = 64;

// Nodes per block of the moments and gradient phases, one thread per node.
#ifndef RLBM_NODE_TILE
#define RLBM_NODE_TILE 64
#endif
constexpr int NODE_TILE = RLBM_NODE_TILE;

// phase 0: boundary (BC_NODES interface nodes per block); phases 1 and 2:
// moments, diffusion and forward-Euler chemistry, then gradients (with the
// linearly implicit chemistry first where selected) (NODE_TILE-thread blocks
// over nodes); phase 3: update (one block per 64 nodes).
hipError_t launch_phase(int phase, int M, int storage, int weak, const StepLaunch& a);
// weak: the weakly coupled storage (all M species lattices, no slaved species)
hipError_t launch_init(int M, int storage, int weak, const LatDev* lat, long long N, const double* rho,
                       const double* u, const double* T, const double* Y, hipStream_t st);
hipError_t launch_refs(int M, int weak, const LatDev* lat, double* ref, double rho, double T, const double* Y,
                       hipStream_t st);
hipError_t launch_fields(int M, int storage, int weak, const LatDev* lat, long long N, long long t, double* rho,
                         double* u, double* T, double* Y, double* P, hipStream_t st);
hipError_t launch_pops(int M, int storage, int weak, const LatDev* lat, long long N, int l0, int nl, long long t,
                       double* buf, int write, hipStream_t st);
hipError_t launch_invariants(int M, int storage, int weak, const LatDev* lat, long long N, long long t,
                             double* partial, int nv, double* out, hipStream_t st);
// batched steps: advance the device step counter; read and clear k flags
hipError_t launch_advance_time(long long* tp, long long n, hipStream_t st);
hipError_t launch_gather_flags(int* const* flags, int k, int* out, hipStream_t st);
bool species_supported(int M);

// Allocation-free group steps (rlbm_step_group): at most GROUP_MAX lattices,
// their table in a file-scope device array of the kernel library.
constexpr int GROUP_MAX = RLBM_GROUP_MAX_LATTICES;
constexpr int GROUP_CHUNK = 32;   // table entries filled per gather launch (kernel arguments)
struct GroupChunk {
    const LatDev* src[GROUP_CHUNK];   // the lattices' device entries
    long long t_end[GROUP_CHUNK];     // steps of this call
    int parity[GROUP_CHUNK];          // buffer holding the current populations
    int blk[3][GROUP_CHUNK + 1];      // node, interface and 64-node block prefixes of entries base..base+n
    int base, n, k;
};
// Layout of the group scratch: the step counter, the lattice table
// [GROUP_MAX] and the three block prefixes [GROUP_MAX + 1] each.
constexpr size_t GROUP_OFF_TABLE = 256;
constexpr size_t GROUP_OFF_BLK = GROUP_OFF_TABLE + (((size_t)GROUP_MAX * sizeof(LatDev) + 255) & ~(size_t)255);
constexpr size_t GROUP_SCRATCH_BYTES =
    GROUP_OFF_BLK + (((size_t)3 * (GROUP_MAX + 1) * sizeof(int) + 255) & ~(size_t)255);
// Device address of the group scratch on `device` (the current device),
// looked up once per device.
hipError_t group_scratch(int device, char** ptr);
hipError_t launch_group_gather(char* sc, const GroupChunk& c, hipStream_t st);

}  // namespace rlbm
