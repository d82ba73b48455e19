// Lattice geometry and device-side descriptors of the pyhea library.
//
// Positions are in half lattice constants.  A site is 2*cell + basis_b with the
// FCC basis {(0,0,0),(1,1,0),(1,0,1),(0,1,1)} or the BCC basis {(0,0,0),(1,1,1)}
// (S = A L^3 sites, Sec. 2.2 and the Table 1 caption).  Shell k holds the lattice
// vectors of the k-th smallest length (squared radii FCC 2, 4, 6, 8 and BCC 3,
// 4, 8, 11 in these units; coordination 12, 6, 24, 12 and 8, 6, 12, 24).
//
// Kernels never stream a neighbour list: each site id is turned into cell
// coordinates and every neighbour is reached by adding a per-(basis, offset)
// linear delta in a halo-padded copy of the configuration, so no modulo is
// evaluated per neighbour.
#pragma once

#include <stdint.h>

#include <string>

#include "pyhea.h"

namespace pyhea {

constexpr int kMaxShells = 4;
constexpr int kMaxSpecies = 8;
constexpr int kMaxOffsets = 56;  // FCC shells 1-4: 54, BCC: 50
constexpr int kMaxB = 256;       // trial swaps per step
constexpr int kWave = 64;

struct Geometry {
    int lattice = 0;
    int A = 4;      // sites per conventional cell
    int lgA = 2;    // log2(A)
    int L[3] = {0, 0, 0};
    int M = 0, S = 0;
    int Z = 0;                       // offsets in shells 1..S
    int z[kMaxShells] = {0};         // coordination numbers
    int r2[kMaxShells] = {0};        // squared radii (half units)
    int zstart[kMaxShells + 1] = {0};
    int8_t off[kMaxOffsets][3] = {};  // offsets, shell by shell
    int halo = 1;                    // largest |cell delta| of any (basis, offset)
    int small_cell = 0;              // some axis too short for the min-image shortcut
    int64_t N = 0;
    int P[3] = {0, 0, 0};            // padded cells per axis (L + 2 halo)
    int64_t Npad = 0;                // padded sites
};

// Fills `g` from a descriptor.  Returns PYHEA_OK or PYHEA_EINVAL with a message.
pyhea_status build_geometry(const pyhea_lattice *lat, Geometry *g, std::string *err);

// Basis vector b of a lattice (half units).
void basis_vector(int lattice, int b, int out[3]);

// Cell delta and target basis of offset t from basis b.
void offset_target(const Geometry &g, int b, int t, int dc[3], int *b_to);

// Linear delta in the padded layout for (basis b, offset t).
int32_t padded_delta(const Geometry &g, int b, int t);

// ---------------------------------------------------------------------------
// Device descriptors
// ---------------------------------------------------------------------------

// Mutable per-chain state kept in device memory between launches.
struct ChainState {
    int64_t trials;
    int64_t null_trials;
    int64_t commits;
    int64_t steps;
    int32_t depth;
    int32_t stop_reason;
    int32_t done;
    int32_t status;
    double S, F;   // objective of the final counts (Eq. 3), written after the run
};

enum SpeciesStore : int32_t {
    kStoreLds8 = 0,    // padded configuration in LDS, one byte per site
    kStoreLds4 = 1,    // padded configuration in LDS, one nibble per site
    kStoreGlobal = 2,  // padded configuration in HBM (one byte per site)
};

// Everything one chain needs on the device.  Read-only for kernels except the
// buffers it points to.
struct ChainDesc {
    int32_t A, lgA, Lx, Ly, Lz, M, S, Z;
    int32_t halo, PX, PY, PZ;
    int32_t small_cell;
    int32_t zk[kMaxShells];
    int32_t zstart[kMaxShells + 1];
    int32_t r2[kMaxShells];
    uint32_t N;
    uint32_t Npad;
    double inv_Lx, inv_Ly;          // 1/Lx, 1/Ly for exact small-integer division
    int8_t off[kMaxOffsets][4];     // dx, dy, dz, shell
    int32_t dlin[4][kMaxOffsets];   // padded linear delta per (basis, offset)
    int32_t off_mod[kMaxOffsets];   // offsets reduced mod the box, packed 10 bits/axis
    uint64_t seed;
    uint32_t chain_id;
    int32_t B;
    int64_t n_trials;
    int32_t mode;
    int32_t depth_limit;
    double tau;
    double w[kMaxShells];
    int8_t *species;       // [N] unpadded configuration, in/out
    int8_t *pad_global;    // [Npad] padded copy when store == kStoreGlobal
    const double *R;       // [S][M][M]
    const double *target;  // [S][M][M]
    int32_t *counts;       // [S][M][M] maintained pair counts, in/out
    uint32_t *log;         // [log_cap][4] or null
    int64_t log_cap;
    ChainState *state;
    int32_t store;
    int32_t lds_bytes;     // LDS needed by this chain
    int32_t sym;           // 1 if target[k][i][j] == target[k][j][i] bit for bit
};

// 1 if a [S][M][M] target table equals its transpose bit for bit.
int symmetric_target(const double *t, int S, int M);

// Fills the geometry part of a ChainDesc.
void fill_chain_geometry(const Geometry &g, ChainDesc *d);

}  // namespace pyhea
