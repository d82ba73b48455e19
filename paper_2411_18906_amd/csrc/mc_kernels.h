// Launchers of the pyhea kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "geometry.h"

namespace pyhea {

// LDS layout of the MC kernel (must match the carve order in mc_kernels.hip).
// W = wavefronts per slot group (>= S), bal = offsets spread evenly over them
// (partial histograms exchanged through LDS), K = steps whose candidates one
// pass evaluates (records for K * B slots), CH = members of the conflict-free
// set the speculative commit phase evaluates together (0: one by one; <= 16).
__host__ __device__ inline int mc_lds_bytes(int S, int M, int B, int W = 0, int bal = 0, int K = 1, int CH = 0) {
    auto r = [](int b) { return (b + 15) & ~15; };
    const int E = S * M * M;
    const int Bt = K * B;
    int n = 0;
    n += r(E * 32);                               // entry records
    n += r(kMaxOffsets * 16) + r(kMaxOffsets * 4);     // dlin4, offmod
    n += r(Bt * 8) + 3 * r(Bt * 4);               // rec_dS, pp, pq, ab
    n += 2 * r(S * Bt * (M > 6 ? 8 : 4));         // rec_cp, rec_cq (histograms)
    n += r(S * Bt * 8);                           // rec_dQ
    n += 2 * r(Bt * 4);                           // order, list (per step of a pass)
    n += r(2 * kMaxShells * 8) + r(32 * 4);       // sh_dQ (two buffers), sh_int
    if (bal) n += r(S * W * 2 * Bt * (M > 6 ? 8 : 4));  // partial histograms
    if (CH > 0) n += r(64 * 8) + r(CH * E * 8) + r(CH * E * 4) + r(16 * kMaxShells * 8) + r(16 * 4) + r(4 * 4);
    return n;
}

// bytes of the species store for a padded chain
inline int64_t species_store_bytes(int store, int64_t Npad) {
    if (store == kStoreLds8) return (Npad + 15) & ~int64_t(15);
    if (store == kStoreLds4) return (((Npad + 7) / 8) * 4 + 15) & ~int64_t(15);
    return 0;
}

// Raises a kernel's dynamic LDS limit to at least `lds` bytes on the current
// device; remembers what it set, so repeated launches make no runtime call.
hipError_t set_max_lds(const void *fn, size_t lds);

// Wavefronts of one chain's block: K steps x slot groups x W.
inline int mc_block_waves(int B, int W, int K) { return K * ((B + 63) / 64) * W; }
int mc_block_threads(int B, int W, int K);
constexpr int kMaxLookahead = 8;

// One launch of n_chains chains (one block each) for up to max_steps steps.
hipError_t launch_mc(const ChainDesc *descs_dev, int n_chains, int store, int M, int S, int B, int W, int bal,
                     int K, int CH, int lds_bytes, int max_steps, hipStream_t stream);
// Ratio tables of chains from their initial counts (descriptor order; bad [n]
// the invalid-id flags in the same order); invalid chains get status EINVAL.
hipError_t launch_chain_ratio(const ChainDesc *descs_dev, int n_chains, const int32_t *bad, hipStream_t stream);
hipError_t launch_pad_fill(const ChainDesc *descs_dev, int n_chains, hipStream_t stream);
hipError_t launch_pad_drain(const ChainDesc *descs_dev, int n_chains, hipStream_t stream);
// out[i] = *descs_dev[i].state (device array of n_chains states).
hipError_t launch_gather_states(const ChainDesc *descs_dev, int n_chains, ChainState *out, hipStream_t stream);
// S and F of every chain's maintained counts into its state (Eq. 2-3).
hipError_t launch_final_objective(const ChainDesc *descs_dev, int n_chains, hipStream_t stream);

// Full evaluation: pair counts of K configurations of one geometry.
struct EvalDesc {
    int32_t A, lgA, Lx, Ly, Lz, M, S;
    int32_t n_half;                       // offsets with one of each +-d pair
    int32_t z0;                           // coordination number of shell 1
    int32_t zk[kMaxShells];
    double inv_Lx, inv_Ly;
    uint32_t N;
    int32_t Z;                            // all offsets of shells 1..S
    // per (basis, half offset): dcx, dcy, dcz, target basis, shell (int8 each)
    int8_t half[4][kMaxOffsets / 2][5];
    int8_t off[kMaxOffsets][4];           // dx, dy, dz, shell (half units)
};

void fill_eval_desc(const Geometry &g, EvalDesc *d);

// One configuration of a many-chain count launch (each its own geometry).
struct CountTask {
    EvalDesc ed;
    const int8_t *species;  // N sites, unpadded
    int32_t *counts;        // [S][M][M], zero before the launch
    int32_t *bad;           // set to 1 if a species id lies outside [0, M); zero before the launch
};
// Sites per workgroup of the many-configuration count: 2048, halved (down to
// 256) while the launch would have fewer than 2048 workgroups, so that a few
// small configurations still spread over the chip.
inline uint32_t count_tile_for(uint64_t total_sites) {
    uint32_t tile = 2048;
    while (tile > 256 && total_sites < (uint64_t)tile * 2048) tile >>= 1;
    return tile;
}
inline uint32_t count_tiles(uint32_t N, uint32_t tile) { return (N + tile - 1) / tile; }

// Pair counts of n configurations with different geometries in one launch.
// tile0[c] = first tile of task c (prefix sums of count_tiles(N, tile)),
// n_tiles = total; max_E = the largest S M M of the tasks (LDS histograms).
hipError_t launch_count_tasks(const CountTask *tasks, const uint32_t *tile0, int n, uint32_t n_tiles, uint32_t tile,
                              int max_E, hipStream_t stream);

hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t stream);

// Target and weight tables (at most S M M + S doubles) copied to the device by a
// kernel whose arguments carry them: stream-ordered, and the host never waits.
constexpr int kMaxTable = kMaxShells * kMaxSpecies * kMaxSpecies + kMaxShells;
struct SmallTable {
    double v[kMaxTable];
};
hipError_t launch_upload(const SmallTable &t, int n, double *dst, hipStream_t stream);

hipError_t launch_count_gather(const EvalDesc &ed, int64_t K, const int8_t *species,
                               int32_t *counts, int32_t *bad, hipStream_t stream);
// alpha (optional, [K][S][M][M]) and, with a target, S_F [K][2] from counts.
hipError_t launch_objective_epilogue(const EvalDesc &ed, int64_t K, const int32_t *counts,
                                     const int32_t *bad, const double *target, const double *weight,
                                     double *S_F, double *alpha, hipStream_t stream);
hipError_t launch_trial_eval(const EvalDesc &ed, const int8_t *species, const int32_t *counts,
                             const double *target, const double *weight, int64_t n_pairs,
                             const int32_t *pairs, double *dS, int32_t *dN, hipStream_t stream);
// Non-incremental baseline: out[i] = base with sites pairs[i] swapped (out
// [n][N]); *bad |= 1 for a pair outside [0, N).  dS[i] = S_F[i][0] - S0[0].
hipError_t launch_swap_copies(const int8_t *base, int64_t N, const int32_t *pairs, int n, int8_t *out, int32_t *bad,
                              hipStream_t stream);
hipError_t launch_sub_objective(const double *S_F, const double *S0, int n, double *dS, hipStream_t stream);

// Random solutions of the global search: configuration c of n_configs is pool
// slot d.slot0 + c (out [n_configs][N]); d.prefix[j] = sum of the first j
// species counts (prefix[M] = N).
struct RandomConfigDesc {
    uint64_t seed;
    uint32_t iteration;
    uint32_t slot0;
    int32_t M;
    uint32_t prefix[9];
};
hipError_t launch_random_configs(uint32_t N, const RandomConfigDesc &d, int n_configs, int8_t *out,
                                 hipStream_t stream);

hipError_t launch_philox(const uint32_t *ctr, uint64_t seed, int64_t n, uint32_t *out,
                         hipStream_t stream);

}  // namespace pyhea
