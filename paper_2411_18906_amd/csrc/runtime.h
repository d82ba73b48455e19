// Host runtime shared by the C ABI entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "geometry.h"
#include "mc_kernels.h"

namespace pyhea {

void set_error(const std::string &msg);
pyhea_status device_error(hipError_t e, const char *what);

#define PYHEA_HIP(expr)                                       \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return device_error(_e, #expr); \
    } while (0)

// Stream-ordered allocation from the current device's default pool.  The first
// call on a device makes the pool keep up to kPoolRetainBytes of freed memory
// across synchronisations, so that repeated calls do not map and unmap pages.
constexpr uint64_t kPoolRetainBytes = uint64_t(2) << 30;
hipError_t pool_alloc(void **ptr, size_t bytes, hipStream_t stream);

// Largest dynamic LDS one workgroup may allocate on the current device.
int max_lds_per_block();

// Checks target/weight of an objective (host pointers).
pyhea_status check_objective(const Geometry &g, const pyhea_objective *obj);

// Checks MC parameters.
pyhea_status check_params(const pyhea_mc_params *p);

// Species totals from exact counts (int64 [S][M][M]): n[i] = row sum of shell 1
// / z_1.  Returns false if some n_i == 0 (input validation).
bool species_totals(const Geometry &g, const int64_t *counts, int64_t *n);
// R[k][i][j] = N / (n_i n_j z_k): one exact int64 product and one IEEE division
// per entry, the table the kernels read (Eq. 2).
void ratio_table(const Geometry &g, const int64_t *n, double *R);

// One chain prepared for the MC kernel.
struct ChainJob {
    Geometry g;
    pyhea_mc_params params;
    std::vector<double> target, weight;
    int8_t *species_dev = nullptr;  // unpadded configuration (in/out)
    uint32_t *log_dev = nullptr;
    int64_t log_cap = 0;
};

// Runs a set of chains to completion on `stream` (synchronous).  Groups chains
// by launch shape; every chain's trajectory is independent of the grouping.
// `variant` < 0 lets the autotuner choose the launch shape.
pyhea_status run_chains(std::vector<ChainJob> &jobs, pyhea_mc_stats *stats,
                        std::vector<std::vector<int64_t>> *final_counts, hipStream_t stream,
                        int variant);

// Pair counts of K configurations of one geometry (counts [K][S][M][M], bad [K]):
// the bit-sliced kernel when it covers the geometry, else the gather kernel.
// With S_F (and tw = {target, weight} on the device) the objective may be
// computed by the counting kernel itself; *fused says whether it was.
// `partial` (optional) is caller-owned scratch for configurations that span
// several workgroups, at least count_partial_bytes(g, K) bytes; without it the
// function allocates that scratch itself.
pyhea_status count_configs(const Geometry &g, int64_t K, const int8_t *species, int32_t *counts,
                           int32_t *bad, hipStream_t stream, const double *tw = nullptr, double *S_F = nullptr,
                           bool *fused = nullptr, void *partial = nullptr);
// Scratch bytes count_configs needs for K configurations of g (0 if none).
size_t count_partial_bytes(const Geometry &g, int64_t K);

// Full evaluation of K configurations (pyhea_sro_eval_batch after argument
// checks): counts [K][S][M][M] and, with obj, S_F [K][2], on `stream`.
// `scratch` (optional, eval_batch_scratch_bytes(g, K) bytes, device) holds the
// per-configuration flags, the target table and the multi-workgroup partial
// sums; without it they come from the stream-ordered pool.
pyhea_status eval_batch(const Geometry &g, int64_t K, const int8_t *species, const pyhea_objective *obj,
                        int32_t *counts, double *S_F, hipStream_t stream, void *scratch = nullptr);
size_t eval_batch_scratch_bytes(const Geometry &g, int64_t K);


}  // namespace pyhea
