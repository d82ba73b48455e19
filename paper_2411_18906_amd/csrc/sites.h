// Nearest-site assignment of external structures: descriptor and launcher.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pyhea {

struct SiteMapDesc {
    int32_t lattice;     // PYHEA_FCC or PYHEA_BCC
    int32_t A;           // sites per conventional cell
    int32_t L[3];
    int32_t M;           // species ids must lie in [0, M)
    int64_t N;           // sites
    double scale[3];     // half lattice units per unit of length, per axis (2 L / box)
    double max_disp2;    // squared largest accepted displacement (length units)
};

// owner [N] int32 and flags [4] int32 are device scratch (the entry point's or
// the caller's): flags = {displacement too large, two atoms on one site, type
// out of range, vacant site}.  Writes species [N].
hipError_t launch_map_sites(const SiteMapDesc &md, int64_t n, const double *xyz, const int8_t *types,
                            int32_t *owner, int32_t *flags, int8_t *species, hipStream_t stream);

}  // namespace pyhea
