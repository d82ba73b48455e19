// Bit-sliced full evaluation (FCC): descriptor and launcher.
#pragma once

#include <hip/hip_runtime.h>

#include "geometry.h"

namespace pyhea {

struct BitDesc {
    int32_t Lx, Ly, Lz;
    int32_t RS;        // flat row stride in bits (Lx + 2)
    int32_t LW;        // words per plane (flat (Ly + 2) * RS bits)
    int32_t PADW;      // zero words before and after each plane
    int32_t PW;        // LW + 2 * PADW
    int32_t cw0, NCW;  // words that hold centre sites
    int32_t nchx;      // 32-position chunks per padded row (RS bits)
    int32_t vec4;      // rows read as 16-byte blocks (Lx % 4 == 0, 16-byte aligned configurations)
    int32_t ZC;        // centre layers per workgroup
    int32_t nchunks;   // workgroups per configuration
    int32_t threads;   // workgroup size
    int32_t partial_stride;
    uint32_t N;
    int32_t nh;
    int32_t hstart[kMaxShells + 1];
    int32_t zk[kMaxShells];
    int32_t tab_delta[4][kMaxOffsets / 2];  // neighbour dword offset per (basis, half offset)
    int32_t tab_r[4][kMaxOffsets / 2];      // funnel-shift amount
};

// Fills bd; false if the bit-sliced kernel does not cover this geometry (it
// covers FCC, and BCC with an even number of cells along x, for shells whose
// neighbours lie at most one cell away).
// K is the number of configurations of the launch: few configurations are
// split along z over more workgroups.  With split > 1, a configuration whose
// layers would take more than 1/split of a CU's LDS is cut along z so that
// `split` workgroups share each CU.
bool fill_bit_desc(const Geometry &g, int lds_budget, int64_t K, int split, BitDesc *bd);

// counts [K][S][M][M] and bad [K] of K configurations; `partial` is scratch of
// K * bd.nchunks * bd.partial_stride int32 (used when a configuration spans several
// workgroups).  With S_F != null (and bd.nchunks == 1) the kernel also writes
// S_F [K][2] from tw = {target [S][M][M], weight [S]} (device).
hipError_t launch_count_bits(const Geometry &g, const BitDesc &bd, int64_t K, const int8_t *species,
                             int32_t *partial, int32_t *counts, int32_t *bad, const double *tw, double *S_F,
                             hipStream_t stream);

}  // namespace pyhea
