// Bit-sliced full evaluation (FCC): descriptor and launcher.
#pragma once

#include <hip/hip_runtime.h>

#include "geometry.h"

namespace pyhea {

struct BitDesc {
    int32_t Lx, Ly, Lz;  // four-site cells per axis (Lz: the layers of the periodic layout)
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
    // BCC with an odd number of cells along x: a four-site cell is BCC cell
    // (x, y, 2z) and (x, y, 2z + 1) along z (zpair = 1; Lzs = the BCC cells
    // along z).  With Lzs odd the layout holds the configuration twice along z
    // (Lz = Lzs layers) and only BCC layers 0 .. Lzs - 1 are centres: layers
    // 0 .. Lzc - 2 whole, and layer Lzc - 1 for its first BCC layer only
    // (half_last = 1).  Otherwise Lzc = Lz.
    int32_t zpair, Lzs, Lzc, half_last;
    int32_t al2;       // the batch starts on an even address (z-paired rows read 16 bytes at a time)
    int32_t hx, hy, hz;  // border of the layout: columns and rows each side, layers above
    int32_t nh;
    int32_t hstart[kMaxShells + 1];
    int32_t zk[kMaxShells];
    int32_t tab_delta[4][kMaxOffsets / 2];  // neighbour dword offset per (basis, half offset)
    int32_t tab_r[4][kMaxOffsets / 2];      // funnel-shift amount
};

// Streaming form (batches): one workgroup per configuration at a time, z
// layers walked in groups of G while the next chunk's bytes arrive.
struct StreamDesc {
    int32_t Lx, Ly, Lz;     // four-site cells per axis
    int32_t RS, LW, PADW, PW, cw0, NCW;   // as in BitDesc
    int32_t G;              // centre layers per group
    int32_t ngroups;        // ceil(Lz / G)
    int32_t ndma;           // 64-position load blocks per staged layer
    int32_t raw_dw;         // dwords per staged layer (64 * ndma)
    int32_t slot_dw;        // dwords per plane slot (4 * PW * planes padded to even)
    int32_t o_planes, o_cmask, o_red2, o_red, o_epi;   // LDS offsets (dwords)
    int32_t lds_bytes;
    int32_t threads;
    int32_t maxd;           // load blocks per lane the kernel holds offsets for
    int32_t grid;           // persistent workgroups
    uint32_t N;
    int32_t zk[kMaxShells];
    int32_t hs[4][2][kMaxShells + 1];   // per basis and layer step dz: start of shell k's half offsets
    int32_t tab[4][kMaxOffsets / 2];     // (dword delta within a layer slot) * 32 + funnel shift
};

// Fills sd for a batch of K configurations; false if the streaming kernel does
// not cover the geometry (same lattices as the bit-sliced kernel).  G and
// threads = 0 pick the launch shape automatically.
bool fill_stream_desc(const Geometry &g, int lds_budget, int n_cus, int64_t K, int G, int threads, StreamDesc *sd);

hipError_t launch_count_stream(const Geometry &g, const StreamDesc &sd, int64_t K, const int8_t *species,
                               int32_t *counts, int32_t *bad, const double *tw, double *S_F, hipStream_t stream);

// Fills bd; false if the bit-sliced kernel does not cover this geometry (it
// covers FCC and BCC for shells whose neighbours lie at most two cells away;
// four-site cells pair BCC cells along x, or along z when Lx is odd).
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
