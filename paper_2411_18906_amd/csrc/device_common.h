// Device helpers shared by the pyhea kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geometry.h"

namespace pyhea {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products by the published multipliers with a Weyl key bump.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo0 = 0xD2511F53u * c[0];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// floor(n / d) for n < 2^31 and d < 10^6, from a binary64 reciprocal: the
// product (n + 0.5) * fl(1/d) is within 2^-21 of (n + 0.5)/d, whose distance to
// the nearest integer is at least 0.5/d, so truncation is exact.
__device__ __forceinline__ uint32_t div_small(uint32_t n, double inv_d) {
    return (uint32_t)(((double)n + 0.5) * inv_d);
}

// Site coordinates: cell (cx, cy, cz) and basis b of site id p.
struct SiteCoord {
    int32_t cx, cy, cz, b;
};

__device__ __forceinline__ SiteCoord site_coord(uint32_t p, int32_t lgA, int32_t Lx, int32_t Ly,
                                                double inv_Lx, double inv_Ly) {
    SiteCoord s;
    s.b = (int32_t)(p & ((1u << lgA) - 1u));
    const uint32_t c = p >> lgA;
    const uint32_t yz = div_small(c, inv_Lx);
    s.cx = (int32_t)(c - yz * (uint32_t)Lx);
    const uint32_t z = div_small(yz, inv_Ly);
    s.cy = (int32_t)(yz - z * (uint32_t)Ly);
    s.cz = (int32_t)z;
    return s;
}

// Basis vector components of basis b (FCC: A = 4, BCC: A = 2), half units.
__device__ __forceinline__ void basis_bits(int32_t A, int32_t b, int32_t &bx, int32_t &by,
                                           int32_t &bz) {
    if (A == 4) {
        // (0,0,0), (1,1,0), (1,0,1), (0,1,1)
        bx = (b == 1 || b == 2) ? 1 : 0;
        by = (b == 1 || b == 3) ? 1 : 0;
        bz = (b == 2 || b == 3) ? 1 : 0;
    } else {
        bx = by = bz = b;
    }
}

// Wave-level helpers.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const uint64_t u = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), lane);
    return __longlong_as_double(((uint64_t)hi << 32) | lo);
}

// value of v in lane src (any lane index per lane; one LDS permute per half)
__device__ __forceinline__ double shfl_f64(double v, int src) {
    const uint64_t u = __double_as_longlong(v);
    const int addr = (src & 63) << 2;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(u >> 32));
    return __longlong_as_double(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t ballot64(bool pred) { return __ballot(pred); }

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

}  // namespace pyhea
