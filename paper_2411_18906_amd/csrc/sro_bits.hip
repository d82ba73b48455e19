// Bit-sliced full SRO evaluation for FCC supercells (Sec. 4.3, Eq. 2).
//
// One workgroup counts a range of z-layers of one configuration:
//  1. Conversion.  Each FCC cell is one dword (4 sublattice bytes).  A v_perm
//     lookup table maps species ids to one-hot bits; 8 cells are merged per
//     byte lane with shift-or and a 4x4 byte transpose yields, per sublattice b
//     and species j < M-1, a 32-cell bit row.  Rows are OR-ed into a flat bit
//     array per (layer, b, j) with a one-cell periodic border:
//     bit = (cy + 1) * (Lx + 2) + (cx + 1).
//  2. Counting.  For a half-offset d (one of each +-d pair) from sublattice b
//     to b' with cell delta (dx, dy, dz), the neighbour bits of a 32-bit word
//     are a funnel shift by dy*(Lx+2)+dx of plane (layer+dz, b', j).  With
//     P_i the centre planes and Q_j the shifted ones,
//        T_d[i][i] = 2 popc(P_i & Q_i),
//        T_d[i][j] = popc((P_i & Q_j) | (P_j & Q_i))     (i < j < M-1)
//     (the two sets are disjoint), and T_d = H_d + H_d^T.  Rows of T_d sum to
//     2 n_i, so entries involving species M-1 follow from the others.
//  3. Finalisation.  N_k = sum over the shell's half-offsets of T_d.
// Counts are exact integers; invalid ids are detected per configuration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "device_common.h"
#include "sro_bits.h"

namespace pyhea {

namespace {

constexpr int kMaxThreads = 1024;

template <int M>
struct Pairs {
    static constexpr int P = M - 1;                 // explicit planes
    static constexpr int NP = P * (P + 1) / 2;      // i <= j < M-1
};

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

__device__ __forceinline__ void or_row(uint32_t *plane, int o, uint32_t r) {
    const int w = o >> 5, s = o & 31;
    atomicOr(&plane[w], r << s);
    if (s) atomicOr(&plane[w + 1], r >> (32 - s));
}

__device__ __forceinline__ void or_bit(uint32_t *plane, int o) { atomicOr(&plane[o >> 5], 1u << (o & 31)); }

// Sum over the 64 lanes of a wave, valid in lane 63: quad swaps, half-row and
// row mirrors, then row broadcasts 15 and 31 (DPP; no LDS traffic).
__device__ __forceinline__ int wave_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);  // row_mirror
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

// floor(n / d) for small non-negative n, d (see div_small)
__device__ __forceinline__ int qdiv(int n, double inv) { return (int)div_small((uint32_t)n, inv); }

// Counts of one configuration from its pair sums (S x NP, then n_0..n_{M-2}, then the
// bad-species flag), rows completed from the row-sum identity sum_j N_ij = z_k n_i,
// then Eq. 2-3: R = N / (n_i n_j z_k), alpha = 1 - N_ij R, each row's (alpha - t)^2
// summed over j, Q_k the sum of the rows, S = sum_k w_k Q_k, F = sqrt(S).  All
// threads of the block call it; lc, lsq, lrow are LDS scratch.
template <int M, int S>
__device__ __forceinline__ void epilogue(const int32_t *pairs, const BitDesc &bd, int32_t *lc, double *lsq, double *lrow,
                         int32_t *cnt, int32_t *bad_out, const double *tw, double *S_F) {
    constexpr int P = Pairs<M>::P;
    constexpr int NP = Pairs<M>::NP;
    int64_t n[M];
    {
        int64_t rest = bd.N;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            n[i] = pairs[S * NP + i];
            rest -= n[i];
        }
        n[M - 1] = rest;
    }
    const bool bad = pairs[S * NP + P] != 0;
    if (threadIdx.x < S) {
        const int k = threadIdx.x;
        const int32_t *pa = pairs + k * NP;
        int32_t *c = lc + k * M * M;
        int q = 0;
        for (int i = 0; i < P; ++i) {
            c[i * M + i] = 2 * pa[q++];
            for (int j = i + 1; j < P; ++j) {
                c[i * M + j] = pa[q];
                c[j * M + i] = pa[q];
                ++q;
            }
        }
        int64_t last = 0;
        for (int i = 0; i < P; ++i) {
            int64_t r = (int64_t)bd.zk[k] * n[i];
            for (int j = 0; j < P; ++j) r -= c[i * M + j];
            c[i * M + (M - 1)] = (int32_t)r;
            c[(M - 1) * M + i] = (int32_t)r;
            last += r;
        }
        c[(M - 1) * M + (M - 1)] = (int32_t)((int64_t)bd.zk[k] * n[M - 1] - last);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < S * M * M; e += blockDim.x) {
        cnt[e] = lc[e];
        if (S_F) {
            const int k = e / (M * M), i = (e / M) % M, j = e % M;
            const double R = (double)bd.N / (double)(n[i] * n[j] * (int64_t)bd.zk[k]);
            const double a = 1.0 - (double)lc[e] * R;
            const double dd = a - tw[e];
            lsq[e] = dd * dd;
        }
    }
    if (threadIdx.x == 0) *bad_out = bad ? 1 : 0;
    if (S_F) {
        __syncthreads();
        for (int r = threadIdx.x; r < S * M; r += blockDim.x) {
            double row = 0.0;
#pragma unroll
            for (int j = 0; j < M; ++j) row = row + lsq[r * M + j];
            lrow[r] = row;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            bool ok = !bad;
#pragma unroll
            for (int i = 0; i < M; ++i) ok = ok && n[i] > 0;
            double sum = 0.0;
            for (int k = 0; k < S; ++k) {
                double Q = 0.0;
#pragma unroll
                for (int i = 0; i < M; ++i) Q = Q + lrow[k * M + i];
                sum = sum + tw[S * M * M + k] * Q;
            }
            const double nan = __longlong_as_double(0x7ff8000000000000ll);
            S_F[0] = ok ? sum : nan;
            S_F[1] = ok ? sqrt(sum) : nan;
        }
    }
}

// MaxW: the wavefronts per SIMD the register allocation aims for -- 4 for a
// workgroup alone on its CU (registers spent on overlapping loads), 8 when
// several workgroups share the CU.
template <int M, int S, int MaxW>
__global__ void __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(4, MaxW)))
count_bits_kernel(BitDesc bd, int64_t K,
                                                               const int8_t *__restrict__ species,
                                                               int32_t *__restrict__ partial,
                                                               int32_t *__restrict__ counts_out,
                                                               int32_t *__restrict__ bad_out,
                                                               const double *__restrict__ tw,
                                                               double *__restrict__ S_F) {
    constexpr int P = Pairs<M>::P;
    constexpr int NP = Pairs<M>::NP;
    extern __shared__ __align__(16) uint32_t lds[];
    const int kc = blockIdx.y;
    if (kc >= K) return;
    const int chunk = blockIdx.x;
    const int z0 = chunk * bd.ZC;
    const int nz = min(bd.ZC, bd.Lz - z0);   // centre layers of this workgroup
    const int nl = nz + 1;                   // plus the next layer (dz in {0, 1})
    const int PW = bd.PW;
    const int LWD = 4 * P * PW;              // words per layer
    uint32_t *cmask = lds + nl * LWD;        // centre mask per word [LW]
    int32_t *red = (int32_t *)(cmask + bd.LW);  // reduction [S*NP + P + 1]
    int32_t *tab = red + S * NP + P + 1;        // (delta, shift) per (basis, half offset)
    for (int i = threadIdx.x; i < 4 * bd.nh; i += blockDim.x) {
        tab[2 * i] = bd.tab_delta[i / bd.nh][i % bd.nh];
        tab[2 * i + 1] = bd.tab_r[i / bd.nh][i % bd.nh];
    }

    // zero planes and the reduction area
    const int nzero = nl * LWD;
    for (int i = threadIdx.x; i < nzero; i += blockDim.x) lds[i] = 0;
    for (int i = threadIdx.x; i < S * NP + P + 1; i += blockDim.x) red[i] = 0;
    // centre mask: bit x of the flat array is a real site if row and column are inside
    for (int w = threadIdx.x; w < bd.LW; w += blockDim.x) {
        const int x0 = 32 * w;
        int row = x0 / bd.RS, col = x0 - row * bd.RS;
        uint32_t m = 0;
        for (int t = 0; t < 32; ++t) {
            if (row >= 1 && row <= bd.Ly && col >= 1 && col <= bd.Lx) m |= 1u << t;
            if (++col == bd.RS) {
                col = 0;
                ++row;
            }
        }
        cmask[w] = m;
    }
    __syncthreads();

    // ---- 1. conversion ------------------------------------------------------------
    const uint32_t *cfg = reinterpret_cast<const uint32_t *>(species + kc * (int64_t)bd.N);
    uint32_t badacc = 0;
    const int nitems = nl * bd.Ly * bd.nchx;
    const double inv_nchx = 1.0 / bd.nchx, inv_rows = 1.0 / (bd.nchx * bd.Ly);
#pragma unroll 1
    for (int it = threadIdx.x; it < nitems; it += blockDim.x) {
        const int ll = qdiv(it, inv_rows);
        const int rem = it - ll * bd.nchx * bd.Ly;
        const int cy = qdiv(rem, inv_nchx);
        const int cxc = rem - cy * bd.nchx;
        int cz = z0 + ll;
        if (cz >= bd.Lz) cz -= bd.Lz;
        const int cx0 = 32 * cxc;
        const int ncell = min(32, bd.Lx - cx0);
        const uint32_t *row = cfg + ((int64_t)cz * bd.Ly + cy) * bd.Lx + cx0;
        uint32_t acc[P][4];
#pragma unroll
        for (int j = 0; j < P; ++j)
#pragma unroll
            for (int g = 0; g < 4; ++g) acc[j][g] = 0;
        const int ngroups = (ncell + 7) >> 3;
#pragma unroll 1
        for (int g = 0; g < ngroups; ++g) {
            uint32_t part[P];
#pragma unroll
            for (int j = 0; j < P; ++j) part[j] = 0;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int c = 8 * g + m;
                const uint32_t d = row[min(c, ncell - 1)];
                const uint32_t lane_pad = c < ncell ? 0u : 0xFFFFFFFFu;
                // ids must be in [0, M): (d & 0x7f) + (0x80 - M) has its high bit set iff id >= M
                badacc |= ((((d & 0x7F7F7F7Fu) + (0x80u - M) * 0x01010101u) | d) & ~lane_pad) & 0x80808080u;
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    // one-hot lookup: byte value s -> (s == j)
                    const uint64_t lut = 1ull << (8 * j);
                    const uint32_t o = perm((uint32_t)(lut >> 32), (uint32_t)lut, d) & ~lane_pad;
                    part[j] |= o << m;
                }
            }
#pragma unroll
            for (int j = 0; j < P; ++j) {
                // groups are visited in order; select the slot without dynamic indexing
                acc[j][0] = g == 0 ? part[j] : acc[j][0];
                acc[j][1] = g == 1 ? part[j] : acc[j][1];
                acc[j][2] = g == 2 ? part[j] : acc[j][2];
                acc[j][3] = g == 3 ? part[j] : acc[j][3];
            }
        }
        // 4x4 byte transpose: acc[j][g] byte b = bits of cells 8g..8g+7 of sublattice b
        const bool last = cx0 + ncell == bd.Lx, first = cx0 == 0;
        const int fr0 = cy + 1;
        const int fr1 = cy == bd.Ly - 1 ? 0 : -1;       // periodic border rows
        const int fr2 = cy == 0 ? bd.Ly + 1 : -1;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const uint32_t u0 = perm(acc[j][1], acc[j][0], 0x05010400u);
            const uint32_t u1 = perm(acc[j][1], acc[j][0], 0x07030602u);
            const uint32_t v0 = perm(acc[j][3], acc[j][2], 0x05010400u);
            const uint32_t v1 = perm(acc[j][3], acc[j][2], 0x07030602u);
            const uint32_t R[4] = {perm(v0, u0, 0x05040100u), perm(v0, u0, 0x07060302u),
                                   perm(v1, u1, 0x05040100u), perm(v1, u1, 0x07060302u)};
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                uint32_t *plane = lds + ((ll * 4 + b) * P + j) * PW + bd.PADW;
                const uint32_t r = R[b];
                if (r == 0) continue;
                const bool bl = last && ((r >> (ncell - 1)) & 1u);  // column 0 <- cell Lx-1
                const bool bf = first && (r & 1u);                  // column Lx+1 <- cell 0
                or_row(plane, fr0 * bd.RS + 1 + cx0, r);
                if (bl) or_bit(plane, fr0 * bd.RS);
                if (bf) or_bit(plane, fr0 * bd.RS + bd.Lx + 1);
                if (fr1 >= 0) {
                    or_row(plane, fr1 * bd.RS + 1 + cx0, r);
                    if (bl) or_bit(plane, fr1 * bd.RS);
                    if (bf) or_bit(plane, fr1 * bd.RS + bd.Lx + 1);
                }
                if (fr2 >= 0) {
                    or_row(plane, fr2 * bd.RS + 1 + cx0, r);
                    if (bl) or_bit(plane, fr2 * bd.RS);
                    if (bf) or_bit(plane, fr2 * bd.RS + bd.Lx + 1);
                }
            }
        }
    }
    __syncthreads();

    // ---- 2. counting --------------------------------------------------------------
    int32_t acc[S][NP];
#pragma unroll
    for (int k = 0; k < S; ++k)
#pragma unroll
        for (int q = 0; q < NP; ++q) acc[k][q] = 0;
    int32_t ncnt[P];
#pragma unroll
    for (int i = 0; i < P; ++i) ncnt[i] = 0;
    const int nwork = nz * 4 * bd.NCW;
    const double inv_ncw = 1.0 / bd.NCW;
#pragma unroll 1
    for (int it = threadIdx.x; it < nwork; it += blockDim.x) {
        const int lb = qdiv(it, inv_ncw);      // layer * 4 + basis
        const int w = bd.cw0 + it - lb * bd.NCW;
        const int b = lb & 3;
        const int ll = lb >> 2;
        const uint32_t cm = cmask[w];
        const uint32_t *pc = lds + (ll * 4 + b) * P * PW + bd.PADW + w;
        uint32_t Pv[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            Pv[i] = pc[i * PW] & cm;
            ncnt[i] += __popc(Pv[i]);
        }
        const uint32_t *lbase = lds + ll * LWD + bd.PADW + w;
#pragma unroll
        for (int k = 0; k < S; ++k) {
#pragma unroll 1
            for (int h = bd.hstart[k]; h < bd.hstart[k + 1]; ++h) {
                const int delta = tab[2 * (b * bd.nh + h)];
                const uint32_t r = (uint32_t)tab[2 * (b * bd.nh + h) + 1];
                const uint32_t *nb = lbase + delta;
                uint32_t Q[P];
#pragma unroll
                for (int j = 0; j < P; ++j) Q[j] = __builtin_amdgcn_alignbit(nb[j * PW + 1], nb[j * PW], r);
                int q = 0;
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    acc[k][q] += __popc(Pv[i] & Q[i]);
                    ++q;
#pragma unroll
                    for (int j = i + 1; j < P; ++j) {
                        // (P_i & Q_j) | (P_j & Q_i): one AND and one three-input op (0xEA = (a & b) | c)
                        acc[k][q] += __popc(__builtin_amdgcn_bitop3_b32(Pv[i], Q[j], Pv[j] & Q[i], 0xEA));
                        ++q;
                    }
                }
            }
        }
    }
    // ---- 3. reduce over the workgroup, then into the per-configuration partials ------
#pragma unroll
    for (int k = 0; k < S; ++k)
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int v = wave_sum(acc[k][q]);
            if ((threadIdx.x & 63) == 63 && v) atomicAdd(&red[k * NP + q], v);
        }
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int v = wave_sum(ncnt[i]);
        if ((threadIdx.x & 63) == 63 && v) atomicAdd(&red[S * NP + i], v);
    }
    {
        uint64_t anybad = __ballot(badacc != 0);
        if ((threadIdx.x & 63) == 0 && anybad) atomicOr(&red[S * NP + P], 1);
    }
    __syncthreads();
    if (bd.nchunks > 1) {
        int32_t *out = partial + kc * (int64_t)bd.partial_stride;
        for (int i = threadIdx.x; i < S * NP + P + 1; i += blockDim.x) {
            if (i < S * NP + P)
                atomicAdd(&out[i], red[i]);
            else if (red[i])
                atomicOr(&out[i], red[i]);
        }
        return;
    }
    // ---- 4. one workgroup holds the whole configuration: counts and Eq. 2-3 here ----
    // epilogue scratch after the offset table: [S][M][M] counts, [S][M][M] and [S][M] doubles
    int32_t *lc = tab + 8 * bd.nh;
    double *lsq = reinterpret_cast<double *>((reinterpret_cast<uintptr_t>(lc + S * M * M) + 7) & ~uintptr_t(7));
    epilogue<M, S>(red, bd, lc, lsq, lsq + S * M * M, counts_out + kc * (int64_t)(S * M * M), bad_out + kc, tw,
                   S_F ? S_F + 2 * kc : nullptr);
}


// partial sums -> full counts N[k][i][j] (one thread per configuration)
template <int M, int S>
__global__ void finalize_bits_kernel(BitDesc bd, int64_t K, const int32_t *__restrict__ partial,
                                     int32_t *__restrict__ counts, int32_t *__restrict__ bad) {
    constexpr int P = Pairs<M>::P;
    constexpr int NP = Pairs<M>::NP;
    const int64_t kc = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (kc >= K) return;
    const int32_t *pa = partial + kc * (int64_t)bd.partial_stride;
    int32_t *c = counts + kc * (int64_t)(S * M * M);
    int64_t n[M];
    int64_t rest = bd.N;
    for (int i = 0; i < P; ++i) {
        n[i] = pa[S * NP + i];
        rest -= n[i];
    }
    n[M - 1] = rest;
    bad[kc] = pa[S * NP + P] ? 1 : 0;
    for (int k = 0; k < S; ++k) {
        int q = 0;
        for (int i = 0; i < P; ++i) {
            c[(k * M + i) * M + i] = 2 * pa[k * NP + q];
            ++q;
            for (int j = i + 1; j < P; ++j) {
                c[(k * M + i) * M + j] = pa[k * NP + q];
                c[(k * M + j) * M + i] = pa[k * NP + q];
                ++q;
            }
        }
        // rows sum to z_k n_i
        int64_t last_col_sum = 0;
        for (int i = 0; i < P; ++i) {
            int64_t r = (int64_t)bd.zk[k] * n[i];
            for (int j = 0; j < P; ++j) r -= c[(k * M + i) * M + j];
            c[(k * M + i) * M + (M - 1)] = (int32_t)r;
            c[(k * M + (M - 1)) * M + i] = (int32_t)r;
            last_col_sum += r;
        }
        c[(k * M + (M - 1)) * M + (M - 1)] = (int32_t)((int64_t)bd.zk[k] * n[M - 1] - last_col_sum);
    }
}

// partial sums -> counts and Eq. 2-3 (one 64-thread block per configuration)
template <int M, int S>
__global__ void __launch_bounds__(64) finalize_objective_kernel(BitDesc bd, const int32_t *__restrict__ partial,
                                                               int32_t *__restrict__ counts,
                                                               int32_t *__restrict__ bad,
                                                               const double *__restrict__ tw,
                                                               double *__restrict__ S_F) {
    __shared__ int32_t lc[S * M * M];
    __shared__ double lsq[S * M * M];
    __shared__ double lrow[S * M];
    const int64_t kc = blockIdx.x;
    epilogue<M, S>(partial + kc * bd.partial_stride, bd, lc, lsq, lrow, counts + kc * (int64_t)(S * M * M), bad + kc,
                   tw, S_F + 2 * kc);
}

__global__ void zero_kernel(int32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <int M, int S>
hipError_t launch_ms(const BitDesc &bd, int64_t K, const int8_t *species, int32_t *partial, int32_t *counts,
                     int32_t *bad, const double *tw, double *S_F, hipStream_t stream) {
    const int P = M - 1;
    const size_t lds = ((size_t)(bd.ZC + 1) * 4 * P * bd.PW + bd.LW + S * Pairs<M>::NP + P + 1 + 8 * bd.nh + 1 +
                        3 * S * M * M + 2 * S * M + 2) * 4;
    const bool lone = bd.threads > 512;   // one workgroup per CU
    const void *fn = lone ? (const void *)count_bits_kernel<M, S, 4> : (const void *)count_bits_kernel<M, S, 8>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (bd.nchunks > 1) {
        const int64_t n = K * bd.partial_stride;
        hipLaunchKernelGGL(zero_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0,
                           stream, partial, n);
    }
    for (int64_t k0 = 0; k0 < K; k0 += 65535) {
        const int64_t kn = std::min<int64_t>(65535, K - k0);
        if (!lone)
            hipLaunchKernelGGL((count_bits_kernel<M, S, 8>), dim3(bd.nchunks, (unsigned)kn), dim3(bd.threads), lds, stream,
                               bd, kn, species + k0 * (int64_t)bd.N, partial + k0 * bd.partial_stride,
                               counts + k0 * (int64_t)(S * M * M), bad + k0, tw, S_F ? S_F + 2 * k0 : nullptr);
        else
            hipLaunchKernelGGL((count_bits_kernel<M, S, 4>), dim3(bd.nchunks, (unsigned)kn), dim3(bd.threads), lds, stream,
                               bd, kn, species + k0 * (int64_t)bd.N, partial + k0 * bd.partial_stride,
                               counts + k0 * (int64_t)(S * M * M), bad + k0, tw, S_F ? S_F + 2 * k0 : nullptr);
    }
    if (bd.nchunks > 1 && S_F)
        hipLaunchKernelGGL((finalize_objective_kernel<M, S>), dim3((unsigned)K), dim3(64), 0, stream, bd, partial,
                           counts, bad, tw, S_F);
    else if (bd.nchunks > 1)
        hipLaunchKernelGGL((finalize_bits_kernel<M, S>), dim3((unsigned)((K + 127) / 128)), dim3(128), 0, stream, bd, K,
                           partial, counts, bad);
    return hipGetLastError();
}

using LaunchFn = hipError_t (*)(const BitDesc &, int64_t, const int8_t *, int32_t *, int32_t *, int32_t *,
                                const double *, double *, hipStream_t);

template <int M>
LaunchFn pick_s(int S) {
    switch (S) {
        case 1: return launch_ms<M, 1>;
        case 2: return launch_ms<M, 2>;
        case 3: return Pairs<M>::NP * 3 <= 64 ? launch_ms<M, 3> : nullptr;
        case 4: return Pairs<M>::NP * 4 <= 64 ? launch_ms<M, 4> : nullptr;
    }
    return nullptr;
}

LaunchFn pick(int M, int S) {
    switch (M) {
        case 2: return pick_s<2>(S);
        case 3: return pick_s<3>(S);
        case 4: return pick_s<4>(S);
        case 5: return pick_s<5>(S);
        case 6: return pick_s<6>(S);
        case 7: return S <= 2 ? pick_s<7>(S) : nullptr;
        case 8: return S <= 2 ? pick_s<8>(S) : nullptr;
    }
    return nullptr;
}

}  // namespace

bool fill_bit_desc(const Geometry &g, int lds_budget, int64_t K, BitDesc *bd) {
    std::memset(bd, 0, sizeof(*bd));
    if (g.lattice != PYHEA_FCC || g.halo != 1 || !pick(g.M, g.S)) return false;
    const int P = g.M - 1;
    bd->Lx = g.L[0];
    bd->Ly = g.L[1];
    bd->Lz = g.L[2];
    bd->RS = g.L[0] + 2;
    const int bits = (g.L[1] + 2) * bd->RS;
    bd->LW = (bits + 31) / 32;
    bd->PADW = (bd->RS + 2 + 31) / 32 + 1;
    bd->PW = bd->LW + 2 * bd->PADW;
    bd->cw0 = bd->RS / 32;
    bd->NCW = ((g.L[1] + 1) * bd->RS - 1) / 32 - bd->cw0 + 1;
    bd->nchx = (g.L[0] + 31) / 32;
    bd->N = (uint32_t)g.N;
    const int np = P * (P + 1) / 2;
    bd->partial_stride = ((g.S * np + P + 1) + 3) & ~3;
    for (int k = 0; k < kMaxShells; ++k) bd->zk[k] = k < g.S ? g.z[k] : 0;
    // largest z-chunk whose planes fit in LDS
    const int fixed = (bd->LW + g.S * np + P + 1 + 8 * kMaxOffsets / 2 + 3 * g.S * g.M * g.M + 2 * g.S * g.M + 3) * 4;
    const int per_layer = 4 * P * bd->PW * 4;
    int zc = (lds_budget - fixed) / per_layer - 1;
    if (zc < 1) return false;
    zc = std::min(zc, g.L[2]);
    zc = (g.L[2] + (g.L[2] + zc - 1) / zc - 1) / ((g.L[2] + zc - 1) / zc);
    // few configurations: spread each over up to 512 / K workgroups along z
    const int64_t want = std::max<int64_t>(1, 512 / std::max<int64_t>(K, 1));
    if (want > 1) zc = std::min<int64_t>(zc, std::max<int64_t>(2, (g.L[2] + want - 1) / want));
    bd->ZC = zc;
    bd->nchunks = (g.L[2] + zc - 1) / zc;
    // a workgroup that needs more than half the LDS runs alone on its CU: give it
    // 16 wavefronts so the CU still has latency to hide behind
    bd->threads = fixed + (zc + 1) * per_layer > lds_budget / 2 ? 1024 : 512;
    // half offsets ordered by shell
    int nh = 0;
    for (int k = 0; k < g.S; ++k) {
        bd->hstart[k] = nh;
        for (int t = g.zstart[k]; t < g.zstart[k + 1]; ++t) {
            const int dx = g.off[t][0], dy = g.off[t][1], dz = g.off[t][2];
            const bool keep = dz > 0 || (dz == 0 && (dy > 0 || (dy == 0 && dx > 0)));
            if (!keep) continue;
            for (int b = 0; b < 4; ++b) {
                int dc[3], bt;
                offset_target(g, b, t, dc, &bt);
                // plane word of the neighbour: layer +dz, sublattice bt, bit shift s
                const int s = dc[1] * bd->RS + dc[0];
                const int q = s >= 0 ? s / 32 : -((-s + 31) / 32);
                const int r = s - 32 * q;
                bd->tab_delta[b][nh] = (dc[2] * 4 + bt) * P * bd->PW + q;
                bd->tab_r[b][nh] = r;
            }
            ++nh;
        }
    }
    bd->hstart[g.S] = nh;
    bd->nh = nh;
    return true;
}

hipError_t launch_count_bits(const Geometry &g, const BitDesc &bd, int64_t K, const int8_t *species,
                             int32_t *partial, int32_t *counts, int32_t *bad, const double *tw, double *S_F,
                             hipStream_t stream) {
    LaunchFn f = pick(g.M, g.S);
    if (!f) return hipErrorInvalidValue;
    return f(bd, K, species, partial, counts, bad, tw, S_F, stream);
}

}  // namespace pyhea
