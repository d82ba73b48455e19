// Bit-sliced full SRO evaluation (Sec. 4.3, Eq. 2) for lattices laid out as
// cells of four sites: FCC, and BCC (two BCC cells along x, or along z when
// the number of cells along x is odd, form one four-site cell; see
// fill_bit_desc).
//
// One workgroup counts a range of z-layers of one configuration:
//  1. Conversion.  Per sublattice b and species j < M-1 a layer becomes a flat
//     bit array with a periodic border of hx columns and hy rows (one each,
//     two for BCC shell 4): bit fy * RS + fx (RS = Lx + 2 hx) holds cell
//     ((fx - hx) mod Lx, (fy - hy) mod Ly).  A lane converts one padded row:
//     each cell is one dword (4 sublattice bytes), converted eight at a time
//     through their species' binary digits, and a 4x4 byte transpose yields
//     32-position bit rows (one-hot per species) that are OR-ed into LDS.  The M-1 species planes are interleaved word by word:
//     dword ((layer * 4 + b) * PW + word) * (M - 1) + j.
//  2. Counting.  For a half-offset d (one of each +-d pair) from sublattice b to
//     b' with cell delta (dx, dy, dz), the neighbour bits of a 32-bit word are a
//     funnel shift by dy*RS+dx of plane (layer+dz, b', j).  With P_i the centre
//     planes and Q_j the shifted ones (each set pairwise disjoint),
//        D_i  = popc(P_i & Q_i),
//        U_ij = popc((P_i | P_j) & (Q_i | Q_j))
//             = D_i + D_j + popc(P_i & Q_j) + popc(P_j & Q_i)        (i < j),
//     so T_d = H_d + H_d^T has T_d[i][i] = 2 D_i and T_d[i][j] = U_ij - D_i - D_j.
//     Rows of T_d sum to 2 n_i, so entries involving species M-1 follow from
//     the others.
//  3. Finalisation.  N_k = sum over the shell's half-offsets of T_d.
// Counts are exact integers; invalid ids are detected per configuration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "device_common.h"
#include "mc_kernels.h"
#include "sro_bits.h"

namespace pyhea {

namespace {

constexpr int kMaxThreads = 1024;

template <int M>
struct Pairs {
    static constexpr int P = M - 1;                 // explicit planes
    static constexpr int NP = P * (P + 1) / 2;      // i <= j < M-1
    // position of (i, j), i <= j, in the per-shell sums: (0,0), (0,1), ..., (1,1), ...
    static constexpr __host__ __device__ int q(int i, int j) { return i * P - i * (i - 1) / 2 + (j - i); }
};

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

// floor(n / d) for small non-negative n, d (see div_small)
__device__ __forceinline__ int qdiv(int n, double inv) { return (int)div_small((uint32_t)n, inv); }

// Counts [M][M] of one shell from its sums pa (D_i at q(i,i), U_ij at q(i,j)),
// the shell's coordination number and the species totals n: T entries from
// D and U, then rows completed from sum_j N_ij = z_k n_i.
template <int M>
__device__ __forceinline__ void expand_shell(const int32_t *pa, int64_t zk, const int64_t *n, int32_t *c) {
    constexpr int P = Pairs<M>::P;
    for (int i = 0; i < P; ++i) {
        const int32_t Di = pa[Pairs<M>::q(i, i)];
        c[i * M + i] = 2 * Di;
        for (int j = i + 1; j < P; ++j) {
            const int32_t t = pa[Pairs<M>::q(i, j)] - Di - pa[Pairs<M>::q(j, j)];
            c[i * M + j] = t;
            c[j * M + i] = t;
        }
    }
    int64_t last = 0;
    for (int i = 0; i < P; ++i) {
        int64_t r = zk * n[i];
        for (int j = 0; j < P; ++j) r -= c[i * M + j];
        c[i * M + (M - 1)] = (int32_t)r;
        c[(M - 1) * M + i] = (int32_t)r;
        last += r;
    }
    c[(M - 1) * M + (M - 1)] = (int32_t)(zk * n[M - 1] - last);
}

// Counts of one configuration from its sums (S x NP, then n_0..n_{M-2}, then the
// bad-species flag), then Eq. 2-3: R = N / (n_i n_j z_k), alpha = 1 - N_ij R, each
// row's (alpha - t)^2 summed over j, Q_k the sum of the rows, S = sum_k w_k Q_k,
// F = sqrt(S).  All threads of the block call it; lc, lsq, lrow are LDS scratch.
template <int M, int S, class Desc>
__device__ __forceinline__ void epilogue(const int32_t *pairs, const Desc &bd, int32_t *lc, double *lsq, double *lrow,
                         int32_t *cnt, int32_t *bad_out, const double *tw, double *S_F,
                         int tid = (int)threadIdx.x) {
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
    if (tid < S) {
        const int k = tid;
        expand_shell<M>(pairs + k * NP, bd.zk[k], n, lc + k * M * M);
    }
    __syncthreads();
    for (int e = tid; e < S * M * M; e += blockDim.x) {
        cnt[e] = lc[e];
        if (S_F) {
            const int k = e / (M * M), i = (e / M) % M, j = e % M;
            const double R = (double)bd.N / (double)(n[i] * n[j] * (int64_t)bd.zk[k]);
            const double a = 1.0 - (double)lc[e] * R;
            const double dd = a - tw[e];
            lsq[e] = dd * dd;
        }
    }
    if (tid == 0) *bad_out = bad ? 1 : 0;
    if (S_F) {
        __syncthreads();
        for (int r = tid; r < S * M; r += blockDim.x) {
            double row = 0.0;
#pragma unroll
            for (int j = 0; j < M; ++j) row = row + lsq[r * M + j];
            lrow[r] = row;
        }
        __syncthreads();
        if (tid == 0) {
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

// P consecutive LDS dwords (16- or 8-byte loads where P allows: every group of
// P dwords starts at a multiple of P dwords)
template <int P>
__device__ __forceinline__ void lds_planes(const uint32_t *p, uint32_t *v) {
    if constexpr (P == 4) {
        const uint4 t = *reinterpret_cast<const uint4 *>(p);
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
        v[3] = t.w;
    } else if constexpr (P % 2 == 0) {
#pragma unroll
        for (int i = 0; i < P; i += 2) {
            const uint2 t = *reinterpret_cast<const uint2 *>(p + i);
            v[i] = t.x;
            v[i + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < P; ++i) v[i] = p[i];
    }
}

// Centre planes of one word: P dwords at p masked to the centre sites cm, their
// species totals added to this lane's slots, and Un = P_i | P_j at q(i, j), i < j.
template <int M>
__device__ __forceinline__ void centre_word(const uint32_t *p, uint32_t cm, int32_t *slots, uint32_t *Pv,
                                            uint32_t *Un) {
    constexpr int P = Pairs<M>::P;
    lds_planes<P>(p, Pv);
#pragma unroll
    for (int i = 0; i < P; ++i) {
        Pv[i] &= cm;
        // species totals go straight to this lane's slots (no registers held)
        atomicAdd(slots + i * 64, (int32_t)__popc(Pv[i]));
    }
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
        for (int j = i + 1; j < P; ++j) Un[Pairs<M>::q(i, j)] = Pv[i] | Pv[j];
}

// One half offset: D_i = popc(P_i & Q_i) and U_ij = popc((P_i | P_j) & (Q_i | Q_j))
// added to the sums a of its shell; Q are the neighbour planes.
template <int M>
__device__ __forceinline__ void count_offset(int32_t *a, const uint32_t *Pv, const uint32_t *Un, const uint32_t *Q) {
    constexpr int P = Pairs<M>::P;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        a[Pairs<M>::q(i, i)] += __popc(Pv[i] & Q[i]);
#pragma unroll
        for (int j = i + 1; j < P; ++j)
            // (P_i | P_j) & (Q_i | Q_j): one three-input op (0xE0 = a & (b | c))
            a[Pairs<M>::q(i, j)] += __popc(__builtin_amdgcn_bitop3_b32(Un[Pairs<M>::q(i, j)], Q[i], Q[j], 0xE0));
    }
}


// Binary digits of species ids: ND digits per byte (ids < 2^ND).
template <int M>
struct Digits {
    static constexpr int ND = M <= 2 ? 1 : M <= 4 ? 2 : 3;
};

// Eight cells d[0..7] (four sublattice bytes each, ids < 2^ND) -> for each
// digit beta a word whose byte b has bit m = digit beta of byte b of d[m].
// ND = 2: cells of even and odd index are packed two bits apart (no field
// overlaps), then one bitfield insert per digit merges them; ND = 3: cells r
// and r + 4 share a byte four bits apart, and each digit is gathered from the
// four packed words by a shift and a masked insert.
template <int ND>
__device__ __forceinline__ void digits8(const uint32_t *d, uint32_t *D) {
    if constexpr (ND == 1) {
        uint32_t a = d[0];
#pragma unroll
        for (int m = 1; m < 8; ++m) a |= d[m] << m;
        D[0] = a;
    } else if constexpr (ND == 2) {
        const uint32_t e = d[0] | (d[2] << 2) | (d[4] << 4) | (d[6] << 6);   // cell m: digits at bits m, m + 1
        const uint32_t o = d[1] | (d[3] << 2) | (d[5] << 4) | (d[7] << 6);   // cell m: digits at bits m - 1, m
        D[0] = (e & 0x55555555u) | ((o << 1) & 0xAAAAAAAAu);
        D[1] = ((e >> 1) & 0x55555555u) | (o & 0xAAAAAAAAu);
    } else {
        uint32_t A[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) A[r] = d[r] | (d[r + 4] << 4);   // cells r, r + 4 at bits 0-2, 4-6
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            uint32_t v = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t t = r >= b ? A[r] << (r - b) : A[r] >> (b - r);
                v |= t & (0x11111111u << r);
            }
            D[b] = v;
        }
    }
}

// One-hot plane j < M - 1 (bit set where the id equals j) of ND digit planes.
template <int ND>
__device__ __forceinline__ uint32_t onehot_plane(const uint32_t *Dg, int j) {
    // bitop3 truth-table index is 4a + 2b + c for operands (a, b, c)
    if constexpr (ND == 1) {
        return j == 0 ? ~Dg[0] : Dg[0];
    } else {
        const uint32_t a = ND == 3 ? Dg[ND - 1] : 0u, b = Dg[1], c = Dg[0];
        switch (j) {   // the truth table must be an immediate (j is constant once loops unroll)
            case 0: return __builtin_amdgcn_bitop3_b32(a, b, c, 0x01);
            case 1: return __builtin_amdgcn_bitop3_b32(a, b, c, 0x02);
            case 2: return __builtin_amdgcn_bitop3_b32(a, b, c, 0x04);
            case 3: return __builtin_amdgcn_bitop3_b32(a, b, c, 0x08);
            case 4: return __builtin_amdgcn_bitop3_b32(a, b, c, 0x10);
            case 5: return __builtin_amdgcn_bitop3_b32(a, b, c, 0x20);
            default: return __builtin_amdgcn_bitop3_b32(a, b, c, 0x40);
        }
    }
}

// Eight consecutive 2-byte cells c0 .. c0 + 7 of a BCC row at byte address a
// (2-byte aligned), as four dwords of two cells each, read with one 16-byte
// load from the dword boundary at or below a and, when a is not on one, the
// dword after it.  head_ok / tail_ok: the 2 bytes before a / after the eight
// cells may be read (false only at the ends of the buffer); otherwise those
// dwords are replaced by 2-byte reads of the cells' own bytes.
struct __attribute__((packed, aligned(4))) Dw4 {
    uint32_t x, y, z, w;
};
__device__ __forceinline__ void row_cells8(const uint8_t *a, bool head_ok, bool tail_ok, uint32_t u[4]) {
    const uint32_t sh = (uint32_t)(reinterpret_cast<uintptr_t>(a) & 3u);   // 0 or 2
    const uint8_t *A = a - sh;
    uint32_t w0, w1, w2, w3, w4 = 0;
    if (sh == 0 || head_ok) {
        const Dw4 v = *reinterpret_cast<const Dw4 *>(A);
        w0 = v.x;
        w1 = v.y;
        w2 = v.z;
        w3 = v.w;
    } else {   // the first cell's bytes only, placed where the shift takes them from
        w0 = (uint32_t)(*reinterpret_cast<const uint16_t *>(a)) << 16;
        w1 = *reinterpret_cast<const uint32_t *>(A + 4);
        w2 = *reinterpret_cast<const uint32_t *>(A + 8);
        w3 = *reinterpret_cast<const uint32_t *>(A + 12);
    }
    if (sh != 0)
        w4 = tail_ok ? *reinterpret_cast<const uint32_t *>(A + 16)
                     : (uint32_t)(*reinterpret_cast<const uint16_t *>(A + 16));
    u[0] = __builtin_amdgcn_alignbyte(w1, w0, sh);
    u[1] = __builtin_amdgcn_alignbyte(w2, w1, sh);
    u[2] = __builtin_amdgcn_alignbyte(w3, w2, sh);
    u[3] = __builtin_amdgcn_alignbyte(w4, w3, sh);
}

// MaxW: the wavefronts per SIMD the register allocation aims for -- 4 for a
// workgroup alone on its CU (registers spent on overlapping loads), 8 when
// several workgroups share the CU.
// V4: rows read as 16-byte blocks (Lx % 4 == 0 and a 16-byte aligned batch).
template <int M, int S, int MaxW, bool V4>
__global__ void __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(4, MaxW)))
count_bits_kernel(BitDesc bd, int64_t K, const int8_t *__restrict__ species, int32_t *__restrict__ partial,
                  int32_t *__restrict__ counts_out, int32_t *__restrict__ bad_out, const double *__restrict__ tw,
                  double *__restrict__ S_F) {
    constexpr int P = Pairs<M>::P;
    constexpr int NP = Pairs<M>::NP;
    constexpr int NV = S * NP + P;           // per-lane sums
    extern __shared__ __align__(16) uint32_t lds[];
    const int kc = blockIdx.y;
    if (kc >= K) return;
    const int chunk = blockIdx.x;
    const int z0 = chunk * bd.ZC;
    const int nz = min(bd.ZC, bd.Lzc - z0);  // centre layers of this workgroup
    const int nl = nz + bd.hz;               // plus the layers above (dz in 0 .. hz)
    const int PW = bd.PW;
    const int RS = bd.RS;
    const int nplane = nl * 4 * PW * P;      // plane dwords (a multiple of 4)
    uint32_t *cmask = lds + nplane;          // centre mask per word [LW]
    int32_t *red2 = (int32_t *)(cmask + ((bd.LW + 3) & ~3));  // per-lane sums [NV][64], 16-byte aligned
    int32_t *red = red2 + NV * 64;               // totals [NV + 1]
    int32_t *tab = red + NV + 1;                 // (delta, shift) per (basis, half offset)
    for (int i = threadIdx.x; i < 4 * bd.nh; i += blockDim.x) {
        tab[2 * i] = bd.tab_delta[i / bd.nh][i % bd.nh];
        tab[2 * i + 1] = bd.tab_r[i / bd.nh][i % bd.nh];
    }

    // zero planes and sums
    {
        uint4 *p4 = reinterpret_cast<uint4 *>(lds);
        const uint4 z4 = {0u, 0u, 0u, 0u};
        for (int i = threadIdx.x; i < nplane / 4; i += blockDim.x) p4[i] = z4;
    }
    for (int i = threadIdx.x; i < NV * 64 + NV + 1; i += blockDim.x) red2[i] = 0;
    // centre mask: bit t of word w is a real site if its row and column are inside
    for (int w = threadIdx.x; w < bd.LW; w += blockDim.x) {
        const int x0 = 32 * w;
        uint32_t m = 0xFFFFFFFFu;
        const int lo = bd.hy * RS - x0;          // bits below lo lie in the border rows below
        if (lo > 0) m &= lo >= 32 ? 0u : (0xFFFFFFFFu << lo);
        const int hi = (bd.Ly + bd.hy) * RS - x0;   // bits from hi on lie in the border rows above
        if (hi < 32) m &= hi <= 0 ? 0u : (0xFFFFFFFFu >> (32 - hi));
        const int c0 = x0 % RS;                  // column of bit 0
        for (int e = 0; e < bd.hx; ++e) {        // border columns e and RS - 1 - e
            for (int t = (RS + e - c0) % RS; t < 32; t += RS) m &= ~(1u << t);
            for (int t = (2 * RS - 1 - e - c0) % RS; t < 32; t += RS) m &= ~(1u << t);
        }
        cmask[w] = m;
    }
    __syncthreads();

    // ---- 1. conversion: one padded row (layer ll, row fy) per item ------------------
    const uint8_t *cfg = reinterpret_cast<const uint8_t *>(species) + kc * (int64_t)bd.N;
    uint32_t badacc = 0;
    const uint32_t kBad = (0x80u - M) * 0x01010101u;   // byte + kBad has bit 7 set iff byte >= M (bytes < 0x80)
    const int rows = bd.Ly + 2 * bd.hy;
    const int nitems = nl * rows;
    const double inv_rows = 1.0 / rows;
#pragma unroll 1
    for (int it = threadIdx.x; it < nitems; it += blockDim.x) {
        const int ll = qdiv(it, inv_rows);
        const int fy = it - ll * rows;
        int cy = fy - bd.hy;   // in -hy .. Ly + hy - 1
        cy = cy < 0 ? cy + bd.Ly : (cy >= bd.Ly ? cy - bd.Ly : cy);
        cy = cy < 0 || cy >= bd.Ly ? 0 : cy;   // one row (Ly = 1 < hy)
        int cz = z0 + ll;
        while (cz >= bd.Lz) cz -= bd.Lz;
        const uint32_t rowoff = (uint32_t)((cz * bd.Ly + cy) * bd.Lx) * 4u;
        // z-paired BCC: the row's two BCC rows (layers 2 cz and 2 cz + 1 mod Lzs), 2 Lx bytes each
        uint32_t rowlo = 0, rowhi = 0;
        if (bd.zpair) {
            int zl = 2 * cz;
            zl = zl >= bd.Lzs ? zl - bd.Lzs : zl;
            const int zh = zl + 1 >= bd.Lzs ? zl + 1 - bd.Lzs : zl + 1;
            rowlo = (uint32_t)((zl * bd.Ly + cy) * bd.Lx) * 2u;
            rowhi = (uint32_t)((zh * bd.Ly + cy) * bd.Lx) * 2u;
        }
#pragma unroll 1
        for (int cxc = 0; cxc < bd.nchx; ++cxc) {
            constexpr int ND = Digits<M>::ND;
            uint32_t dacc[ND][4];   // digit planes: byte b of dacc[beta][g] = cells 8g..8g+7 of sublattice b
            if constexpr (V4) {
                // rows of whole 16-byte blocks: window block t (0..8) of the chunk is
                // block 8 cxc - 1 + t (mod Lx / 4) of the row, and padded column q of
                // the chunk (cell 32 cxc + q - 1) is word (q + 3) & 3 of window block
                // (q + 3) >> 2.  Only the chunk's ncol padded columns are converted
                // (blocks past the row end wrap to its start: always in bounds).
                const int nb = bd.Lx >> 2;
                const int ncol = min(32, RS - 32 * cxc);   // uniform, >= 1
                // with 4 wavefronts per SIMD every block of the chunk is in flight at
                // once; with 8, the second half's blocks are read after the first
                // half's columns (bounds the registers held by loads in flight)
                constexpr int kFirst = MaxW <= 4 ? 9 : 5;
                uint4 blk[9];
                auto load_blk = [&](int t) {
                    int k = 8 * cxc - 1 + t;
                    k = k < 0 ? k + nb : k;
                    while (k >= nb) k -= nb;
                    blk[t] = *reinterpret_cast<const uint4 *>(cfg + (rowoff + 16u * (uint32_t)k));
                };
#pragma unroll
                for (int t = 0; t < kFirst; ++t) load_blk(t);
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    if (kFirst < 9 && g == 2) {
                        __builtin_amdgcn_sched_barrier(0);
                        if (ncol > 16) {   // uniform
#pragma unroll
                            for (int t = kFirst; t < 9; ++t) load_blk(t);
                        }
                    }
                    uint32_t d8[8];
                    if (8 * g >= ncol) {   // uniform: the whole group lies past the chunk
#pragma unroll
                        for (int b = 0; b < ND; ++b) dacc[b][g] = 0;
                        continue;
                    }
#pragma unroll
                    for (int m = 0; m < 8; ++m) {
                        const int q = 8 * g + m;
                        const int t = (q + 3) >> 2, w = (q + 3) & 3;
                        const uint32_t d = w == 0 ? blk[t].x : w == 1 ? blk[t].y : w == 2 ? blk[t].z : blk[t].w;
                        d8[m] = (8 * g + 8 <= ncol || q < ncol) ? d : 0u;   // columns past the chunk: id 0, masked below
                        badacc |= d8[m] | (d8[m] + kBad);
                    }
                    uint32_t Dg[ND];
                    digits8<ND>(d8, Dg);
#pragma unroll
                    for (int b = 0; b < ND; ++b) dacc[b][g] = Dg[b];
                    __builtin_amdgcn_sched_barrier(0);   // one group of eight columns at a time
                }
            } else {
            // padded column pos holds cell (pos - hx) mod Lx; columns past the row
            // end read some cell and are masked below, so every load is in bounds.
            // GF groups of 8 loads are issued before any of them is used.
            constexpr int GF = MaxW <= 4 ? 4 : 2;
#pragma unroll
            for (int g0 = 0; g0 < 4; g0 += GF) {
                uint32_t d[GF][8];
#pragma unroll
                for (int gg = 0; gg < GF; ++gg) {
                    const int g = g0 + gg;
                    if (32 * cxc + 8 * g >= RS) continue;   // uniform
                    const int c0 = 32 * cxc + 8 * g - bd.hx;
                    // the row's first group: the wrapped cell Lx - 1, then cells 0 .. 6
                    const bool first = c0 == -1 && bd.Lx >= 10;
                    if (bd.zpair && bd.al2 && (first || (c0 >= 0 && c0 + 8 <= bd.Lx))) {   // uniform
                        // wide reads of both BCC rows (cells r0 .. r0 + 7); a row's bytes
                        // before / after them lie in the buffer unless the row opens /
                        // closes it
                        const int r0 = first ? 0 : c0;
                        const bool lo_first = kc == 0 && rowlo == 0, hi_first = kc == 0 && rowhi == 0;
                        const uint32_t last = bd.N - 2u * (uint32_t)bd.Lx;
                        const bool lo_last = kc == K - 1 && rowlo == last, hi_last = kc == K - 1 && rowhi == last;
                        const bool tail = r0 + 8 < bd.Lx;
                        uint32_t ul[4], uh[4];
                        row_cells8(cfg + rowlo + 2u * (uint32_t)r0, r0 > 0 || !lo_first, tail || !lo_last, ul);
                        row_cells8(cfg + rowhi + 2u * (uint32_t)r0, r0 > 0 || !hi_first, tail || !hi_last, uh);
                        uint32_t e[8];   // cells r0 .. r0 + 7 as four-site dwords
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            e[2 * k] = perm(uh[k], ul[k], 0x05040100u);
                            e[2 * k + 1] = perm(uh[k], ul[k], 0x07060302u);
                        }
                        uint32_t w0 = 0;
                        if (first) {   // column m holds cell m - 1: the loaded cells move up one column
                            const uint32_t cl = 2u * (uint32_t)(bd.Lx - 1);
                            const uint32_t a = *reinterpret_cast<const uint16_t *>(cfg + (rowlo + cl));
                            const uint32_t b = *reinterpret_cast<const uint16_t *>(cfg + (rowhi + cl));
                            w0 = a | (b << 16);
                        }
#pragma unroll
                        for (int m = 0; m < 8; ++m) d[gg][m] = first ? (m == 0 ? w0 : e[m - 1]) : e[m];
                        continue;
                    }
#pragma unroll
                    for (int m = 0; m < 8; ++m) {
                        // padded column pos holds cell (pos - hx) mod Lx; columns past
                        // the padded row read some cell and are masked below
                        int c = 32 * cxc + 8 * g + m - bd.hx;
                        c = c < 0 ? c + bd.Lx : (c >= bd.Lx ? c - bd.Lx : c);
                        c = c < 0 || c >= bd.Lx ? 0 : c;   // past the padded row, or a row of one cell
                        if (bd.zpair) {   // uniform: sublattices 0, 1 from the lower BCC row, 2, 3 from the upper
                            const uint32_t a = *reinterpret_cast<const uint16_t *>(cfg + (rowlo + 2u * (uint32_t)c));
                            const uint32_t b = *reinterpret_cast<const uint16_t *>(cfg + (rowhi + 2u * (uint32_t)c));
                            d[gg][m] = a | (b << 16);
                        } else {
                            d[gg][m] = *reinterpret_cast<const uint32_t *>(cfg + (rowoff + 4u * (uint32_t)c));
                        }
                    }
                }
#pragma unroll
                for (int gg = 0; gg < GF; ++gg) {
                    const int g = g0 + gg;
                    uint32_t Dg[ND];
                    if (32 * cxc + 8 * g >= RS) {   // uniform: past the row, masked below
#pragma unroll
                        for (int b = 0; b < ND; ++b) dacc[b][g] = 0;
                        continue;
                    }
#pragma unroll
                    for (int m = 0; m < 8; ++m) badacc |= d[gg][m] | (d[gg][m] + kBad);
                    digits8<ND>(d[gg], Dg);
#pragma unroll
                    for (int b = 0; b < ND; ++b) dacc[b][g] = Dg[b];
                }
            }
            }
            // 4x4 byte transpose: acc[j][g] byte b = bits of positions 8g..8g+7 of sublattice b
            const int o = fy * RS + 32 * cxc;
            const int wd = o >> 5, s = o & 31;
            uint32_t *row0 = lds + (ll * 4 * PW + bd.PADW + wd) * P;
            const int nvalid = RS - 32 * cxc;   // padded columns in this chunk
            const uint32_t keep = nvalid >= 32 ? 0xFFFFFFFFu : (1u << nvalid) - 1u;
            // digit rows per sublattice, then the one-hot planes (bit set where id == j)
            uint32_t RD[ND][4];
#pragma unroll
            for (int b2 = 0; b2 < ND; ++b2) {
                const uint32_t u0 = perm(dacc[b2][1], dacc[b2][0], 0x05010400u);
                const uint32_t u1 = perm(dacc[b2][1], dacc[b2][0], 0x07030602u);
                const uint32_t v0 = perm(dacc[b2][3], dacc[b2][2], 0x05010400u);
                const uint32_t v1 = perm(dacc[b2][3], dacc[b2][2], 0x07030602u);
                RD[b2][0] = perm(v0, u0, 0x05040100u);
                RD[b2][1] = perm(v0, u0, 0x07060302u);
                RD[b2][2] = perm(v1, u1, 0x05040100u);
                RD[b2][3] = perm(v1, u1, 0x07060302u);
            }
            uint32_t R[P][4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                uint32_t Db[ND];
#pragma unroll
                for (int b2 = 0; b2 < ND; ++b2) Db[b2] = RD[b2][b];
#pragma unroll
                for (int j = 0; j < P; ++j) R[j][b] = onehot_plane<ND>(Db, j) & keep;
            }
            // planes j and j + 1 of a word are adjacent dwords (8-byte aligned for
            // even j when P is even): one 64-bit OR for both
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                uint32_t *dst = row0 + b * PW * P;
#pragma unroll
                for (int j = 0; j < P; j += (P % 2 == 0 ? 2 : 1)) {
                    if constexpr (P % 2 == 0) {
                        const uint64_t lo = ((uint64_t)(R[j + 1][b] << s) << 32) | (R[j][b] << s);
                        const uint64_t hi = ((uint64_t)((R[j + 1][b] >> 1) >> (31 - s)) << 32) |
                                            ((R[j][b] >> 1) >> (31 - s));
                        atomicOr(reinterpret_cast<unsigned long long *>(dst + j), (unsigned long long)lo);
                        atomicOr(reinterpret_cast<unsigned long long *>(dst + P + j), (unsigned long long)hi);
                    } else {
                        atomicOr(dst + j, R[j][b] << s);
                        atomicOr(dst + P + j, (R[j][b] >> 1) >> (31 - s));
                    }
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
    const int lane = threadIdx.x & 63;
    int32_t *slots = red2 + S * NP * 64 + lane;   // this lane's species-total slots
    // Basis-major order with each basis's words padded to whole wavefronts makes
    // the basis uniform per wavefront: its offset table then comes through scalar
    // loads, and offsets with no bit shift skip the funnel shift.  Taken when the
    // padding adds at most a tenth of the words; otherwise words in layer-major
    // order, each lane reading its basis's table from LDS.
    const int nbw = nz * bd.NCW;                 // centre words per basis
    const int nbw64 = (nbw + 63) & ~63;
    const double inv_ncw = 1.0 / bd.NCW;
    if (10 * nbw64 <= 11 * nbw) {
        const int nwork = 4 * nbw64;
        const double inv_nbw = 1.0 / nbw64;
#pragma unroll 1
        for (int it = threadIdx.x; it < nwork; it += blockDim.x) {
            const int bu = __builtin_amdgcn_readfirstlane(qdiv(it, inv_nbw));
            const int rem = it - bu * nbw64;
            if (rem >= nbw) continue;   // padding
            const int ll = qdiv(rem, inv_ncw);
            // z-paired BCC with an odd Lzs: the last centre layer's upper BCC layer repeats layer 0
            if (bu >= 2 && bd.half_last && z0 + ll == bd.Lzc - 1) continue;
            const int w = bd.cw0 + rem - ll * bd.NCW;
            const uint32_t *lbase = lds + (ll * 4 * PW + bd.PADW + w) * P;
            uint32_t Pv[P], Un[NP];
            centre_word<M>(lbase + bu * PW * P, cmask[w], slots, Pv, Un);
#pragma unroll
            for (int k = 0; k < S; ++k) {
#pragma unroll 1
                for (int h = bd.hstart[k]; h < bd.hstart[k + 1]; ++h) {
                    const int r = bd.tab_r[bu][h];
                    const uint32_t *nb = lbase + bd.tab_delta[bu][h];
                    uint32_t Q[P];
                    lds_planes<P>(nb, Q);
                    if (r != 0) {
                        uint32_t hi[P];
                        lds_planes<P>(nb + P, hi);
#pragma unroll
                        for (int j = 0; j < P; ++j) Q[j] = __builtin_amdgcn_alignbit(hi[j], Q[j], (uint32_t)r);
                    }
                    count_offset<M>(acc[k], Pv, Un, Q);
                }
            }
        }
    } else {
        const int nwork = nz * 4 * bd.NCW;
#pragma unroll 1
        for (int it = threadIdx.x; it < nwork; it += blockDim.x) {
            const int lb = qdiv(it, inv_ncw);      // layer * 4 + basis
            const int w = bd.cw0 + it - lb * bd.NCW;
            const int b = lb & 3;
            const int ll = lb >> 2;
            if (b >= 2 && bd.half_last && z0 + ll == bd.Lzc - 1) continue;   // as above
            const uint32_t *lbase = lds + (ll * 4 * PW + bd.PADW + w) * P;
            uint32_t Pv[P], Un[NP];
            centre_word<M>(lbase + b * PW * P, cmask[w], slots, Pv, Un);
            const int32_t *tb = tab + 2 * b * bd.nh;
#pragma unroll
            for (int k = 0; k < S; ++k) {
#pragma unroll 1
                for (int h = bd.hstart[k]; h < bd.hstart[k + 1]; ++h) {
                    const uint32_t *nb = lbase + tb[2 * h];
                    const uint32_t r = (uint32_t)tb[2 * h + 1];
                    uint32_t lo[P], hi[P], Q[P];
                    lds_planes<P>(nb, lo);
                    lds_planes<P>(nb + P, hi);
#pragma unroll
                    for (int j = 0; j < P; ++j) Q[j] = __builtin_amdgcn_alignbit(hi[j], lo[j], r);
                    count_offset<M>(acc[k], Pv, Un, Q);
                }
            }
        }
    }
    // ---- 3. reduce over the workgroup: per-lane slots, then one lane per value ----
    {
#pragma unroll
        for (int k = 0; k < S; ++k)
#pragma unroll
            for (int q = 0; q < NP; ++q) atomicAdd(&red2[(k * NP + q) * 64 + lane], acc[k][q]);
        const uint64_t anybad = __ballot((badacc & 0x80808080u) != 0);
        if (lane == 0 && anybad) atomicOr(&red[NV], 1);
        __syncthreads();
        // one lane per value adds its 64 slots (16-byte reads, rotated per lane
        // so that lanes start on different banks)
        if (threadIdx.x < NV) {
            const int v = threadIdx.x;
            const uint4 *row = reinterpret_cast<const uint4 *>(red2 + v * 64);
            uint32_t t = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const uint4 x = row[(j + v) & 15];
                t += x.x + x.y + x.z + x.w;
            }
            red[v] = (int32_t)t;
        }
    }
    __syncthreads();
    if (bd.nchunks > 1) {
        // this workgroup's own slot; the finishing kernel adds the slots up
        int32_t *out = partial + ((int64_t)kc * bd.nchunks + chunk) * bd.partial_stride;
        for (int i = threadIdx.x; i < NV + 1; i += blockDim.x) out[i] = red[i];
        return;
    }
    // ---- 4. one workgroup holds the whole configuration: counts and Eq. 2-3 here ----
    // epilogue scratch after the offset table: [S][M][M] counts, [S][M][M] and [S][M] doubles
    int32_t *lc = tab + 8 * bd.nh;
    double *lsq = reinterpret_cast<double *>((reinterpret_cast<uintptr_t>(lc + S * M * M) + 7) & ~uintptr_t(7));
    epilogue<M, S>(red, bd, lc, lsq, lsq + S * M * M, counts_out + kc * (int64_t)(S * M * M), bad_out + kc, tw,
                   S_F ? S_F + 2 * kc : nullptr);
}


// The sums of one configuration from its workgroups' slots [nchunks][stride]
// into sum [NV + 1] (the last entry ORs the bad-species flags).
template <int M, int S>
__device__ __forceinline__ void add_slots(const int32_t *slots, const BitDesc &bd, int i0, int di, int32_t *sum) {
    constexpr int NV = S * Pairs<M>::NP + M - 1;
    for (int i = i0; i < NV + 1; i += di) {
        int32_t v = 0;
        for (int c = 0; c < bd.nchunks; ++c) v = i < NV ? v + slots[c * bd.partial_stride + i] : (v | slots[c * bd.partial_stride + i]);
        sum[i] = v;
    }
}

// slot sums -> counts, and Eq. 2-3 when S_F is given (one 64-thread block per
// configuration: the slot sums, the entries and the rows are spread over its lanes)
template <int M, int S>
__global__ void __launch_bounds__(64) finalize_objective_kernel(BitDesc bd, const int32_t *__restrict__ partial,
                                                               int32_t *__restrict__ counts,
                                                               int32_t *__restrict__ bad,
                                                               const double *__restrict__ tw,
                                                               double *__restrict__ S_F) {
    __shared__ int32_t lsum[S * Pairs<M>::NP + M];
    __shared__ int32_t lc[S * M * M];
    __shared__ double lsq[S * M * M];
    __shared__ double lrow[S * M];
    const int64_t kc = blockIdx.x;
    add_slots<M, S>(partial + kc * bd.nchunks * (int64_t)bd.partial_stride, bd, threadIdx.x, blockDim.x, lsum);
    __syncthreads();
    epilogue<M, S>(lsum, bd, lc, lsq, lrow, counts + kc * (int64_t)(S * M * M), bad + kc, tw,
                   S_F ? S_F + 2 * kc : nullptr);
}


// ---------------------------------------------------------------------------
// Streaming form for batches of configurations.
//
// A workgroup takes whole configurations (kc = blockIdx.x, + gridDim.x, ...)
// and walks each along z in groups of G centre layers.  The bytes of a layer
// reach LDS by direct global-to-LDS loads (global_load_lds_dword: each
// wavefront instruction moves 64 consecutive positions of the padded layer, so
// the periodic border is just another source address and the loads are
// coalesced); the loads of the next-but-one chunk of layers are issued before
// the current group is counted, so HBM traffic overlaps the counting.
// Conversion then works on whole destination words: word w of a padded layer
// is 32 consecutive padded positions, i.e. 128 consecutive staged bytes, so it
// needs no atomics and no bit shifts.  Plane slots form a ring of G + 1 layers
// (layer l in slot l mod (G + 1)) plus one slot that keeps layer 0 for the
// wrap of the last layer.
//
// Step s of a workgroup is (configuration j, group g).  Chunk 0 of a
// configuration is layers 0..G, chunk g >= 1 layers gG+1..gG+G (capped at
// Lz-1); group g's centre layers gG..gG+G-1 need chunks 0..g.  Per step:
//   count group s | wait for own loads, barrier | convert chunk s+1 | barrier |
//   issue the loads of chunk s+2
// ---------------------------------------------------------------------------

using lds_void_t = __attribute__((address_space(3))) void;
using glb_cvoid_t = __attribute__((address_space(1))) const void;

// first and last layer of chunk g (chunk 0: layers 0..G; chunk g: gG+1..gG+G; capped at Lz - 1)
__device__ __forceinline__ void chunk_range(int g, int G, int Lz, int &first, int &last) {
    first = g == 0 ? 0 : g * G + 1;
    last = min(g * G + G, Lz - 1);
}

// plane slot of layer l: layer 0 (and its periodic copy Lz) in slot G + 1, others l mod (G + 1)
__device__ __forceinline__ int slot_of(int l, int G, int Lz) { return (l == 0 || l == Lz) ? G + 1 : l % (G + 1); }

// Direct global-to-LDS loads of layers first..last of one configuration into
// the staged layers: load block n (64 consecutive padded positions) of a layer
// is issued by wavefront n mod nwaves; doff holds this lane's source cells.
template <int MAXD>
__device__ __forceinline__ void stream_issue(const uint8_t *cfg, int first, int last, uint32_t layer_bytes,
                                             uint32_t *raw, int raw_dw, int ndma, int wave, int nwaves,
                                             const uint32_t *doff) {
    for (int l = first; l <= last; ++l) {
        const uint8_t *lb = cfg + (uint32_t)l * layer_bytes;
        uint32_t *dst = raw + (l - first) * raw_dw;
#pragma unroll
        for (int i = 0; i < MAXD; ++i) {
            const int n = wave + i * nwaves;
            const uint32_t cell = i % 2 == 0 ? doff[i / 2] & 0xFFFFu : doff[i / 2] >> 16;
            if (n < ndma)
                __builtin_amdgcn_global_load_lds((glb_cvoid_t *)(lb + 4u * cell), (lds_void_t *)(dst + 64 * n), 4, 0,
                                                 0);
        }
    }
}

// Staged layers first..last -> their plane slots, one destination word per
// item: word w is 32 consecutive padded positions = 128 staged bytes.  Returns
// this lane's bad-species bits.
template <int M>
__device__ __forceinline__ uint32_t stream_convert(const uint32_t *raw, uint32_t *planes, int first, int last, int G,
                                                   int Lz, int LW, int raw_dw, int slot_dw, int PADW, int PW,
                                                   double inv_lw, int tid, int nthreads) {
    constexpr int P = Pairs<M>::P;
    constexpr int PP = (P + 1) & ~1;
    constexpr int ND = Digits<M>::ND;
    const uint32_t kBad = (0x80u - M) * 0x01010101u;   // byte + kBad has bit 7 set iff byte >= M (bytes < 0x80)
    const int nitems = (last - first + 1) * LW;
    uint32_t badacc = 0;
#pragma unroll 1
    for (int it = tid; it < nitems; it += nthreads) {
        const int li = qdiv(it, inv_lw);
        const int w = it - li * LW;
        const uint4 *src = reinterpret_cast<const uint4 *>(raw + li * raw_dw + 32 * w);
        uint32_t dacc[ND][4];   // byte b of dacc[beta][g]: digit beta of cells 8g..8g+7, sublattice b
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
            // eight cells (two 16-byte reads) at a time: bounds the registers in flight
            const uint4 va = src[2 * gq], vb = src[2 * gq + 1];
            const uint32_t d8[8] = {va.x, va.y, va.z, va.w, vb.x, vb.y, vb.z, vb.w};
#pragma unroll
            for (int m = 0; m < 8; ++m) badacc |= d8[m] | (d8[m] + kBad);
            uint32_t Dg[ND];
            digits8<ND>(d8, Dg);
#pragma unroll
            for (int b2 = 0; b2 < ND; ++b2) dacc[b2][gq] = Dg[b2];
            __builtin_amdgcn_sched_barrier(0);
        }
        // 4x4 byte transposes give the digit rows of each sublattice, then the one-hot planes
        uint32_t *dst = planes + slot_of(first + li, G, Lz) * slot_dw + (PADW + w) * PP;
        uint32_t RD[ND][4];
#pragma unroll
        for (int b2 = 0; b2 < ND; ++b2) {
            const uint32_t u0 = perm(dacc[b2][1], dacc[b2][0], 0x05010400u);
            const uint32_t u1 = perm(dacc[b2][1], dacc[b2][0], 0x07030602u);
            const uint32_t v0 = perm(dacc[b2][3], dacc[b2][2], 0x05010400u);
            const uint32_t v1 = perm(dacc[b2][3], dacc[b2][2], 0x07030602u);
            RD[b2][0] = perm(v0, u0, 0x05040100u);
            RD[b2][1] = perm(v0, u0, 0x07060302u);
            RD[b2][2] = perm(v1, u1, 0x05040100u);
            RD[b2][3] = perm(v1, u1, 0x07060302u);
        }
        uint32_t R[4][PP];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            uint32_t Db[ND];
#pragma unroll
            for (int b2 = 0; b2 < ND; ++b2) Db[b2] = RD[b2][b];
#pragma unroll
            for (int jj = 0; jj < P; ++jj) R[b][jj] = onehot_plane<ND>(Db, jj);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
#pragma unroll
            for (int jj = P; jj < PP; ++jj) R[b][jj] = 0;
            uint32_t *o = dst + b * PW * PP;
            if constexpr (PP % 4 == 0) {
#pragma unroll
                for (int jj = 0; jj < PP; jj += 4)
                    *reinterpret_cast<uint4 *>(o + jj) = make_uint4(R[b][jj], R[b][jj + 1], R[b][jj + 2], R[b][jj + 3]);
            } else {
#pragma unroll
                for (int jj = 0; jj < PP; jj += 2) *reinterpret_cast<uint2 *>(o + jj) = make_uint2(R[b][jj], R[b][jj + 1]);
            }
        }
    }
    return badacc;
}

template <int M, int S, int MAXD>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 8)))
count_stream_kernel(StreamDesc sd, int64_t K, const int8_t *__restrict__ species, int32_t *__restrict__ counts_out,
                    int32_t *__restrict__ bad_out, const double *__restrict__ tw, double *__restrict__ S_F) {
    constexpr int P = Pairs<M>::P;
    constexpr int NP = Pairs<M>::NP;
    constexpr int PP = (P + 1) & ~1;          // dwords per (basis, word): the planes, padded to even
    constexpr int NV = S * NP + P;
    extern __shared__ __align__(16) uint32_t lds[];
    uint32_t *raw = lds;                                   // (G + 1) staged layers
    uint32_t *planes = lds + sd.o_planes;                  // (G + 2) plane slots
    int32_t *red2 = reinterpret_cast<int32_t *>(lds + sd.o_red2);   // per-lane sums [NV][64]
    int32_t *red = reinterpret_cast<int32_t *>(lds + sd.o_red);     // totals [NV], bad, flags [2]
    int32_t *badflag = red + NV + 1;

    const int nthreads = blockDim.x;
    const int nwaves = nthreads >> 6;
    const int G = sd.G;
    const int Lz = sd.Lz;
    const int ng = sd.ngroups;
    const int PW = sd.PW;
    const int NCW = sd.NCW;
    const int npos = (sd.Ly + 2) * sd.RS;
    const uint32_t layer_bytes = (uint32_t)sd.Lx * (uint32_t)sd.Ly * 4u;

    // source cell (within a layer) of each padded position this lane loads:
    // position p = 64 n + lane of load block n = wave + i * nwaves holds cell
    // ((p mod RS) - 1 mod Lx, (p div RS) - 1 mod Ly); positions past the padded
    // layer read cell 0 (in bounds, a valid id, never a neighbour of a centre
    // site).  Two 16-bit fields per register (a layer has < 65,536 cells).
    uint32_t doff[MAXD / 2];
    {
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
        for (int i = 0; i < MAXD; ++i) {
            const int p = 64 * (wave + i * nwaves) + lane;
            uint32_t o = 0;
            if (p < npos) {
                const int py = p / sd.RS;
                const int px = p - py * sd.RS;
                int y = py - 1, x = px - 1;
                y = y < 0 ? sd.Ly - 1 : (y >= sd.Ly ? 0 : y);
                x = x < 0 ? sd.Lx - 1 : (x >= sd.Lx ? 0 : x);
                o = (uint32_t)(y * sd.Lx + x);
            }
            if (i % 2 == 0)
                doff[i / 2] = o;
            else
                doff[i / 2] |= o << 16;
        }
        // centre mask: bit t of word w is a real site if its row and column are inside
        for (int w = tid; w < sd.LW; w += nthreads) {
            const int RS = sd.RS;
            const int x0 = 32 * w;
            uint32_t m = 0xFFFFFFFFu;
            const int lo = RS - x0;
            if (lo > 0) m &= lo >= 32 ? 0u : (0xFFFFFFFFu << lo);
            const int hi = (sd.Ly + 1) * RS - x0;
            if (hi < 32) m &= hi <= 0 ? 0u : (0xFFFFFFFFu >> (32 - hi));
            const int c0 = x0 % RS;
            for (int t = (RS - c0) % RS; t < 32; t += RS) m &= ~(1u << t);
            for (int t = (2 * RS - 1 - c0) % RS; t < 32; t += RS) m &= ~(1u << t);
            lds[sd.o_cmask + w] = m;
        }
        for (int i = tid; i < NV * 64; i += nthreads) red2[i] = 0;
        if (tid < NV + 3) red[tid] = 0;
    }
    __syncthreads();

    if ((int64_t)blockIdx.x >= K) return;
    const int64_t ncfg = (K - 1 - (int64_t)blockIdx.x) / gridDim.x + 1;
    const int64_t nsteps = ncfg * ng;
    const double inv_lw = 1.0 / sd.LW;
    const double inv_ncw = 1.0 / NCW;
    const uint8_t *cfg0 = reinterpret_cast<const uint8_t *>(species) + (int64_t)blockIdx.x * sd.N;
    const int64_t cfg_stride = (int64_t)gridDim.x * sd.N;

    // prologue: chunk 0 staged and converted, chunk 1 on its way
    {
        const int tid = threadIdx.x;
        int first, last;
        chunk_range(0, G, Lz, first, last);
        stream_issue<MAXD>(cfg0, first, last, layer_bytes, raw, sd.raw_dw, sd.ndma, tid >> 6, nwaves, doff);
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        __syncthreads();
        const uint32_t bad = stream_convert<M>(raw, planes, first, last, G, Lz, sd.LW, sd.raw_dw, sd.slot_dw, sd.PADW,
                                               PW, inv_lw, tid, nthreads);
        if (__ballot((bad & 0x80808080u) != 0) && (tid & 63) == 0) atomicOr(&badflag[0], 1);
        __syncthreads();
        if (nsteps > 1) {
            const int64_t j1 = 1 / ng;
            chunk_range((int)(1 - j1 * ng), G, Lz, first, last);
            stream_issue<MAXD>(cfg0 + j1 * cfg_stride, first, last, layer_bytes, raw, sd.raw_dw, sd.ndma, tid >> 6,
                               nwaves, doff);
        }
    }

#pragma unroll 1
    for (int64_t s = 0; s < nsteps; ++s) {
        // the thread index is re-read through an empty asm each step so that
        // addresses derived from it are not hoisted out of this loop (they
        // would otherwise stay live across it and spill)
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int lane = tid & 63;
        const int64_t j = s / ng;
        const int g = (int)(s - j * ng);
        const bool last = g == ng - 1;   // uniform

        // ---- count group g of configuration j: items (basis, layer, centre word),
        // basis-major, each basis padded to whole wavefronts (uniform basis)
        int32_t acc[S][NP];
        int32_t ntot[P];
#pragma unroll
        for (int k = 0; k < S; ++k)
#pragma unroll
            for (int q = 0; q < NP; ++q) acc[k][q] = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) ntot[i] = 0;
        {
            const int z0 = g * G;
            const int nz = min(G, Lz - z0);
            const int s0 = z0 % (G + 1);   // slot of layer z0 (z0 > 0), uniform
            const int nbw = nz * NCW;
            const int nbw64 = (nbw + 63) & ~63;
            const int nwork = 4 * nbw64;
            const uint32_t *cmask = lds + sd.o_cmask;
#pragma unroll 1
            for (int it = tid; it < nwork; it += nthreads) {
                const int bu = __builtin_amdgcn_readfirstlane(it - lane) / nbw64;
                const int rem = it - bu * nbw64;
                if (rem >= nbw) continue;   // padding
                const int li = qdiv(rem, inv_ncw);
                const int w = sd.cw0 + rem - li * NCW;
                const int l = z0 + li;
                // slot of layer l: (s0 + li) mod (G + 1), with layers 0 and Lz in slot G + 1
                int sl0 = s0 + li, sl1 = s0 + li + 1;
                sl0 = sl0 > G ? sl0 - (G + 1) : sl0;
                sl1 = sl1 > G ? sl1 - (G + 1) : sl1;
                sl0 = l == 0 ? G + 1 : sl0;
                sl1 = l + 1 == Lz ? G + 1 : sl1;
                const uint32_t *c0 = planes + sl0 * sd.slot_dw + (sd.PADW + w) * PP;
                const uint32_t *c1 = planes + sl1 * sd.slot_dw + (sd.PADW + w) * PP;
                uint32_t Pv[PP], Un[NP];
                lds_planes<PP>(c0 + bu * PW * PP, Pv);
                const uint32_t cm = cmask[w];
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    Pv[i] &= cm;
                    ntot[i] += (int32_t)__popc(Pv[i]);
                }
#pragma unroll
                for (int i = 0; i < P; ++i)
#pragma unroll
                    for (int jj = i + 1; jj < P; ++jj) Un[Pairs<M>::q(i, jj)] = Pv[i] | Pv[jj];
#pragma unroll
                for (int dz = 0; dz < 2; ++dz) {
                    const uint32_t *cb = dz ? c1 : c0;
#pragma unroll
                    for (int k = 0; k < S; ++k) {
#pragma unroll 1
                        for (int h = sd.hs[bu][dz][k]; h < sd.hs[bu][dz][k + 1]; ++h) {
                            const int v = sd.tab[bu][h];
                            const uint32_t r = (uint32_t)v & 31u;
                            const uint32_t *nb = cb + (v >> 5);
                            uint32_t Q[PP];
                            lds_planes<PP>(nb, Q);
                            if (r != 0) {
                                uint32_t hi[PP];
                                lds_planes<PP>(nb + PP, hi);
#pragma unroll
                                for (int jj = 0; jj < P; ++jj) Q[jj] = __builtin_amdgcn_alignbit(hi[jj], Q[jj], r);
                            }
                            count_offset<M>(acc[k], Pv, Un, Q);
                        }
                    }
                }
            }
        }
        // this step's sums go to the lane's slots now, so that no accumulator
        // stays live through the conversion below (it bounds the registers)
#pragma unroll
        for (int k = 0; k < S; ++k)
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                atomicAdd(&red2[(k * NP + q) * 64 + lane], acc[k][q]);
                acc[k][q] = 0;
            }
#pragma unroll
        for (int i = 0; i < P; ++i) {
            atomicAdd(&red2[(S * NP + i) * 64 + lane], ntot[i]);
            ntot[i] = 0;
        }
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wavefront's loads of chunk s + 1 are in LDS
        __syncthreads();
        if (last) {
            if (tid < NV) {
                // one lane per value adds its 64 slots (16-byte reads, rotated start bank)
                const uint4 *row = reinterpret_cast<const uint4 *>(red2 + tid * 64);
                uint32_t t = 0;
#pragma unroll 2
                for (int u = 0; u < 16; ++u) {
                    const uint4 x = row[(u + tid) & 15];
                    t += x.x + x.y + x.z + x.w;
                }
                red[tid] = (int32_t)t;
            } else if (tid == NV) {
                red[NV] = badflag[j & 1];
                badflag[j & 1] = 0;
            }
        }
        if (s + 1 < nsteps) {
            const int64_t j1 = (s + 1) / ng;
            int first, lastl;
            chunk_range((int)(s + 1 - j1 * ng), G, Lz, first, lastl);
            const uint32_t bad = stream_convert<M>(raw, planes, first, lastl, G, Lz, sd.LW, sd.raw_dw, sd.slot_dw,
                                                   sd.PADW, PW, inv_lw, tid, nthreads);
            if (__ballot((bad & 0x80808080u) != 0) && lane == 0) atomicOr(&badflag[j1 & 1], 1);
        }
        __syncthreads();
        if (last) {
            for (int i = tid; i < NV * 64; i += nthreads) red2[i] = 0;
            const int64_t kc = (int64_t)blockIdx.x + j * gridDim.x;
            int32_t *lc = reinterpret_cast<int32_t *>(lds + sd.o_epi);
            double *lsq = reinterpret_cast<double *>(lds + sd.o_epi + ((S * M * M + 1) & ~1));
            epilogue<M, S>(red, sd, lc, lsq, lsq + S * M * M, counts_out + kc * (int64_t)(S * M * M), bad_out + kc,
                           tw, S_F ? S_F + 2 * kc : nullptr, tid);
        }
        // likewise the load offsets (their 64-bit forms would otherwise be hoisted)
#pragma unroll
        for (int i = 0; i < MAXD / 2; ++i) asm volatile("" : "+v"(doff[i]));
        if (s + 2 < nsteps) {
            const int64_t j2 = (s + 2) / ng;
            int first, lastl;
            chunk_range((int)(s + 2 - j2 * ng), G, Lz, first, lastl);
            stream_issue<MAXD>(cfg0 + j2 * cfg_stride, first, lastl, layer_bytes, raw, sd.raw_dw, sd.ndma, tid >> 6,
                               nwaves, doff);
        }
    }
}

template <int M, int S>
hipError_t launch_ms(const BitDesc &bd, int64_t K, const int8_t *species, int32_t *partial, int32_t *counts,
                     int32_t *bad, const double *tw, double *S_F, hipStream_t stream) {
    const int P = M - 1;
    const int NV = S * Pairs<M>::NP + P;
    const size_t lds = ((size_t)(bd.ZC + bd.hz) * 4 * P * bd.PW + ((bd.LW + 3) & ~3) + NV * 64 + NV + 1 + 8 * bd.nh + 1 +
                        3 * S * M * M + 2 * S * M + 2) * 4;
    const bool lone = bd.threads > 512;   // one workgroup per CU
    using KernelFn = void (*)(BitDesc, int64_t, const int8_t *, int32_t *, int32_t *, int32_t *, const double *,
                              double *);
    const KernelFn fn = lone ? (bd.vec4 ? count_bits_kernel<M, S, 4, true> : count_bits_kernel<M, S, 4, false>)
                             : (bd.vec4 ? count_bits_kernel<M, S, 8, true> : count_bits_kernel<M, S, 8, false>);
    hipError_t e = set_max_lds((const void *)fn, lds);
    if (e != hipSuccess) return e;
    for (int64_t k0 = 0; k0 < K; k0 += 65535) {
        const int64_t kn = std::min<int64_t>(65535, K - k0);
        hipLaunchKernelGGL(fn, dim3(bd.nchunks, (unsigned)kn), dim3(bd.threads), lds, stream, bd, kn,
                           species + k0 * (int64_t)bd.N, partial + k0 * bd.nchunks * bd.partial_stride,
                           counts + k0 * (int64_t)(S * M * M), bad + k0, tw, S_F ? S_F + 2 * k0 : nullptr);
    }
    if (bd.nchunks > 1)
        hipLaunchKernelGGL((finalize_objective_kernel<M, S>), dim3((unsigned)K), dim3(64), 0, stream, bd, partial,
                           counts, bad, tw, S_F);
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

// Cell delta and target sublattice of offset t from sublattice b of a
// four-site cell (an FCC cell, or two BCC cells along x: BCC site (2X + e,
// b & 1) of four-site cell X, e = b >> 1).
// Four-site cells: an FCC cell, or two BCC cells adjacent along `axis` (0 = x,
// 2 = z); sublattice 2 e + b is BCC basis b of the pair's cell e.  Cell delta
// dc and sublattice bt of the target of offset t from sublattice b.
static void four_site_target(const Geometry &g, int axis, int b, int t, int dc[3], int *bt) {
    if (g.lattice == PYHEA_FCC) {
        offset_target(g, b, t, dc, bt);
        return;
    }
    const int e = b >> 1;
    int dcb[3], btb;
    offset_target(g, b & 1, t, dcb, &btb);
    const int x = e + dcb[axis];
    const int X = x >= 0 ? x / 2 : -((1 - x) / 2);
    dc[0] = dcb[0];
    dc[1] = dcb[1];
    dc[2] = dcb[2];
    dc[axis] = X;
    *bt = 2 * (x - 2 * X) + btb;
}

bool fill_bit_desc(const Geometry &g, int lds_budget, int64_t K, int split, BitDesc *bd) {
    std::memset(bd, 0, sizeof(*bd));
    if (!pick(g.M, g.S)) return false;
    // Cells of four sites: an FCC cell, or two BCC cells along x (site id
    // ((cz Ly + cy) Lx + cx) 2 + b is ((cz Ly + cy) (Lx/2) + cx/2) 4 + 2 (cx % 2) + b,
    // so an even-Lx BCC configuration is laid out as cells of four sublattices).
    // With Lx odd the pairs run along z instead: four-site layer z holds BCC
    // layers 2z and 2z + 1, read as two rows of 2 Lx bytes.  An odd Lz makes the
    // pairs wrap: the layout then holds the configuration twice along z (Lz
    // four-site layers = 2 Lz BCC layers, periodic with period Lz, so every
    // centre sees the neighbours it has in the configuration) and counts only
    // the first copy's sites as centres.
    int Lx4, Lz4 = g.L[2], Lzc = g.L[2], zpair = 0, half_last = 0;
    if (g.lattice == PYHEA_FCC) {
        Lx4 = g.L[0];
    } else if (g.lattice == PYHEA_BCC && g.L[0] % 2 == 0) {
        Lx4 = g.L[0] / 2;
    } else if (g.lattice == PYHEA_BCC) {
        Lx4 = g.L[0];
        zpair = 1;
        if (g.L[2] % 2 == 0) {
            Lz4 = Lzc = g.L[2] / 2;
        } else {
            Lz4 = g.L[2];
            Lzc = (g.L[2] + 1) / 2;
            half_last = 1;
        }
    } else {
        return false;
    }
    const int P = g.M - 1;
    // the layout's border: every kept half-offset's target lies within hx cells
    // along x, hy along y and 0 .. hz layers up (1 each for shells whose
    // neighbours lie at most one cell away; 2 for BCC shell 4)
    const int axis = zpair ? 2 : 0;
    int hx = 1, hy = 1, hz = 1;
    for (int t = g.zstart[0]; t < g.zstart[g.S]; ++t) {
        const int dx = g.off[t][0], dy = g.off[t][1], dz = g.off[t][2];
        if (!(dz > 0 || (dz == 0 && (dy > 0 || (dy == 0 && dx > 0))))) continue;
        for (int b = 0; b < 4; ++b) {
            int dc[3], bt;
            four_site_target(g, axis, b, t, dc, &bt);
            if (dc[2] < 0) return false;
            hx = std::max(hx, std::abs(dc[0]));
            hy = std::max(hy, std::abs(dc[1]));
            hz = std::max(hz, dc[2]);
        }
    }
    if (hx > 2 || hy > 2 || hz > 2) return false;
    bd->hx = hx;
    bd->hy = hy;
    bd->hz = hz;
    bd->Lx = Lx4;
    bd->Ly = g.L[1];
    bd->Lz = Lz4;
    bd->zpair = zpair;
    bd->Lzs = g.L[2];
    bd->Lzc = Lzc;
    bd->half_last = half_last;
    bd->RS = Lx4 + 2 * hx;
    const int bits = (g.L[1] + 2 * hy) * bd->RS;
    bd->LW = (bits + 31) / 32;
    bd->PADW = (hy * bd->RS + hx + 1 + 31) / 32 + 1;
    bd->PW = bd->LW + 2 * bd->PADW;
    bd->cw0 = hy * bd->RS / 32;
    bd->NCW = ((g.L[1] + hy) * bd->RS - 1) / 32 - bd->cw0 + 1;
    bd->nchx = (bd->RS + 31) / 32;
    bd->N = (uint32_t)g.N;
    const int np = P * (P + 1) / 2;
    bd->partial_stride = ((g.S * np + P + 1) + 3) & ~3;
    for (int k = 0; k < kMaxShells; ++k) bd->zk[k] = k < g.S ? g.z[k] : 0;
    // largest z-chunk whose planes fit in LDS
    const int nv = g.S * np + P;
    const int fixed = (((bd->LW + 3) & ~3) + nv * 64 + nv + 1 + 8 * kMaxOffsets / 2 + 3 * g.S * g.M * g.M + 2 * g.S * g.M + 3) * 4;
    const int per_layer = 4 * P * bd->PW * 4;
    // split > 1: a configuration whose layers would take more than 1/split of a
    // CU's LDS is cut along z so that `split` workgroups share each CU
    const int budget = split > 1 && fixed + (Lzc + hz) * per_layer > lds_budget / split ? lds_budget / split
                                                                                         : lds_budget;
    int zc = (budget - fixed) / per_layer - hz;
    if (zc < 1) return false;
    zc = std::min(zc, Lzc);
    zc = (Lzc + (Lzc + zc - 1) / zc - 1) / ((Lzc + zc - 1) / zc);
    // few configurations: spread each over up to 512 / K workgroups along z
    const int64_t want = std::max<int64_t>(1, 512 / std::max<int64_t>(K, 1));
    if (want > 1) zc = std::min<int64_t>(zc, std::max<int64_t>(2, (Lzc + want - 1) / want));
    bd->ZC = zc;
    bd->nchunks = (Lzc + zc - 1) / zc;
    // a workgroup that needs more than half the LDS runs alone on its CU: give it
    // 16 wavefronts so the CU still has latency to hide behind
    bd->threads = fixed + (zc + hz) * per_layer > lds_budget / 2 ? 1024 : 512;
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
                four_site_target(g, axis, b, t, dc, &bt);
                // plane word of the neighbour: layer +dz, sublattice bt, bit shift s
                const int s = dc[1] * bd->RS + dc[0];
                const int q = s >= 0 ? s / 32 : -((-s + 31) / 32);
                const int r = s - 32 * q;
                bd->tab_delta[b][nh] = ((dc[2] * 4 + bt) * bd->PW + q) * P;
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
    BitDesc b = bd;
    b.vec4 = !bd.zpair && bd.hx == 1 && bd.Lx % 4 == 0 && (reinterpret_cast<uintptr_t>(species) & 15) == 0 ? 1 : 0;
    b.al2 = (reinterpret_cast<uintptr_t>(species) & 1) == 0 ? 1 : 0;
    return f(b, K, species, partial, counts, bad, tw, S_F, stream);
}


namespace {

template <int M, int S>
hipError_t launch_stream_ms(const StreamDesc &sd, int64_t K, const int8_t *species, int32_t *counts, int32_t *bad,
                            const double *tw, double *S_F, hipStream_t stream) {
    using KernelFn = void (*)(StreamDesc, int64_t, const int8_t *, int32_t *, int32_t *, const double *, double *);
    const KernelFn fn = sd.maxd <= 8 ? count_stream_kernel<M, S, 8> : count_stream_kernel<M, S, 16>;
    hipError_t e = set_max_lds((const void *)fn, sd.lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(sd.grid), dim3(sd.threads), sd.lds_bytes, stream, sd, K, species, counts, bad, tw,
                       S_F);
    return hipGetLastError();
}

using StreamLaunchFn = hipError_t (*)(const StreamDesc &, int64_t, const int8_t *, int32_t *, int32_t *,
                                      const double *, double *, hipStream_t);

template <int M>
StreamLaunchFn stream_pick_s(int S) {
    switch (S) {
        case 1: return launch_stream_ms<M, 1>;
        case 2: return launch_stream_ms<M, 2>;
        case 3: return Pairs<M>::NP * 3 <= 64 ? launch_stream_ms<M, 3> : nullptr;
    }
    return nullptr;
}

StreamLaunchFn stream_pick(int M, int S) {
    switch (M) {
        case 2: return stream_pick_s<2>(S);
        case 3: return stream_pick_s<3>(S);
        case 4: return stream_pick_s<4>(S);
        case 5: return stream_pick_s<5>(S);
        case 6: return S <= 2 ? stream_pick_s<6>(S) : nullptr;
    }
    return nullptr;
}

// LDS dwords of one streaming workgroup
int stream_lds_dw(const StreamDesc &sd, int M, int S) {
    const int P = M - 1, NP = P * (P + 1) / 2, NV = S * NP + P;
    const int raw = (sd.G + 1) * sd.raw_dw;
    const int pl = (sd.G + 2) * sd.slot_dw;
    const int cm = (sd.LW + 3) & ~3;
    const int red2 = NV * 64;
    const int red = (NV + 3 + 3) & ~3;
    const int epi = ((S * M * M + 1) & ~1) + 2 * (S * M * M + S * M);
    return raw + pl + cm + red2 + red + epi;
}

}  // namespace

bool fill_stream_desc(const Geometry &g, int lds_budget, int n_cus, int64_t K, int G, int threads, StreamDesc *sd) {
    std::memset(sd, 0, sizeof(*sd));
    if (K < 1 || g.halo != 1 || !stream_pick(g.M, g.S)) return false;
    int Lx4;
    if (g.lattice == PYHEA_FCC)
        Lx4 = g.L[0];
    else if (g.lattice == PYHEA_BCC && g.L[0] % 2 == 0)
        Lx4 = g.L[0] / 2;
    else
        return false;
    const int P = g.M - 1, PP = (P + 1) & ~1;
    if ((int64_t)Lx4 * g.L[1] >= 65536) return false;   // cell indices of a layer fit 16 bits
    sd->Lx = Lx4;
    sd->Ly = g.L[1];
    sd->Lz = g.L[2];
    sd->RS = Lx4 + 2;
    const int npos = (g.L[1] + 2) * sd->RS;
    sd->LW = (npos + 31) / 32;
    sd->PADW = (sd->RS + 2 + 31) / 32 + 1;
    sd->PW = sd->LW + 2 * sd->PADW;
    sd->cw0 = sd->RS / 32;
    sd->NCW = ((g.L[1] + 1) * sd->RS - 1) / 32 - sd->cw0 + 1;
    sd->ndma = (npos + 63) / 64;
    sd->raw_dw = 64 * sd->ndma;
    sd->slot_dw = 4 * sd->PW * PP;
    sd->N = (uint32_t)g.N;
    for (int k = 0; k < kMaxShells; ++k) sd->zk[k] = k < g.S ? g.z[k] : 0;
    // half offsets per basis, ordered by (layer step dz, shell)
    for (int b = 0; b < 4; ++b) {
        int n = 0;
        for (int dz = 0; dz < 2; ++dz)
            for (int k = 0; k < g.S; ++k) {
                sd->hs[b][dz][k] = n;
                for (int t = g.zstart[k]; t < g.zstart[k + 1]; ++t) {
                    const int dx = g.off[t][0], dy = g.off[t][1], dzh = g.off[t][2];
                    const bool keep = dzh > 0 || (dzh == 0 && (dy > 0 || (dy == 0 && dx > 0)));
                    if (!keep) continue;
                    int dc[3], bt;
                    four_site_target(g, 0, b, t, dc, &bt);
                    if (dc[0] < -1 || dc[0] > 1 || dc[1] < -1 || dc[1] > 1 || dc[2] < 0 || dc[2] > 1) return false;
                    if (dc[2] != dz) continue;
                    const int sh = dc[1] * sd->RS + dc[0];
                    const int q = sh >= 0 ? sh / 32 : -((-sh + 31) / 32);
                    const int r = sh - 32 * q;
                    if (n >= kMaxOffsets / 2) return false;
                    sd->tab[b][n++] = ((bt * sd->PW + q) * PP) * 32 + r;
                }
                sd->hs[b][dz][k + 1] = n;
            }
        // hs[b][0][S] == hs[b][1][0]: the dz = 0 list ends where the dz = 1 list starts
    }
    // launch shape: workgroup size, layers per group, workgroups per CU
    const int max_waves_cu = 32;
    double best = -1.0;
    StreamDesc pick = *sd;
    for (int th : {256, 512}) {
        if (threads && th != threads) continue;
        const int nw = th / 64;
        const int maxd = (sd->ndma + nw - 1) / nw;
        if (maxd > 16) continue;
        for (int gg = 1; gg <= std::min(8, g.L[2]); ++gg) {
            if (G && gg != G) continue;
            StreamDesc c = *sd;
            c.G = gg;
            c.threads = th;
            c.maxd = maxd <= 8 ? 8 : 16;
            const int dw = stream_lds_dw(c, g.M, g.S);
            if (dw * 4 > lds_budget) continue;
            const int wgs = std::min(lds_budget / (dw * 4), max_waves_cu / nw);
            if (wgs < 1) continue;
            const int nbw = gg * c.NCW;
            const double eff = (double)nbw / (double)((nbw + 63) & ~63);
            const double occ = std::min(1.0, (double)(wgs * nw) / 16.0);
            const double score = eff * occ * (1.0 - 0.03 / gg);
            if (score > best) {
                best = score;
                pick = c;
                pick.grid = (int)std::min<int64_t>(K, (int64_t)n_cus * wgs);
            }
        }
    }
    if (best < 0) return false;
    *sd = pick;
    sd->ngroups = (sd->Lz + sd->G - 1) / sd->G;
    // LDS layout (dwords)
    const int P2 = g.M - 1, NP = P2 * (P2 + 1) / 2, NV = g.S * NP + P2;
    sd->o_planes = (sd->G + 1) * sd->raw_dw;
    sd->o_cmask = sd->o_planes + (sd->G + 2) * sd->slot_dw;
    sd->o_red2 = sd->o_cmask + ((sd->LW + 3) & ~3);
    sd->o_red = sd->o_red2 + NV * 64;
    sd->o_epi = sd->o_red + ((NV + 3 + 3) & ~3);
    sd->lds_bytes = stream_lds_dw(*sd, g.M, g.S) * 4;
    return true;
}

hipError_t launch_count_stream(const Geometry &g, const StreamDesc &sd, int64_t K, const int8_t *species,
                               int32_t *counts, int32_t *bad, const double *tw, double *S_F, hipStream_t stream) {
    StreamLaunchFn f = stream_pick(g.M, g.S);
    if (!f || K <= 0) return hipErrorInvalidValue;
    return f(sd, K, species, counts, bad, tw, S_F, stream);
}

}  // namespace pyhea
