// Full SRO evaluation kernels (Sec. 4.3, Eq. 2; Sec. 4.4, Eq. 3), the
// per-swap evaluation API (Sec. 4.5, Eq. 4) and a device Philox stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "device_common.h"
#include "mc_kernels.h"

namespace pyhea {

void fill_eval_desc(const Geometry &g, EvalDesc *d) {
    std::memset(d, 0, sizeof(*d));
    d->A = g.A;
    d->lgA = g.lgA;
    d->Lx = g.L[0];
    d->Ly = g.L[1];
    d->Lz = g.L[2];
    d->M = g.M;
    d->S = g.S;
    d->z0 = g.z[0];
    for (int k = 0; k < kMaxShells; ++k) d->zk[k] = k < g.S ? g.z[k] : 0;
    d->inv_Lx = 1.0 / (double)g.L[0];
    d->inv_Ly = 1.0 / (double)g.L[1];
    d->N = (uint32_t)g.N;
    d->Z = g.Z;
    int nh = 0;
    for (int t = 0; t < g.Z; ++t) {
        int shell = 0;
        while (t >= g.zstart[shell + 1]) ++shell;
        const int dx = g.off[t][0], dy = g.off[t][1], dz = g.off[t][2];
        d->off[t][0] = (int8_t)dx;
        d->off[t][1] = (int8_t)dy;
        d->off[t][2] = (int8_t)dz;
        d->off[t][3] = (int8_t)shell;
        // keep one offset of each +-d pair
        const bool keep = dz > 0 || (dz == 0 && (dy > 0 || (dy == 0 && dx > 0)));
        if (!keep) continue;
        for (int b = 0; b < g.A; ++b) {
            int dc[3], bt;
            offset_target(g, b, t, dc, &bt);
            d->half[b][nh][0] = (int8_t)dc[0];
            d->half[b][nh][1] = (int8_t)dc[1];
            d->half[b][nh][2] = (int8_t)dc[2];
            d->half[b][nh][3] = (int8_t)bt;
            d->half[b][nh][4] = (int8_t)shell;
        }
        ++nh;
    }
    d->n_half = nh;
}

namespace {

__device__ __forceinline__ int wrap1(int v, int L) {
    while (v < 0) v += L;
    while (v >= L) v -= L;
    return v;
}

// Pair counts by gather: every site visits one offset of each +-d pair,
// N[k][i][j] = H[k][i][j] + H[k][j][i] with H the half counts (the map
// p -> p - d is a bijection of the periodic cell).  LDS-privatised int32
// histogram per workgroup, merged into global counts with one atomic per bin.
__global__ void __launch_bounds__(256) count_gather_kernel(EvalDesc ed, int64_t K,
                                                           const int8_t *__restrict__ species,
                                                           int32_t *__restrict__ counts,
                                                           int32_t *__restrict__ bad) {
    __shared__ int32_t hist[kMaxShells * kMaxSpecies * kMaxSpecies];
    __shared__ int32_t bad_sh;
    const int M = ed.M, E = ed.S * ed.M * ed.M;
    for (int64_t kc = blockIdx.y; kc < K; kc += gridDim.y) {
        for (int e = threadIdx.x; e < E; e += blockDim.x) hist[e] = 0;
        if (threadIdx.x == 0) bad_sh = 0;
        __syncthreads();
        const int8_t *sp = species + kc * (int64_t)ed.N;
        for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < ed.N; p += gridDim.x * blockDim.x) {
            const int s = sp[p];
            if (s < 0 || s >= M) {
                bad_sh = 1;
                continue;
            }
            const SiteCoord c = site_coord(p, ed.lgA, ed.Lx, ed.Ly, ed.inv_Lx, ed.inv_Ly);
            for (int hh = 0; hh < ed.n_half; ++hh) {
                const int8_t *o = ed.half[c.b][hh];
                const int x = wrap1(c.cx + o[0], ed.Lx);
                const int y = wrap1(c.cy + o[1], ed.Ly);
                const int z = wrap1(c.cz + o[2], ed.Lz);
                const int s2 = sp[((z * ed.Ly + y) * ed.Lx + x) * ed.A + o[3]];
                if (s2 < 0 || s2 >= M) continue;
                atomicAdd(&hist[(o[4] * M + s) * M + s2], 1);
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < E; e += blockDim.x) {
            const int kk = e / (M * M), i = (e / M) % M, j = e % M;
            const int v = hist[e] + hist[(kk * M + j) * M + i];
            if (v) atomicAdd(&counts[kc * E + e], v);
        }
        if (threadIdx.x == 0 && bad_sh) atomicOr(&bad[kc], 1);
        __syncthreads();
    }
}

// The same gather count for many configurations of different geometries: the
// grid is the concatenation of every configuration's site tiles.  The LDS
// histogram has kHistCopies interleaved copies (bin e, copy c at e * kHistCopies
// + c; lane l adds into copy l mod kHistCopies), so lanes of a wavefront that
// hit the same bin hit different words.
constexpr int kHistCopies = 16;
__global__ void __launch_bounds__(256) count_tasks_kernel(const CountTask *__restrict__ tasks,
                                                          const uint32_t *__restrict__ tile0, int n, uint32_t tile) {
    extern __shared__ int32_t hist[];   // [E][kHistCopies], then the invalid-id flag
    // owning configuration: the last c with tile0[c] <= blockIdx.x
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile0[mid] <= blockIdx.x)
            lo = mid;
        else
            hi = mid - 1;
    }
    const CountTask &t = tasks[lo];
    const EvalDesc &ed = t.ed;
    const int M = ed.M, E = ed.S * ed.M * ed.M;
    int32_t *bad_sh = hist + E * kHistCopies;
    for (int e = threadIdx.x; e <= E * kHistCopies; e += blockDim.x) hist[e] = 0;
    __syncthreads();
    const int8_t *sp = t.species;
    const int copy = threadIdx.x % kHistCopies;
    const uint32_t p0 = (blockIdx.x - tile0[lo]) * tile;
    const uint32_t p1 = min(p0 + tile, ed.N);
    for (uint32_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const int s = sp[p];
        if (s < 0 || s >= M) {
            *bad_sh = 1;
            continue;
        }
        const SiteCoord c = site_coord(p, ed.lgA, ed.Lx, ed.Ly, ed.inv_Lx, ed.inv_Ly);
        for (int hh = 0; hh < ed.n_half; ++hh) {
            const int8_t *o = ed.half[c.b][hh];
            const int x = wrap1(c.cx + o[0], ed.Lx);
            const int y = wrap1(c.cy + o[1], ed.Ly);
            const int z = wrap1(c.cz + o[2], ed.Lz);
            const int s2 = sp[((z * ed.Ly + y) * ed.Lx + x) * ed.A + o[3]];
            if (s2 < 0 || s2 >= M) continue;
            atomicAdd(&hist[((o[4] * M + s) * M + s2) * kHistCopies + copy], 1);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
        const int kk = e / (M * M), i = (e / M) % M, j = e % M;
        const int eT = (kk * M + j) * M + i;
        int v = 0;
        for (int q = 0; q < kHistCopies; ++q) v += hist[e * kHistCopies + q] + hist[eT * kHistCopies + q];
        if (v) atomicAdd(&t.counts[e], v);
    }
    if (threadIdx.x == 0 && *bad_sh) atomicOr(t.bad, 1);
}

__global__ void upload_kernel(SmallTable t, int n, double *__restrict__ dst) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = t.v[i];
}

__global__ void zero_i32_kernel(int32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// alpha / S / F of Eq. 2-3 per configuration (one thread per configuration),
// binary64, no contraction: R = N / (n_i n_j z_k), alpha = 1 - N_ij R,
// Q_k = sum_i (sum_j (alpha - t)^2), S = sum_k w_k Q_k, F = sqrt(S).  alpha
// [K][S][M][M] is written when non-null, S_F when target is non-null.
__global__ void objective_kernel(EvalDesc ed, int64_t K, const int32_t *__restrict__ counts,
                                 const int32_t *__restrict__ bad, const double *__restrict__ target,
                                 const double *__restrict__ weight, double *__restrict__ S_F,
                                 double *__restrict__ alpha) {
    const int64_t kc = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (kc >= K) return;
    const int M = ed.M, E = ed.S * M * M;
    const int32_t *c = counts + kc * E;
    int64_t n[kMaxSpecies];
    bool ok = bad[kc] == 0;
    for (int i = 0; i < M; ++i) {
        int64_t r = 0;
        for (int j = 0; j < M; ++j) r += c[i * M + j];
        n[i] = r / ed.z0;
        ok = ok && n[i] > 0;
    }
    if (!ok) {
        if (target) {
            S_F[2 * kc] = __longlong_as_double(0x7ff8000000000000ll);
            S_F[2 * kc + 1] = __longlong_as_double(0x7ff8000000000000ll);
        }
        return;
    }
    double sum = 0.0;
    for (int k = 0; k < ed.S; ++k) {
        double Q = 0.0;
        for (int i = 0; i < M; ++i) {
            double row = 0.0;
            for (int j = 0; j < M; ++j) {
                const int e = (k * M + i) * M + j;
                const double R = (double)ed.N / (double)(n[i] * n[j] * (int64_t)ed.zk[k]);
                const double a = 1.0 - (double)c[e] * R;
                if (alpha) alpha[kc * E + e] = a;
                if (target) {
                    const double dd = a - target[e];
                    row = row + dd * dd;
                }
            }
            Q = Q + row;
        }
        if (target) sum = sum + weight[k] * Q;
    }
    if (target) {
        S_F[2 * kc] = sum;
        S_F[2 * kc + 1] = sqrt(sum);
    }
}

// objective_kernel for a few configurations: one 64-thread block per
// configuration, its entries spread over the lanes and its rows summed by one
// lane each, then the rows into Q_k and S by lane 0 -- the same expressions and
// summation order as objective_kernel, so the results are the same bit for bit.
__global__ void __launch_bounds__(64) objective_block_kernel(EvalDesc ed, const int32_t *__restrict__ counts,
                                                             const int32_t *__restrict__ bad,
                                                             const double *__restrict__ target,
                                                             const double *__restrict__ weight,
                                                             double *__restrict__ S_F, double *__restrict__ alpha) {
    __shared__ int64_t n[kMaxSpecies];
    __shared__ double lsq[kMaxShells * kMaxSpecies * kMaxSpecies];
    __shared__ double lrow[kMaxShells * kMaxSpecies];
    const int64_t kc = blockIdx.x;
    const int tid = (int)threadIdx.x;
    const int M = ed.M, E = ed.S * M * M;
    const int32_t *c = counts + kc * E;
    if (tid < M) {
        int64_t r = 0;
        for (int j = 0; j < M; ++j) r += c[tid * M + j];
        n[tid] = r / ed.z0;
    }
    __syncthreads();
    bool ok = bad[kc] == 0;
    for (int i = 0; i < M; ++i) ok = ok && n[i] > 0;
    if (!ok) {
        if (target && tid == 0) {
            S_F[2 * kc] = __longlong_as_double(0x7ff8000000000000ll);
            S_F[2 * kc + 1] = __longlong_as_double(0x7ff8000000000000ll);
        }
        return;
    }
    for (int e = tid; e < E; e += blockDim.x) {
        const int k = e / (M * M), i = (e / M) % M, j = e % M;
        const double R = (double)ed.N / (double)(n[i] * n[j] * (int64_t)ed.zk[k]);
        const double a = 1.0 - (double)c[e] * R;
        if (alpha) alpha[kc * E + e] = a;
        if (target) {
            const double dd = a - target[e];
            lsq[e] = dd * dd;
        }
    }
    if (!target) return;
    __syncthreads();
    for (int r = tid; r < ed.S * M; r += blockDim.x) {
        double row = 0.0;
        for (int j = 0; j < M; ++j) row = row + lsq[r * M + j];
        lrow[r] = row;
    }
    __syncthreads();
    if (tid == 0) {
        double sum = 0.0;
        for (int k = 0; k < ed.S; ++k) {
            double Q = 0.0;
            for (int i = 0; i < M; ++i) Q = Q + lrow[k * M + i];
            sum = sum + weight[k] * Q;
        }
        S_F[2 * kc] = sum;
        S_F[2 * kc + 1] = sqrt(sum);
    }
}

// Eq. 2-3 on a chain's maintained counts, binary64 in the host contract's order
// (alpha = 1 - N R, (alpha - t)^2 summed along a row, rows into Q_k, S = sum_k
// w_k Q_k), written to its state with F = sqrt(S).  One thread per chain.
__global__ void final_objective_kernel(const ChainDesc *__restrict__ descs, int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const ChainDesc &d = descs[c];
    const int M = d.M;
    double sum = 0.0;
    for (int k = 0; k < d.S; ++k) {
        double Q = 0.0;
        for (int i = 0; i < M; ++i) {
            double row = 0.0;
            for (int j = 0; j < M; ++j) {
                const int e = (k * M + i) * M + j;
                const double a = 1.0 - (double)d.counts[e] * d.R[e];
                const double dd = a - d.target[e];
                row = row + dd * dd;
            }
            Q = Q + row;
        }
        sum = sum + d.w[k] * Q;
    }
    d.state->S = sum;
    d.state->F = sqrt(sum);
}

// site id of position (x, y, z) in half units, wrapped into the box
__device__ __forceinline__ int32_t site_at(const EvalDesc &ed, int x, int y, int z) {
    x = wrap1(x, 2 * ed.Lx);
    y = wrap1(y, 2 * ed.Ly);
    z = wrap1(z, 2 * ed.Lz);
    int b;
    const int px = x & 1, py = y & 1, pz = z & 1;
    if (ed.A == 4)
        b = (px && py) ? 1 : (px && pz) ? 2 : (py && pz) ? 3 : 0;
    else
        b = px;
    return (((z >> 1) * ed.Ly + (y >> 1)) * ed.Lx + (x >> 1)) * ed.A + b;
}

// dS and dN of given swaps against one configuration (no swap applied).
__global__ void trial_eval_kernel(EvalDesc ed, const int8_t *__restrict__ sp,
                                  const int32_t *__restrict__ counts, const double *__restrict__ target,
                                  const double *__restrict__ weight, int64_t n_pairs,
                                  const int32_t *__restrict__ pairs, double *__restrict__ dS_out,
                                  int32_t *__restrict__ dN_out) {
    const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (u >= n_pairs) return;
    const int M = ed.M, E = ed.S * M * M;
    const int32_t p = pairs[2 * u], q = pairs[2 * u + 1];
    if (p < 0 || q < 0 || (uint32_t)p >= ed.N || (uint32_t)q >= ed.N) {
        dS_out[u] = __longlong_as_double(0x7ff8000000000000ll);
        return;
    }
    const int a = sp[p], b = sp[q];
    int64_t n[kMaxSpecies];
    for (int i = 0; i < M; ++i) {
        int64_t r = 0;
        for (int j = 0; j < M; ++j) r += counts[i * M + j];
        n[i] = r / ed.z0;
    }
    int pp[3], pq[3];
    {
        const SiteCoord c = site_coord((uint32_t)p, ed.lgA, ed.Lx, ed.Ly, ed.inv_Lx, ed.inv_Ly);
        int bx, by, bz;
        basis_bits(ed.A, c.b, bx, by, bz);
        pp[0] = 2 * c.cx + bx;
        pp[1] = 2 * c.cy + by;
        pp[2] = 2 * c.cz + bz;
        const SiteCoord d = site_coord((uint32_t)q, ed.lgA, ed.Lx, ed.Ly, ed.inv_Lx, ed.inv_Ly);
        basis_bits(ed.A, d.b, bx, by, bz);
        pq[0] = 2 * d.cx + bx;
        pq[1] = 2 * d.cy + by;
        pq[2] = 2 * d.cz + bz;
    }
    double acc = 0.0;
    for (int k = 0; k < ed.S; ++k) {
        int D[kMaxSpecies];
        for (int j = 0; j < M; ++j) D[j] = 0;
        if (a != b) {
            for (int t = 0; t < ed.Z; ++t) {
                if (ed.off[t][3] != k) continue;
                const int32_t rp = site_at(ed, pp[0] + ed.off[t][0], pp[1] + ed.off[t][1], pp[2] + ed.off[t][2]);
                const int32_t rq = site_at(ed, pq[0] + ed.off[t][0], pq[1] + ed.off[t][1], pq[2] + ed.off[t][2]);
                if (rp != q) D[sp[rp]] -= 1;
                if (rq != p) D[sp[rq]] += 1;
            }
        }
        double dQ = 0.0;
        for (int i = 0; i < M; ++i) {
            double rowsum = 0.0;
            for (int j = 0; j < M; ++j) {
                int dn = 0;
                if (a != b) {
                    if (i == a) dn = j == a ? 2 * D[a] : (j == b ? D[b] - D[a] : D[j]);
                    else if (i == b) dn = j == b ? -2 * D[b] : (j == a ? D[b] - D[a] : -D[j]);
                    else if (j == a) dn = D[i];
                    else if (j == b) dn = -D[i];
                }
                const int e = (k * M + i) * M + j;
                if (dN_out) dN_out[u * E + e] = dn;
                const double R = (double)ed.N / (double)(n[i] * n[j] * (int64_t)ed.zk[k]);
                const double a0 = 1.0 - (double)counts[e] * R;
                const double d0 = a0 - target[e];
                const double a1 = 1.0 - (double)(counts[e] + dn) * R;
                const double d1 = a1 - target[e];
                rowsum = rowsum + (d1 * d1 - d0 * d0);
            }
            dQ = dQ + rowsum;
        }
        acc = acc + weight[k] * dQ;
    }
    dS_out[u] = acc;
}

__global__ void philox_kernel(const uint32_t *__restrict__ ctr, uint64_t seed, int64_t n,
                              uint32_t *__restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    for (int w = 0; w < 4; ++w) out[4 * i + w] = c[w];
}

}  // namespace

hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_i32_kernel, dim3(blocks), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_count_gather(const EvalDesc &ed, int64_t K, const int8_t *species, int32_t *counts,
                               int32_t *bad, hipStream_t stream) {
    const int E = ed.S * ed.M * ed.M;
    hipError_t e = launch_zero_i32(counts, K * E, stream);
    if (e != hipSuccess) return e;
    e = launch_zero_i32(bad, K, stream);
    if (e != hipSuccess) return e;
    const int per_cfg = (int)std::min<int64_t>(std::max<int64_t>(1, (ed.N + 2047) / 2048), 1024);
    const int gy = (int)std::min<int64_t>(K, 65535);
    hipLaunchKernelGGL(count_gather_kernel, dim3(per_cfg, gy), dim3(256), 0, stream, ed, K, species,
                       counts, bad);
    return hipGetLastError();
}

hipError_t launch_upload(const SmallTable &t, int n, double *dst, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    if (n > kMaxTable) return hipErrorInvalidValue;
    hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(256), 0, stream, t, n, dst);
    return hipGetLastError();
}

hipError_t launch_count_tasks(const CountTask *tasks, const uint32_t *tile0, int n, uint32_t n_tiles, uint32_t tile,
                              int max_E, hipStream_t stream) {
    if (n <= 0 || n_tiles == 0) return hipSuccess;
    if (tile == 0 || max_E <= 0 || max_E > kMaxShells * kMaxSpecies * kMaxSpecies) return hipErrorInvalidValue;
    const size_t lds = ((size_t)max_E * kHistCopies + 1) * sizeof(int32_t);
    hipLaunchKernelGGL(count_tasks_kernel, dim3(n_tiles), dim3(256), lds, stream, tasks, tile0, n, tile);
    return hipGetLastError();
}

hipError_t launch_objective_epilogue(const EvalDesc &ed, int64_t K, const int32_t *counts,
                                     const int32_t *bad, const double *target, const double *weight,
                                     double *S_F, double *alpha, hipStream_t stream) {
    if (K <= 0) return hipSuccess;
    if (K <= 1024) {   // few configurations: a block each rather than a lane each
        hipLaunchKernelGGL(objective_block_kernel, dim3((unsigned)K), dim3(64), 0, stream, ed, counts, bad, target,
                           weight, S_F, alpha);
        return hipGetLastError();
    }
    const int blocks = (int)((K + 255) / 256);
    hipLaunchKernelGGL(objective_kernel, dim3(blocks), dim3(256), 0, stream, ed, K, counts, bad, target,
                       weight, S_F, alpha);
    return hipGetLastError();
}

hipError_t launch_final_objective(const ChainDesc *descs_dev, int n_chains, hipStream_t stream) {
    if (n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(final_objective_kernel, dim3((n_chains + 63) / 64), dim3(64), 0, stream, descs_dev, n_chains);
    return hipGetLastError();
}

hipError_t launch_trial_eval(const EvalDesc &ed, const int8_t *species, const int32_t *counts,
                             const double *target, const double *weight, int64_t n_pairs,
                             const int32_t *pairs, double *dS, int32_t *dN, hipStream_t stream) {
    if (n_pairs <= 0) return hipSuccess;
    const int blocks = (int)((n_pairs + 127) / 128);
    hipLaunchKernelGGL(trial_eval_kernel, dim3(blocks), dim3(128), 0, stream, ed, species, counts, target,
                       weight, n_pairs, pairs, dS, dN);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, uint64_t seed, int64_t n, uint32_t *out, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int blocks = (int)((n + 255) / 256);
    hipLaunchKernelGGL(philox_kernel, dim3(blocks), dim3(256), 0, stream, ctr, seed, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Random solutions of the global search (Sec. 4.1): the composition-sorted
// species list placed through a keyed permutation of the sites.  The
// permutation is a four-round balanced Feistel network on 2h-bit values whose
// round function is word 0 of Philox4x32-10(counter = (right half, round,
// slot, 0x80000000 | iteration), key = seed), re-applied (cycle walking) until
// the value is below N.  One thread per list position.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t feistel4(uint32_t x, int h, uint32_t slot, uint32_t iteration, uint32_t k0,
                                             uint32_t k1) {
    const uint32_t mask = (1u << h) - 1u;
    uint32_t l = x >> h, r = x & mask;
#pragma unroll
    for (uint32_t round = 0; round < 4; ++round) {
        uint32_t c[4] = {r, round, slot, 0x80000000u | iteration};
        philox4x32_10(c, k0, k1);
        const uint32_t nl = r;
        r = l ^ (c[0] & mask);
        l = nl;
    }
    return (l << h) | r;
}

__global__ void random_configs_kernel(uint32_t N, int h, RandomConfigDesc d, int8_t *__restrict__ out) {
    const uint32_t cfg = blockIdx.y;
    const uint32_t slot = d.slot0 + cfg;
    const uint32_t k0 = (uint32_t)d.seed, k1 = (uint32_t)(d.seed >> 32);
    int8_t *o = out + (int64_t)cfg * N;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        int j = 0;
        while (j + 1 < d.M && i >= d.prefix[j + 1]) ++j;
        uint32_t x = feistel4(i, h, slot, d.iteration, k0, k1);
        while (x >= N) x = feistel4(x, h, slot, d.iteration, k0, k1);
        o[x] = (int8_t)j;
    }
}

hipError_t launch_random_configs(uint32_t N, const RandomConfigDesc &d, int n_configs, int8_t *out,
                                 hipStream_t stream) {
    if (n_configs <= 0 || N == 0) return hipSuccess;
    int h = 1;
    while ((uint64_t(1) << (2 * h)) < N) ++h;
    const int threads = 256;
    const int bx = (int)std::min<uint32_t>((N + threads - 1) / threads, 1024);
    for (int c0 = 0; c0 < n_configs; c0 += 65535) {
        RandomConfigDesc dc = d;
        dc.slot0 = d.slot0 + (uint32_t)c0;
        const int nc = std::min(65535, n_configs - c0);
        hipLaunchKernelGGL(random_configs_kernel, dim3(bx, nc), dim3(threads), 0, stream, N, h, dc,
                           out + (int64_t)c0 * N);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Non-incremental baseline: copies of one configuration with one swap each.
// ---------------------------------------------------------------------------

__global__ void replicate_kernel(const int8_t *__restrict__ base, int64_t N, int n, int8_t *__restrict__ out) {
    const int64_t row = blockIdx.y;
    int8_t *o = out + row * N;
    if ((N & 3) == 0) {
        const uint32_t *b4 = reinterpret_cast<const uint32_t *>(base);
        uint32_t *o4 = reinterpret_cast<uint32_t *>(o);
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N / 4; i += (int64_t)gridDim.x * blockDim.x)
            o4[i] = b4[i];
    } else {
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
            o[i] = base[i];
    }
}

// pair i swaps sites p, q of copy i; a pair outside [0, N) sets *bad and is skipped
__global__ void apply_swaps_kernel(const int8_t *__restrict__ base, int64_t N, const int32_t *__restrict__ pairs,
                                   int n, int8_t *__restrict__ out, int32_t *__restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t p = pairs[2 * i], q = pairs[2 * i + 1];
    if (p < 0 || q < 0 || p >= N || q >= N) {
        atomicOr(bad, 1);
        return;
    }
    out[(int64_t)i * N + p] = base[q];
    out[(int64_t)i * N + q] = base[p];
}

__global__ void sub_objective_kernel(const double *__restrict__ S_F, const double *__restrict__ S0, int n,
                                     double *__restrict__ dS) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dS[i] = S_F[2 * i] - S0[0];
}

hipError_t launch_swap_copies(const int8_t *base, int64_t N, const int32_t *pairs, int n, int8_t *out, int32_t *bad,
                              hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t words = (N & 3) == 0 ? N / 4 : N;
    const int bx = (int)std::min<int64_t>((words + 255) / 256, 256);
    for (int r0 = 0; r0 < n; r0 += 65535) {
        const int nr = std::min(65535, n - r0);
        hipLaunchKernelGGL(replicate_kernel, dim3(bx, nr), dim3(256), 0, stream, base, N, nr, out + (int64_t)r0 * N);
    }
    hipLaunchKernelGGL(apply_swaps_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, base, N, pairs, n, out, bad);
    return hipGetLastError();
}

hipError_t launch_sub_objective(const double *S_F, const double *S0, int n, double *dS, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(sub_objective_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, S_F, S0, n, dS);
    return hipGetLastError();
}

}  // namespace pyhea
