// Persistent Monte Carlo kernel: SRO-targeted swap search (Sec. 4.2,
// Algorithm 3; Sec. 4.5-4.6).
//
// One workgroup runs one chain for up to `max_steps` steps.  The workgroup has
// G * S wavefronts (G = ceil(B / 64) slot groups, S shells); wave w = g * S + k
// evaluates shell k of slots g*64 .. g*64+63, so every wave has a uniform shell
// and its loops over offsets and (i, j) entries are uniform.
//
// Per step:
//  1. every (slot, shell) lane draws the slot's swap (Philox4x32-10, counter
//     (slot, step, chain, 0)), gathers the species of the z_k shell-k
//     neighbours of both sites from the halo-padded configuration (one linear
//     delta per (basis, offset), no modulo), removes the partner site, and
//     forms D = c_q - c_p and dQ_k = sum_i sum_j sq(N + dN) - sq(N) (Eq. 4-5);
//  2. wave 0 sums dS = sum_k w_k dQ_k per slot, compacts the improving slots
//     (dS < -tau) and ranks them by (dS, slot) (Eq. 6);
//  3. all waves walk the ranking in lock step: BEST stops after one commit;
//     DISJOINT skips swaps within shells 1..S of a site already committed in
//     the step and re-checks dS against the updated counts before committing.
// Counts are exact int32; every binary64 value is produced by the same
// expression sequence as the host contract, with contraction disabled.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "mc_kernels.h"

namespace pyhea {

namespace {

template <bool kWide>
struct HistT {
    using type = uint32_t;
};
template <>
struct HistT<true> {
    using type = uint64_t;
};

// 5-bit fields: z_k <= 24 neighbours of one species per shell
template <typename H>
__device__ __forceinline__ int fld(H h, int j) {
    return (int)((h >> (5 * j)) & 31u);
}
template <typename H>
__device__ __forceinline__ H one_at(int j) {
    return (H)1 << (5 * j);
}

__device__ __forceinline__ double sq_dev(int32_t n, double R, double t) {
    const double alpha = 1.0 - (double)n * R;
    const double d = alpha - t;
    return d * d;
}

// One (k, i, j) entry: the ratio R = N/(n_i n_j z_k), the target, the cached
// squared deviation and the exact pair count, read together (two 16-byte loads).
struct Ent {
    double R;
    double t;
    double sq;
    int32_t cnt;
    int32_t pad;
};

struct Lds {
    Ent *ent;       // [S][M][M]
    int4 *dlin4;    // [kMaxOffsets]: linear deltas of offset t from bases 0..3
    int32_t *offmod;
    double *rec_dS;     // [B]
    uint32_t *rec_pp;   // [B] packed position of p (10 bits per axis)
    uint32_t *rec_pq;   // [B]
    uint32_t *rec_ab;   // [B] a | b << 8 | null << 16
    void *rec_cp;       // [S][K B] neighbour histograms of p (Hist)
    void *rec_cq;       // [S][K B] neighbour histograms of q (Hist)
    double *rec_dQ;     // [S][B]
    int32_t *order;     // [B]
    int32_t *list;      // [B]
    double *sh_dQ;      // [2][kMaxShells]
    int32_t *sh_int;    // scalars
    void *part;         // [S][W][2 (cp, cq)][K B] partial histograms (bal)
    uint64_t *spec_cm;  // [64] earlier candidates each improving candidate conflicts with
    double *spec_T;     // [CH][E] change of every entry's term under each member of a chunk
    int32_t *spec_P;    // [CH][E] change of every entry's count after each member
    double *spec_Q;     // [16][kMaxShells] dQ_k of each member of a chunk
    int32_t *spec_mem;  // [16] slots of a chunk's members
    int32_t *spec_ctl;  // [4] members in the current chunk
    uint8_t *store;     // species store
};

__device__ __forceinline__ uint8_t *carve(uint8_t *&p, size_t bytes) {
    uint8_t *r = p;
    p += (bytes + 15) & ~size_t(15);
    return r;
}

template <int kStore>
__device__ __forceinline__ int load_species(const Lds &L, const ChainDesc &d, int32_t pid) {
    if constexpr (kStore == kStoreLds8) {
        return L.store[pid];
    } else if constexpr (kStore == kStoreLds4) {
        const uint32_t w = reinterpret_cast<const uint32_t *>(L.store)[pid >> 3];
        return (int)((w >> ((pid & 7) << 2)) & 0xFu);
    } else {
        return d.pad_global[pid];
    }
}

template <int kStore>
__device__ __forceinline__ void store_species(const Lds &L, const ChainDesc &d, int32_t pid, int v) {
    if constexpr (kStore == kStoreLds8) {
        L.store[pid] = (uint8_t)v;
    } else if constexpr (kStore == kStoreLds4) {
        uint32_t *w = reinterpret_cast<uint32_t *>(L.store) + (pid >> 3);
        const int sh = (pid & 7) << 2;
        atomicAnd(w, ~(0xFu << sh));
        atomicOr(w, (uint32_t)v << sh);
    } else {
        d.pad_global[pid] = (int8_t)v;
    }
}

__device__ __forceinline__ int32_t padded_id(const ChainDesc &d, int px, int py, int pz, int b) {
    return ((pz * d.PY + py) * d.PX + px) * d.A + b;
}

__device__ __forceinline__ int wrap_axis(int v, int L) {
    while (v < 0) v += L;
    while (v >= L) v -= L;
    return v;
}

__device__ __forceinline__ uint32_t pack_pos(int x, int y, int z) {
    return (uint32_t)x | ((uint32_t)y << 10) | ((uint32_t)z << 20);
}

// cell and basis of a packed position, and the site id p = ((cz Ly + cy) Lx + cx) A + b
__device__ __forceinline__ SiteCoord pos_site(const ChainDesc &d, uint32_t pos) {
    const int x = (int)(pos & 1023u), y = (int)((pos >> 10) & 1023u), z = (int)((pos >> 20) & 1023u);
    const int bx = x & 1, by = y & 1, bz = z & 1;
    SiteCoord c;
    c.cx = x >> 1;
    c.cy = y >> 1;
    c.cz = z >> 1;
    // FCC basis (0,0,0), (1,1,0), (1,0,1), (0,1,1); BCC (0,0,0), (1,1,1)
    c.b = d.A == 2 ? bx : ((bx & by) ? 1 : ((bx & bz) ? 2 : ((by & bz) ? 3 : 0)));
    return c;
}

__device__ __forceinline__ uint32_t site_id(const ChainDesc &d, SiteCoord c) {
    return (uint32_t)(((c.cz * d.Ly + c.cy) * d.Lx + c.cx) * d.A + c.b);
}

// squared minimum-image distance (half units) between two packed positions
__device__ __forceinline__ int min_image_r2(const ChainDesc &d, uint32_t u, uint32_t v) {
    const int Ls[3] = {d.Lx, d.Ly, d.Lz};
    int r2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int x = (int)((u >> (10 * a)) & 1023u) - (int)((v >> (10 * a)) & 1023u);
        const int box = 2 * Ls[a];
        if (x > Ls[a]) x -= box;
        if (x < -Ls[a]) x += box;
        r2 += x * x;
    }
    return r2;
}

// the packed (pos_q - pos_p) mod box, for the exact multiplicity count on small cells
__device__ __forceinline__ int32_t mod_delta(const ChainDesc &d, uint32_t pp, uint32_t pq) {
    const int Ls[3] = {d.Lx, d.Ly, d.Lz};
    int32_t out = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int x = (int)((pq >> (10 * a)) & 1023u) - (int)((pp >> (10 * a)) & 1023u);
        if (x < 0) x += 2 * Ls[a];
        out |= x << (10 * a);
    }
    return out;
}

// does a site at packed position u lie on, or in shells 1..S of, position v?
__device__ __forceinline__ bool near_or_equal(const ChainDesc &d, uint32_t u, uint32_t v) {
    const int r2 = min_image_r2(d, u, v);
    if (r2 == 0) return true;
    bool hit = false;
#pragma unroll
    for (int k = 0; k < kMaxShells; ++k) hit |= (k < d.S && r2 == d.r2[k]);
    return hit;
}

// species v at site (cx, cy, cz, b) and at every halo copy of it: padded
// coordinates x0 + i*L < P per axis
template <int kStore>
__device__ void write_site(const Lds &L, const ChainDesc &d, int cx, int cy, int cz, int b, int v) {
    const int h = d.halo;
    const int x0 = wrap_axis(cx + h, d.Lx), y0 = wrap_axis(cy + h, d.Ly), z0 = wrap_axis(cz + h, d.Lz);
    for (int pz = z0; pz < d.PZ; pz += d.Lz)
        for (int py = y0; py < d.PY; py += d.Ly)
            for (int px = x0; px < d.PX; px += d.Lx) store_species<kStore>(L, d, padded_id(d, px, py, pz, b), v);
}

// change of entry (i, j) of shell k's counts when candidate s (record index) commits
template <int M, typename Hist>
__device__ __forceinline__ int entry_dn(const Lds &L, int Bt, int r, int k, int i, int j) {
    const uint32_t ab = L.rec_ab[r];
    const int a = (int)(ab & 0xFFu), b = (int)((ab >> 8) & 0xFFu);
    const Hist cp = ((const Hist *)L.rec_cp)[k * Bt + r], cq = ((const Hist *)L.rec_cq)[k * Bt + r];
    const int ui = (i == a ? 1 : 0) - (i == b ? 1 : 0), uj = (j == a ? 1 : 0) - (j == b ? 1 : 0);
    return __mul24(ui, fld(cq, j) - fld(cp, j)) + __mul24(uj, fld(cq, i) - fld(cp, i));
}

// inclusive prefix sum along each 16-lane row (lanes outside the row read 0)
__device__ __forceinline__ int row_prefix_sum(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, true);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, true);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, true);  // row_shr:8
    return x;
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

template <int kStore, int M>
__global__ void __launch_bounds__(1024) mc_kernel(const ChainDesc *__restrict__ descs,
                                                  int32_t max_steps, int32_t W, int32_t bal, int32_t K, int32_t CH) {
    using Hist = typename HistT<(M > 6)>::type;
    const ChainDesc &d = descs[blockIdx.x];
    ChainState *st = d.state;
    if (st->done) return;

    const int S = d.S, E = S * M * M;
    const int B = d.B;
    const int Gs = (B + kWave - 1) / kWave;  // slot groups per step
    const int Bt = K * B;                    // records: K consecutive steps of B slots
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    // a slot group has W >= S wavefronts; wavefront k < S owns shell k.  With
    // bal, wavefront w gathers offsets [Z w / W, Z (w + 1) / W) of all Z offsets
    // (ordered by shell); without, W == S and wavefront k gathers shell k.
    const int grp = wave / W;         // slot group
    const int widx = wave - grp * W;  // wavefront within the group
    const int k = widx < S ? widx : -1;  // shell owned (-1: gathers only)
    const int kw = grp / Gs;          // step offset of this wave's slots
    const int slot = (grp - kw * Gs) * kWave + lane;  // candidate within its step
    const int rix = kw * B + slot;    // its record (when slot < B)
    const int nthreads = blockDim.x;

    extern __shared__ __align__(16) uint8_t smem[];
    Lds L;
    {
        uint8_t *p = smem;
        L.ent = (Ent *)carve(p, E * sizeof(Ent));
        L.dlin4 = (int4 *)carve(p, kMaxOffsets * 16);
        L.offmod = (int32_t *)carve(p, kMaxOffsets * 4);
        L.rec_dS = (double *)carve(p, Bt * 8);
        L.rec_pp = (uint32_t *)carve(p, Bt * 4);
        L.rec_pq = (uint32_t *)carve(p, Bt * 4);
        L.rec_ab = (uint32_t *)carve(p, Bt * 4);
        L.rec_cp = carve(p, S * Bt * (int)sizeof(Hist));
        L.rec_cq = carve(p, S * Bt * (int)sizeof(Hist));
        L.rec_dQ = (double *)carve(p, S * Bt * 8);
        L.order = (int32_t *)carve(p, Bt * 4);
        L.list = (int32_t *)carve(p, Bt * 4);
        L.sh_dQ = (double *)carve(p, 2 * kMaxShells * 8);
        L.sh_int = (int32_t *)carve(p, 32 * 4);
        if (bal) L.part = carve(p, S * W * 2 * Bt * (int)sizeof(Hist));
        if (CH > 0) {
            L.spec_cm = (uint64_t *)carve(p, kWave * 8);
            L.spec_T = (double *)carve(p, CH * E * 8);
            L.spec_P = (int32_t *)carve(p, CH * E * 4);
            L.spec_Q = (double *)carve(p, 16 * kMaxShells * 8);
            L.spec_mem = (int32_t *)carve(p, 16 * 4);
            L.spec_ctl = (int32_t *)carve(p, 4 * 4);
        }
        L.store = p;
    }

    // ---- load chain state into LDS ------------------------------------------------
    for (int e = threadIdx.x; e < E; e += nthreads) {
        Ent en;
        en.cnt = d.counts[e];
        en.R = d.R[e];
        en.t = d.target[e];
        en.sq = sq_dev(en.cnt, en.R, en.t);
        en.pad = 0;
        L.ent[e] = en;
    }
    for (int t = threadIdx.x; t < kMaxOffsets; t += nthreads)
        L.dlin4[t] = make_int4(d.dlin[0][t], d.dlin[1][t], d.dlin[2][t], d.dlin[3][t]);
    for (int t = threadIdx.x; t < kMaxOffsets; t += nthreads) L.offmod[t] = d.off_mod[t];
    if constexpr (kStore != kStoreGlobal) {
        // fill the halo-padded configuration from the unpadded one
        const double inv_PX = 1.0 / (double)d.PX, inv_PY = 1.0 / (double)d.PY;
        const int h = d.halo;
        if constexpr (kStore == kStoreLds8) {
            for (uint32_t pid = threadIdx.x; pid < d.Npad; pid += nthreads) {
                const SiteCoord c = site_coord(pid, d.lgA, d.PX, d.PY, inv_PX, inv_PY);
                const int cx = wrap_axis(c.cx - h, d.Lx), cy = wrap_axis(c.cy - h, d.Ly),
                          cz = wrap_axis(c.cz - h, d.Lz);
                L.store[pid] = (uint8_t)d.species[((cz * d.Ly + cy) * d.Lx + cx) * d.A + c.b];
            }
        } else {
            const uint32_t nw = (d.Npad + 7) / 8;
            for (uint32_t wI = threadIdx.x; wI < nw; wI += nthreads) {
                uint32_t word = 0;
                for (int s = 0; s < 8; ++s) {
                    const uint32_t pid = wI * 8 + s;
                    if (pid >= d.Npad) break;
                    const SiteCoord c = site_coord(pid, d.lgA, d.PX, d.PY, inv_PX, inv_PY);
                    const int cx = wrap_axis(c.cx - h, d.Lx), cy = wrap_axis(c.cy - h, d.Ly),
                              cz = wrap_axis(c.cz - h, d.Lz);
                    word |= ((uint32_t)d.species[((cz * d.Ly + cy) * d.Lx + cx) * d.A + c.b] & 0xFu)
                            << (4 * s);
                }
                reinterpret_cast<uint32_t *>(L.store)[wI] = word;
            }
        }
    }
    __syncthreads();

    // chain counters: identical copies in every thread
    int64_t trials = st->trials, commits = st->commits, step = st->steps;
    int64_t nulls = st->null_trials;
    int depth = st->depth;
    int stop_reason = 0;
    bool done = false;
    const uint32_t key0 = (uint32_t)d.seed, key1 = (uint32_t)(d.seed >> 32);
    const int h = d.halo;
    // this wave's offsets and rows of shell k
    const int Z = d.zstart[S];
    const int zsk = k >= 0 ? d.zstart[k] : 0, zek = k >= 0 ? d.zstart[k + 1] : 0;
    const int g0 = bal ? (Z * widx) / W : zsk;
    const int g1 = bal ? (Z * (widx + 1)) / W : zek;
    if (trials >= d.n_trials) done = true;
    double wk[kMaxShells];
#pragma unroll
    for (int kk = 0; kk < kMaxShells; ++kk) wk[kk] = d.w[kk];
    const double tau = d.tau;

    // A pass evaluates the candidates of up to K consecutive steps against the
    // current state.  Steps are then taken in order; a step whose candidates
    // include no improving swap commits nothing and leaves the state as it was,
    // so the next step's evaluation is still exact.  The first step that commits
    // ends the pass.  After a pass whose first step committed, the next pass
    // evaluates one step.
    int kpref = K;
    int64_t steps_run = 0;
    while (!done && steps_run < max_steps) {
        const int ke = (int)min((int64_t)kpref, (int64_t)max_steps - steps_run);

        // ---- phase 1: draw and evaluate (step offset kw, slot) --------------------------
        // Each wavefront gathers the neighbours along its offsets [g0, g1) into one
        // histogram pair per shell; shell k's owner (wavefront k of the group) adds
        // the pairs of every wavefront whose offsets meet shell k (exact integer
        // sums) and evaluates dQ_k.
        {
            const int64_t left = d.n_trials - trials - (int64_t)kw * B;
            const int tasks_w = left <= 0 ? 0 : (left < B ? (int)left : B);
            const bool active = kw < ke && slot < tasks_w;
            uint32_t ppos = 0, qpos = 0;
            int a = 0, b = 0;
            bool live = false;
            Hist cp = 0, cq = 0;   // the owner's full shell-k histograms
            double dQ = 0.0;
            // the draws, the two sites and their species: once per candidate, by the
            // group's first wavefront, shared with the others through the records
            if (widx == 0 && slot < B && kw < ke) {
                uint32_t ab = 0;
                if (active) {
                    uint32_t c[4] = {(uint32_t)slot, (uint32_t)(step + kw), d.chain_id, 0u};
                    philox4x32_10(c, key0, key1);
                    const uint32_t p = __umulhi(c[0], d.N), q = __umulhi(c[1], d.N);
                    const SiteCoord sp = site_coord(p, d.lgA, d.Lx, d.Ly, d.inv_Lx, d.inv_Ly);
                    const SiteCoord sq = site_coord(q, d.lgA, d.Lx, d.Ly, d.inv_Lx, d.inv_Ly);
                    int bx, by, bz;
                    basis_bits(d.A, sp.b, bx, by, bz);
                    ppos = pack_pos(2 * sp.cx + bx, 2 * sp.cy + by, 2 * sp.cz + bz);
                    basis_bits(d.A, sq.b, bx, by, bz);
                    qpos = pack_pos(2 * sq.cx + bx, 2 * sq.cy + by, 2 * sq.cz + bz);
                    a = load_species<kStore>(L, d, padded_id(d, sp.cx + h, sp.cy + h, sp.cz + h, sp.b));
                    b = load_species<kStore>(L, d, padded_id(d, sq.cx + h, sq.cy + h, sq.cz + h, sq.b));
                    ab = (uint32_t)a | ((uint32_t)b << 8) | ((uint32_t)(a == b) << 16) | (1u << 17);
                }
                L.rec_pp[rix] = ppos;
                L.rec_pq[rix] = qpos;
                L.rec_ab[rix] = ab;
            }
            if (W > 1) __syncthreads();
            if (active) {
                if (widx != 0) {
                    ppos = L.rec_pp[rix];
                    qpos = L.rec_pq[rix];
                    const uint32_t ab = L.rec_ab[rix];
                    a = (int)(ab & 0xFFu);
                    b = (int)((ab >> 8) & 0xFFu);
                }
                live = (a != b);
                const SiteCoord sp = pos_site(d, ppos), sq = pos_site(d, qpos);
                const int32_t pidp = padded_id(d, sp.cx + h, sp.cy + h, sp.cz + h, sp.b);
                const int32_t pidq = padded_id(d, sq.cx + h, sq.cy + h, sq.cz + h, sq.b);
                if (live) {
                    // padded linear deltas of every offset from the two sites' bases
                    const int32_t *dlp = reinterpret_cast<const int32_t *>(L.dlin4) + sp.b;
                    const int32_t *dlq = reinterpret_cast<const int32_t *>(L.dlin4) + sq.b;
#pragma unroll 1
                    for (int s2 = 0; s2 < S; ++s2) {
                        const int t0 = max(g0, (int)d.zstart[s2]), t1 = min(g1, (int)d.zstart[s2 + 1]);
                        if (t0 >= t1) continue;
                        Hist hp = 0, hq = 0;
                        // 4 offsets at a time: all loads issued before use
                        constexpr int kU = 4;
                        int t = t0;
#pragma unroll 1
                        for (; t + kU <= t1; t += kU) {
                            int ap[kU], aq[kU];
#pragma unroll
                            for (int u = 0; u < kU; ++u) {
                                ap[u] = pidp + dlp[(t + u) * 4];
                                aq[u] = pidq + dlq[(t + u) * 4];
                            }
                            int vp[kU], vq[kU];
#pragma unroll
                            for (int u = 0; u < kU; ++u) {
                                vp[u] = load_species<kStore>(L, d, ap[u]);
                                vq[u] = load_species<kStore>(L, d, aq[u]);
                            }
#pragma unroll
                            for (int u = 0; u < kU; ++u) {
                                hp += one_at<Hist>(vp[u]);
                                hq += one_at<Hist>(vq[u]);
                            }
                        }
#pragma unroll 1
                        for (; t < t1; ++t) {
                            hp += one_at<Hist>(load_species<kStore>(L, d, pidp + dlp[t * 4]));
                            hq += one_at<Hist>(load_species<kStore>(L, d, pidq + dlq[t * 4]));
                        }
                        if (bal) {
                            // this wavefront's part of shell s2 (read by its owner when live)
                            Hist *pt = (Hist *)L.part + ((s2 * W + widx) * 2) * Bt;
                            pt[rix] = hp;
                            pt[Bt + rix] = hq;
                        } else {
                            cp = hp;   // the wavefront's own shell
                            cq = hq;
                        }
                    }
                }
            }
            if (bal) {
                __syncthreads();
                if (k >= 0 && live) {
                    for (int w2 = 0; w2 < W; ++w2) {
                        const int a0 = (Z * w2) / W, a1 = (Z * (w2 + 1)) / W;
                        if (max(a0, zsk) >= min(a1, zek)) continue;
                        const Hist *pt = (const Hist *)L.part + ((k * W + w2) * 2) * Bt;
                        cp += pt[rix];
                        cq += pt[Bt + rix];
                    }
                }
            }
            if (k >= 0 && live) {
                // remove the partner: q is reached from p along m shell-k offsets
                int m;
                if (!d.small_cell) {
                    m = min_image_r2(d, ppos, qpos) == d.r2[k] ? 1 : 0;
                } else {
                    const int32_t md = mod_delta(d, ppos, qpos);
                    m = 0;
                    for (int t = zsk; t < zek; ++t) m += (L.offmod[t] == md) ? 1 : 0;
                }
                cp -= (Hist)m << (5 * b);
                cq -= (Hist)m << (5 * a);
                // D = c_q - c_p and u = +1 at species a, -1 at b: dN[i][j] = u_i D_j + u_j D_i
                int D[M], u[M];
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    D[j] = fld(cq, j) - fld(cp, j);
                    u[j] = (j == a ? 1 : 0) - (j == b ? 1 : 0);
                }
                // dQ_k = sum over rows i of (sum over j of sq(N + dN) - sq(N))
                if (d.sym) {
                    // Symmetric N, dN, R and target: only rows lo = min(a, b) and
                    // hi = max(a, b) need evaluating; row i of the others holds
                    // nonzero terms only at columns lo < hi, equal to entries
                    // (lo, i) and (hi, i).  Terms with dN = 0 are exactly +0.0.
                    const int lo = a < b ? a : b, hi = a < b ? b : a;
                    const int ulo = lo == a ? 1 : -1;
                    const int Dlo = fld(cq, lo) - fld(cp, lo), Dhi = fld(cq, hi) - fld(cp, hi);
                    const Ent *elo = L.ent + (k * M + lo) * M, *ehi = L.ent + (k * M + hi) * M;
                    double ro[M];   // row j's sum when j is neither lo nor hi
                    double rlo = 0.0, rhi = 0.0;
#pragma unroll
                    for (int j = 0; j < M; ++j) {
                        const Ent e1 = elo[j];
                        const int n1 = __mul24(ulo, D[j]) + __mul24(u[j], Dlo);
                        const double dl = sq_dev(e1.cnt + n1, e1.R, e1.t) - e1.sq;
                        const Ent e2 = ehi[j];
                        const int n2 = __mul24(-ulo, D[j]) + __mul24(u[j], Dhi);
                        const double dh = sq_dev(e2.cnt + n2, e2.R, e2.t) - e2.sq;
                        rlo = rlo + dl;
                        rhi = rhi + dh;
                        ro[j] = dl + dh;
                    }
#pragma unroll
                    for (int i = 0; i < M; ++i) dQ = dQ + (i == lo ? rlo : (i == hi ? rhi : ro[i]));
                } else {
                    const Ent *row = L.ent + k * M * M;
#pragma unroll
                    for (int i = 0; i < M; ++i) {
                        double rs = 0.0;
#pragma unroll
                        for (int j = 0; j < M; ++j) {
                            const Ent en = row[i * M + j];
                            const int dn = __mul24(u[i], D[j]) + __mul24(u[j], D[i]);
                            const double sn = sq_dev(en.cnt + dn, en.R, en.t);
                            rs = rs + (sn - en.sq);
                        }
                        dQ = dQ + rs;
                    }
                }
            }
            if (k >= 0 && slot < B && kw < ke) {
                ((Hist *)L.rec_cp)[k * Bt + rix] = cp;
                ((Hist *)L.rec_cq)[k * Bt + rix] = cq;
                L.rec_dQ[k * Bt + rix] = dQ;
            }
        }
        __syncthreads();

        // ---- phase 2: per step of the pass (its first wavefront, steps side by
        // side): dS per slot, nulls, improving slots ranked by (dS, slot) -----------
        if (grp % Gs == 0 && wave == grp * W && kw < ke) {
            const int kk = kw;
            int32_t *ord = L.order + kk * B;
            int32_t *lst = L.list + kk * B;
            int n_impr = 0;
            int step_nulls = 0;
            double my_dS = 0.0;
            uint64_t imp_mask = 0;
            for (int g = 0; g < Gs; ++g) {
                const int s = g * kWave + lane;
                const int r = kk * B + s;
                bool imp = false;
                if (s < B) {
                    const uint32_t ab = L.rec_ab[r];
                    const bool act = (ab >> 17) & 1u, nul = (ab >> 16) & 1u;
                    double dS = 0.0;
#pragma unroll
                    for (int q = 0; q < kMaxShells; ++q)
                        if (q < S) dS = dS + wk[q] * L.rec_dQ[q * Bt + r];
                    L.rec_dS[r] = dS;
                    my_dS = dS;
                    imp = act && !nul && (dS < -tau);
                    step_nulls += (int)__popcll(ballot64(act && nul));
                } else {
                    step_nulls += (int)__popcll(ballot64(false));
                }
                const uint64_t mask = ballot64(imp);
                const int before = (int)__popcll(mask & ((1ull << lane) - 1ull));
                if (imp) lst[n_impr + before] = s;
                n_impr += (int)__popcll(mask);
                imp_mask = mask;
            }
            if (n_impr > 0) {
                if (Gs == 1) {
                    // rank with the improving slots' dS read across lanes
                    int rank = 0;
                    for (uint64_t m = imp_mask; m; m &= m - 1) {
                        const int l = __ffsll((long long)m) - 1;
                        const double d2 = readlane_f64(my_dS, l);
                        rank += (d2 < my_dS || (d2 == my_dS && l < lane)) ? 1 : 0;
                    }
                    if ((imp_mask >> lane) & 1ull) ord[rank] = lane;
                } else {
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_s_waitcnt(0);
                    for (int idx = lane; idx < n_impr; idx += kWave) {
                        const int s = lst[idx];
                        const double ds = L.rec_dS[kk * B + s];
                        int rank = 0;
                        for (int j = 0; j < n_impr; ++j) {
                            const int s2 = lst[j];
                            const double d2 = L.rec_dS[kk * B + s2];
                            rank += (d2 < ds || (d2 == ds && s2 < s)) ? 1 : 0;
                        }
                        ord[rank] = s;
                    }
                }
            }
            if (lane == 0) {
                L.sh_int[4 + kk] = step_nulls;
                L.sh_int[12 + kk] = n_impr;
            }
        }
        __syncthreads();
        int kstar = ke;
        for (int kk = ke - 1; kk >= 0; --kk)
            if (L.sh_int[12 + kk] > 0) kstar = kk;
        const int n_impr = kstar < ke ? L.sh_int[12 + kstar] : 0;
        int pass_steps = 0;
        // steps of the pass before kstar commit nothing
        for (int kk = 0; kk < kstar && !done; ++kk) {
            const int64_t left = d.n_trials - trials;
            trials += left < B ? left : B;
            nulls += L.sh_int[4 + kk];
            ++step;
            ++depth;
            ++pass_steps;
            if (d.depth_limit > 0 && depth >= d.depth_limit) {
                stop_reason = PYHEA_STOP_DEPTH;
                done = true;
            } else if (trials >= d.n_trials) {
                stop_reason = PYHEA_STOP_TRIALS;
                done = true;
            }
        }
        if (done || kstar >= ke) {
            steps_run += pass_steps;
            kpref = K;
            __syncthreads();
            continue;
        }
        const int rb = kstar * B;   // records of the committing step
        const int tasks = (int)min((int64_t)B, d.n_trials - trials);

        // ---- phase 3: commits ---------------------------------------------------------
        // Candidates in rank order.  A candidate within shells 1..S of an earlier
        // commit of this step is skipped; the others keep their neighbour
        // histograms, so re-validation needs only the running counts.  Every wave
        // keeps the committed positions in registers (position 2c + {0,1} of
        // commit c in lane (2c) % 64 of register (2c) / 64) and reaches the same
        // decisions; shell k's entries belong to one wave, and the waves meet once
        // per re-validated candidate to add the shells' dQ.  Site writes wait
        // until the end of the phase: later candidates never read committed sites.
        int n_commit = 0;
        const bool spec = CH > 0 && d.mode == PYHEA_MODE_DISJOINT && n_impr >= 3 && n_impr <= kWave;
        if (spec) {
            // The same rule, evaluated speculatively.  cm[u] marks the earlier
            // candidates that candidate u conflicts with.  The greedy conflict-free
            // set I of the undecided candidates is evaluated against the running
            // counts as if every member commits, CH members at a time; members
            // before the first one that fails re-validation commit, exactly as they
            // would one by one, and the search resumes after the failed member.
            const int nwaves = nthreads / kWave;
            for (int u = wave; u < n_impr; u += nwaves) {
                const int su = L.order[rb + u];
                const uint32_t up = L.rec_pp[rb + su], uq = L.rec_pq[rb + su];
                bool hit = false;
                if (lane < u) {
                    const int sv = L.order[rb + lane];
                    const uint32_t vp = L.rec_pp[rb + sv], vq = L.rec_pq[rb + sv];
                    hit = near_or_equal(d, up, vp) || near_or_equal(d, up, vq) || near_or_equal(d, uq, vp) ||
                          near_or_equal(d, uq, vq);
                }
                const uint64_t mk = ballot64(hit);
                if (lane == 0) L.spec_cm[u] = mk;
            }
            __syncthreads();
            // The search state (committed candidates, the current conflict-free set,
            // the next undecided rank) lives in wavefront 0, which hands each chunk's
            // members to the others through LDS: the scalar work runs once, not once
            // per wavefront on the CU's shared scalar unit.
            const uint64_t my_cm = wave == 0 && lane < n_impr ? L.spec_cm[lane] : 0ull;
            uint64_t committed = 0, I = 0, chunk = 0;
            int next = 0, my_s = 0;
            for (;;) {
                if (wave == 0) {
                    if (I == 0 && next < n_impr) {
                        for (int u = next; u < n_impr; ++u)
                            if ((readlane_u64(my_cm, u) & (committed | I)) == 0) I |= 1ull << u;
                        next = n_impr;
                    }
                    // the next CH members; lane vi < m holds member vi's slot
                    chunk = 0;
                    int m = 0, my_u = 0;
                    for (uint64_t t2 = I; t2 && m < CH; t2 &= t2 - 1, ++m) {
                        const uint64_t low = t2 & (~t2 + 1ull);
                        chunk |= low;
                        if (lane == m) my_u = __ffsll((long long)low) - 1;
                    }
                    my_s = lane < m ? L.order[rb + my_u] : 0;
                    if (lane < m) L.spec_mem[lane] = my_s;
                    if (lane == 0) L.spec_ctl[0] = m;
                }
                __syncthreads();
                const int m = L.spec_ctl[0];
                if (m == 0) break;
                // each entry's count change under each member: the members of a chunk
                // lie along a 16-lane row, an inclusive prefix of the changes gives
                // the counts before each member, then the member's term change
                for (int eb = wave * 4; eb < E; eb += nwaves * 4) {
                    const int e = eb + (lane >> 4), vi = lane & 15;
                    const bool valid = e < E && vi < m;
                    int dn = 0;
                    if (valid) dn = entry_dn<M, Hist>(L, Bt, rb + L.spec_mem[vi], e / (M * M), (e / M) % M, e % M);
                    const int incl = row_prefix_sum(dn);
                    if (valid) {
                        const Ent en = L.ent[e];
                        const int before = en.cnt + incl - dn;
                        double delta = 0.0;
                        if (dn != 0) delta = sq_dev(before + dn, en.R, en.t) - sq_dev(before, en.R, en.t);
                        L.spec_T[vi * E + e] = delta;
                        L.spec_P[vi * E + e] = incl;
                    }
                }
                __syncthreads();
                // dQ_k per member: rows in order, each row's terms in order (terms
                // of unchanged entries are exactly +0.0)
                for (int it = threadIdx.x; it < m * S; it += nthreads) {
                    const int vi = it / S, kk = it - vi * S;
                    const double *T = L.spec_T + vi * E + kk * M * M;
                    double Q = 0.0;
#pragma unroll
                    for (int i = 0; i < M; ++i) {
                        double rs = 0.0;
#pragma unroll
                        for (int j = 0; j < M; ++j) rs = rs + T[i * M + j];
                        Q = Q + rs;
                    }
                    L.spec_Q[vi * kMaxShells + kk] = Q;
                }
                __syncthreads();
                // the first member whose dS fails (the step's first commit is not
                // re-validated); every wavefront finds the same one
                bool fails = false;
                if (lane < m) {
                    double dS = 0.0;
#pragma unroll
                    for (int kk = 0; kk < kMaxShells; ++kk)
                        if (kk < S) dS = dS + wk[kk] * L.spec_Q[lane * kMaxShells + kk];
                    fails = !(dS < -tau) && !(n_commit == 0 && lane == 0);
                }
                const uint64_t fm = ballot64(fails);
                const int f = fm ? __ffsll((long long)fm) - 1 : m;
                // members [0, f) commit: counts after member f - 1, their squared
                // deviations, and the list of committed slots
                if (f > 0)
                    for (int e = threadIdx.x; e < E; e += nthreads) {
                        const int dsum = L.spec_P[(f - 1) * E + e];
                        if (dsum != 0) {
                            Ent en = L.ent[e];
                            en.cnt += dsum;
                            en.sq = sq_dev(en.cnt, en.R, en.t);
                            L.ent[e] = en;
                        }
                    }
                if (wave == 0) {
                    if (lane < f) L.list[n_commit + lane] = my_s;
                    uint64_t t2 = chunk;
                    for (int vi = 0; vi < f; ++vi) {
                        committed |= t2 & (~t2 + 1ull);
                        t2 &= t2 - 1;
                    }
                    I &= ~chunk;
                    if (f < m) {
                        // resume after the member that failed, with a new conflict-free set
                        next = __ffsll((long long)t2);
                        I = 0;
                    }
                }
                n_commit += f;
            }
        }
        int n_meet = 0;
        uint32_t cpr[kMaxB / 32];
#pragma unroll
        for (int r = 0; r < kMaxB / 32; ++r) cpr[r] = 0;
        const bool ewave = grp == 0 && k >= 0;   // one wave per shell handles its entries
        for (int u = 0; !spec && u < n_impr; ++u) {
            if (d.mode == PYHEA_MODE_BEST && n_commit > 0) break;
            const int s = L.order[rb + u];
            const uint32_t upp = L.rec_pp[rb + s], upq = L.rec_pq[rb + s];
            bool hit = false;
#pragma unroll
            for (int r = 0; r < kMaxB / 32; ++r) {
                if (r * kWave >= 2 * n_commit) break;
                if (r * kWave + lane < 2 * n_commit)
                    hit |= near_or_equal(d, upp, cpr[r]) || near_or_equal(d, upq, cpr[r]);
            }
            if (ballot64(hit) != 0) continue;
            const uint32_t ab = L.rec_ab[rb + s];
            const int a = (int)(ab & 0xFFu), b = (int)((ab >> 8) & 0xFFu);
            // this wave's shell-k change of entry e = lane (the S entry waves only)
            int dn = 0;
            int e = 0;
            if (ewave && lane < M * M) {
                const Hist cp = ((const Hist *)L.rec_cp)[k * Bt + rb + s];
                const Hist cq = ((const Hist *)L.rec_cq)[k * Bt + rb + s];
                const int i = lane / M, j = lane - (lane / M) * M;
                const int ui = (i == a ? 1 : 0) - (i == b ? 1 : 0), uj = (j == a ? 1 : 0) - (j == b ? 1 : 0);
                dn = __mul24(ui, fld(cq, j) - fld(cp, j)) + __mul24(uj, fld(cq, i) - fld(cp, i));
                e = k * M * M + lane;
            }
            bool ok = true;
            if (n_commit > 0) {
                double *dq = L.sh_dQ + (n_meet & 1) * kMaxShells;   // alternating buffers
                if (ewave) {
                    double delta = 0.0;
                    if (dn != 0) {
                        const Ent en = L.ent[e];
                        delta = sq_dev(en.cnt + dn, en.R, en.t) - en.sq;
                    }
                    // row i summed in lane i over j in order, then the rows in order.
                    // Entries with dN = 0 hold +0.0; a sum that starts at +0.0 never
                    // becomes -0.0 (deltas are never -0.0), so adding them is exact.
                    double rs = 0.0;
#pragma unroll
                    for (int j = 0; j < M; ++j) rs = rs + shfl_f64(delta, lane * M + j);
                    double acc = 0.0;
#pragma unroll
                    for (int i = 0; i < M; ++i) acc = acc + readlane_f64(rs, i);
                    if (lane == 0) dq[k] = acc;
                }
                __syncthreads();
                double q[kMaxShells];
#pragma unroll
                for (int kk = 0; kk < kMaxShells; ++kk) q[kk] = kk < S ? dq[kk] : 0.0;
                double dS = 0.0;
#pragma unroll
                for (int kk = 0; kk < kMaxShells; ++kk)
                    if (kk < S) dS = dS + wk[kk] * q[kk];
                ok = dS < -tau;
                ++n_meet;
            }
            if (!ok) continue;
            // apply: counts and squared deviations of shell k (wave-private entries)
            if (ewave && dn != 0) {
                Ent en = L.ent[e];
                en.cnt += dn;
                en.sq = sq_dev(en.cnt, en.R, en.t);
                L.ent[e] = en;
            }
            {
                const int c0 = 2 * n_commit, r0 = c0 / kWave;
#pragma unroll
                for (int r = 0; r < kMaxB / 32; ++r)
                    if (r == r0) {
                        cpr[r] = lane == (c0 & (kWave - 1)) ? upp : cpr[r];
                        cpr[r] = lane == ((c0 + 1) & (kWave - 1)) ? upq : cpr[r];
                    }
            }
            if (threadIdx.x == 0) L.list[n_commit] = s;
            ++n_commit;
        }
        __syncthreads();
        // the committed swaps: every copy of both sites, and the log
        for (int t = threadIdx.x; t < n_commit * 2; t += nthreads) {
            const int s = L.list[t >> 1];
            const int side = t & 1;
            const uint32_t ab = L.rec_ab[rb + s];
            const SiteCoord sc = pos_site(d, side ? L.rec_pq[rb + s] : L.rec_pp[rb + s]);
            const int v = side ? (int)(ab & 0xFFu) : (int)((ab >> 8) & 0xFFu);
            write_site<kStore>(L, d, sc.cx, sc.cy, sc.cz, sc.b, v);
        }
        if (d.log) {
            for (int c = threadIdx.x; c < n_commit; c += nthreads) {
                const int64_t at = commits + c;
                if (at < d.log_cap) {
                    const int s = L.list[c];
                    uint32_t *rec = d.log + 4 * at;
                    rec[0] = (uint32_t)step;
                    rec[1] = (uint32_t)s;
                    rec[2] = site_id(d, pos_site(d, L.rec_pp[rb + s]));
                    rec[3] = site_id(d, pos_site(d, L.rec_pq[rb + s]));
                }
            }
        }
        commits += n_commit;

        // ---- phase 4: bookkeeping of the committing step ----------------------------
        trials += tasks;
        nulls += L.sh_int[4 + kstar];
        ++step;
        ++pass_steps;
        depth = n_commit > 0 ? 0 : depth + 1;
        if (d.depth_limit > 0 && depth >= d.depth_limit) {
            stop_reason = PYHEA_STOP_DEPTH;
            done = true;
        } else if (trials >= d.n_trials) {
            stop_reason = PYHEA_STOP_TRIALS;
            done = true;
        }
        steps_run += pass_steps;
        kpref = kstar == 0 ? 1 : K;
        __syncthreads();
    }

    // ---- write back -------------------------------------------------------------------
    for (int e = threadIdx.x; e < E; e += nthreads) d.counts[e] = L.ent[e].cnt;
    if constexpr (kStore != kStoreGlobal) {
        for (uint32_t p = threadIdx.x; p < d.N; p += nthreads) {
            const SiteCoord c = site_coord(p, d.lgA, d.Lx, d.Ly, d.inv_Lx, d.inv_Ly);
            d.species[p] = (int8_t)load_species<kStore>(L, d, padded_id(d, c.cx + h, c.cy + h, c.cz + h, c.b));
        }
    }
    if (threadIdx.x == 0) {
        st->trials = trials;
        st->commits = commits;
        st->steps = step;
        st->null_trials = nulls;
        st->depth = depth;
        if (done) {
            st->stop_reason = stop_reason;
            st->done = 1;
        }
    }
}

// padded HBM copy <-> unpadded configuration (HBM-resident chains)
// Chain states of many chains into one contiguous array (one read-back).
__global__ void gather_states_kernel(const ChainDesc *__restrict__ descs, int n, ChainState *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = *descs[i].state;
}

__global__ void pad_fill_kernel(const ChainDesc *__restrict__ descs) {
    const ChainDesc &d = descs[blockIdx.y];
    if (d.store != kStoreGlobal || d.state->status != 0) return;
    const double inv_PX = 1.0 / (double)d.PX, inv_PY = 1.0 / (double)d.PY;
    for (uint32_t pid = blockIdx.x * blockDim.x + threadIdx.x; pid < d.Npad;
         pid += gridDim.x * blockDim.x) {
        const SiteCoord c = site_coord(pid, d.lgA, d.PX, d.PY, inv_PX, inv_PY);
        const int cx = wrap_axis(c.cx - d.halo, d.Lx), cy = wrap_axis(c.cy - d.halo, d.Ly),
                  cz = wrap_axis(c.cz - d.halo, d.Lz);
        d.pad_global[pid] = d.species[((cz * d.Ly + cy) * d.Lx + cx) * d.A + c.b];
    }
}

__global__ void pad_drain_kernel(const ChainDesc *__restrict__ descs) {
    const ChainDesc &d = descs[blockIdx.y];
    if (d.store != kStoreGlobal || d.state->status != 0) return;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < d.N; p += gridDim.x * blockDim.x) {
        const SiteCoord c = site_coord(p, d.lgA, d.Lx, d.Ly, d.inv_Lx, d.inv_Ly);
        d.species[p] = d.pad_global[padded_id(d, c.cx + d.halo, c.cy + d.halo, c.cz + d.halo, c.b)];
    }
}

}  // namespace

int mc_block_threads(int B, int W, int K) { return mc_block_waves(B, W, K) * kWave; }

template <int kStore>
const void *mc_fn(int M) {
    switch (M) {
        case 2: return (const void *)mc_kernel<kStore, 2>;
        case 3: return (const void *)mc_kernel<kStore, 3>;
        case 4: return (const void *)mc_kernel<kStore, 4>;
        case 5: return (const void *)mc_kernel<kStore, 5>;
        case 6: return (const void *)mc_kernel<kStore, 6>;
        case 7: return (const void *)mc_kernel<kStore, 7>;
        default: return (const void *)mc_kernel<kStore, 8>;
    }
}

hipError_t launch_mc(const ChainDesc *descs_dev, int n_chains, int store, int M, int S, int B, int W, int bal,
                     int K, int CH, int lds_bytes, int max_steps, hipStream_t stream) {
    if (mc_block_threads(B, W, K) > 1024 || K < 1 || K > kMaxLookahead || W < S || (!bal && W != S) || CH < 0 ||
        CH > 16)
        return hipErrorInvalidValue;
    const dim3 grid(n_chains), block(mc_block_threads(B, W, K));
    const void *fn = store == kStoreLds8 ? mc_fn<kStoreLds8>(M)
                     : store == kStoreLds4 ? mc_fn<kStoreLds4>(M)
                                           : mc_fn<kStoreGlobal>(M);
    hipError_t e = set_max_lds(fn, lds_bytes);
    if (e != hipSuccess) return e;
    void *args[] = {(void *)&descs_dev, (void *)&max_steps, (void *)&W, (void *)&bal, (void *)&K, (void *)&CH};
    return hipLaunchKernel(fn, grid, block, args, (size_t)lds_bytes, stream);
}

hipError_t launch_gather_states(const ChainDesc *descs_dev, int n_chains, ChainState *out, hipStream_t stream) {
    if (n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_states_kernel, dim3((n_chains + 255) / 256), dim3(256), 0, stream, descs_dev, n_chains,
                       out);
    return hipGetLastError();
}

// Species totals and the ratio table R = N / (n_i n_j z_k) of each chain from
// its initial pair counts (Eq. 2; n_i = row sum of shell 1 / z_1, one exact
// integer product and one IEEE division per entry).  A chain with an invalid id
// or an absent species is marked done with status EINVAL and left untouched.
__global__ void chain_ratio_kernel(const ChainDesc *__restrict__ descs, int n, const int32_t *__restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const ChainDesc &d = descs[i];
    const int M = d.M, S = d.S;
    int64_t nsp[kMaxSpecies];
    bool ok = bad[i] == 0;
    for (int a = 0; a < M; ++a) {
        int64_t r = 0;
        for (int b = 0; b < M; ++b) r += d.counts[a * M + b];
        nsp[a] = r / d.zk[0];
        ok = ok && nsp[a] > 0;
    }
    if (!ok) {
        d.state->status = PYHEA_EINVAL;
        d.state->done = 1;
        return;
    }
    double *R = const_cast<double *>(d.R);
    for (int k = 0; k < S; ++k)
        for (int a = 0; a < M; ++a)
            for (int b = 0; b < M; ++b)
                R[(k * M + a) * M + b] = (double)d.N / (double)(nsp[a] * nsp[b] * (int64_t)d.zk[k]);
}

hipError_t launch_chain_ratio(const ChainDesc *descs_dev, int n_chains, const int32_t *bad, hipStream_t stream) {
    if (n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(chain_ratio_kernel, dim3((n_chains + 63) / 64), dim3(64), 0, stream, descs_dev, n_chains, bad);
    return hipGetLastError();
}

hipError_t launch_pad_fill(const ChainDesc *descs_dev, int n_chains, hipStream_t stream) {
    hipLaunchKernelGGL(pad_fill_kernel, dim3(64, n_chains), dim3(256), 0, stream, descs_dev);
    return hipGetLastError();
}

hipError_t launch_pad_drain(const ChainDesc *descs_dev, int n_chains, hipStream_t stream) {
    hipLaunchKernelGGL(pad_drain_kernel, dim3(64, n_chains), dim3(256), 0, stream, descs_dev);
    return hipGetLastError();
}

}  // namespace pyhea
