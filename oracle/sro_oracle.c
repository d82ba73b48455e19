/*
 * CPU oracle for Warren-Cowley short-range-order (SRO) evaluation and the
 * incremental-swap Monte Carlo search of Niu & Liu, "Short-Range Order Based
 * Ultra Fast Large-Scale Modeling of High-Entropy Alloys" (arXiv:2411.18906).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, single-threaded
 * restatement of the method, used to check the HIP library.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC.
 * All floating point is IEEE binary64 with +, -, *, /, sqrt only and no fused
 * multiply-add, so every value below is fixed to the bit.
 *
 * Readings of the paper that this file takes where the text is silent or
 * garbled (each one is also listed with its reason in the design notes):
 *  - periodic boundaries; ideal FCC/BCC shells selected by squared distance;
 *  - pair counts are ordered and symmetric, counted once per (site, offset);
 *  - P_ij = N_ij / (n_i z_k) (conditional probability, Sec. 4.3, Eq. 2);
 *  - decisions use S = F^2 (the sum under the square root of Eq. 3); an
 *    improvement is S_new - S_cur < -tau, tau = 0 meaning strict improvement
 *    (the sign printed in Algorithms 2 and 3 contradicts the text of Sec. 4.2);
 *  - ties in the per-step sort (Eq. 6) are broken by the task (slot) index;
 *  - the search depth counts steps that committed nothing (Sec. 4.2, 4.6.4);
 *  - random trial swaps come from Philox4x32-10 (Salmon et al., SC'11).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_FCC 0
#define OR_BCC 1
#define OR_MAX_SHELLS 4
#define OR_MAX_SPECIES 8
#define OR_MAX_OFFSETS 64 /* FCC shells 1-4: 54 offsets; BCC: 50 */

/* ------------------------------------------------------------------------ */
/* Lattice geometry in half-lattice-constant integer units.                  */
/* FCC sites: 2*cell + {(0,0,0),(1,1,0),(1,0,1),(0,1,1)} (4 atoms per cell,   */
/* S = 4 L^3); BCC: 2*cell + {(0,0,0),(1,1,1)} (2 per cell, S = 2 L^3).       */
/* These are the supercells of the benchmark tables (S = A * L^3).            */
/* ------------------------------------------------------------------------ */

static const int FCC_BASIS[4][3] = {{0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
static const int BCC_BASIS[2][3] = {{0, 0, 0}, {1, 1, 1}};

static int n_basis(int lattice) { return lattice == OR_FCC ? 4 : 2; }

static const int *basis_vec(int lattice, int b) {
    return lattice == OR_FCC ? FCC_BASIS[b] : BCC_BASIS[b];
}

/* Is the integer vector v a translation of the lattice? */
static int is_lattice_vector(int lattice, int x, int y, int z) {
    int px = x & 1, py = y & 1, pz = z & 1; /* parity; & works for negatives */
    if (lattice == OR_FCC) return ((px + py + pz) & 1) == 0;
    return px == py && py == pz;
}

/*
 * Coordination shells: shell k is the set of lattice vectors with the k-th
 * smallest nonzero squared length.  Found by brute force over a cube large
 * enough for four shells.  Offsets are listed shell by shell in a fixed order.
 * Returns the total number of offsets, or -1 on bad arguments.
 */
int or_shells(int lattice, int n_shells, int *r2_out, int *z_out, int *offsets_out /* [n][3] */) {
    if ((lattice != OR_FCC && lattice != OR_BCC) || n_shells < 1 || n_shells > OR_MAX_SHELLS)
        return -1;
    /* distinct squared lengths in ascending order */
    int r2s[OR_MAX_SHELLS];
    int found = 0;
    int last = 0;
    while (found < n_shells) {
        int best = 1 << 30;
        for (int z = -4; z <= 4; ++z)
            for (int y = -4; y <= 4; ++y)
                for (int x = -4; x <= 4; ++x) {
                    int r2 = x * x + y * y + z * z;
                    if (r2 > last && r2 < best && is_lattice_vector(lattice, x, y, z)) best = r2;
                }
        r2s[found++] = best;
        last = best;
    }
    int n = 0;
    for (int k = 0; k < n_shells; ++k) {
        int zk = 0;
        for (int z = -4; z <= 4; ++z)
            for (int y = -4; y <= 4; ++y)
                for (int x = -4; x <= 4; ++x) {
                    if (x * x + y * y + z * z != r2s[k] || !is_lattice_vector(lattice, x, y, z))
                        continue;
                    offsets_out[3 * n + 0] = x;
                    offsets_out[3 * n + 1] = y;
                    offsets_out[3 * n + 2] = z;
                    ++n;
                    ++zk;
                }
        r2_out[k] = r2s[k];
        z_out[k] = zk;
    }
    return n;
}

int64_t or_n_sites(int lattice, const int *L) {
    return (int64_t)n_basis(lattice) * L[0] * L[1] * L[2];
}

/* site id p = ((cz*Ly + cy)*Lx + cx)*A + b  <->  position 2*cell + basis_b */
void or_site_pos(int lattice, const int *L, int64_t p, int *pos) {
    int A = n_basis(lattice);
    int b = (int)(p % A);
    int64_t c = p / A;
    int cx = (int)(c % L[0]);
    c /= L[0];
    int cy = (int)(c % L[1]);
    int cz = (int)(c / L[1]);
    const int *bv = basis_vec(lattice, b);
    pos[0] = 2 * cx + bv[0];
    pos[1] = 2 * cy + bv[1];
    pos[2] = 2 * cz + bv[2];
}

static int wrap(int v, int m) {
    int r = v % m;
    return r < 0 ? r + m : r;
}

/* id of the site at a lattice position (wrapped periodically); -1 if the
 * position is not a lattice site */
int64_t or_site_id(int lattice, const int *L, const int *pos_in) {
    int pos[3];
    for (int a = 0; a < 3; ++a) pos[a] = wrap(pos_in[a], 2 * L[a]);
    int A = n_basis(lattice);
    for (int b = 0; b < A; ++b) {
        const int *bv = basis_vec(lattice, b);
        if ((pos[0] & 1) == bv[0] && (pos[1] & 1) == bv[1] && (pos[2] & 1) == bv[2]) {
            int cx = pos[0] >> 1, cy = pos[1] >> 1, cz = pos[2] >> 1;
            return (((int64_t)cz * L[1] + cy) * L[0] + cx) * A + b;
        }
    }
    return -1;
}

/* neighbour of site p along lattice vector d (periodic) */
static int64_t nbr(int lattice, const int *L, int64_t p, const int *d) {
    int pos[3];
    or_site_pos(lattice, L, p, pos);
    pos[0] += d[0];
    pos[1] += d[1];
    pos[2] += d[2];
    return or_site_id(lattice, L, pos);
}

/* all neighbours of p in shells 1..S, in offset order; returns the count */
int or_neighbors(int lattice, const int *L, int n_shells, int64_t p, int64_t *out) {
    int r2[OR_MAX_SHELLS], z[OR_MAX_SHELLS], off[OR_MAX_OFFSETS * 3];
    int n = or_shells(lattice, n_shells, r2, z, off);
    for (int t = 0; t < n; ++t) out[t] = nbr(lattice, L, p, &off[3 * t]);
    return n;
}

/*
 * Input validation.  Returns 0 if the problem is well posed, else a negative
 * code: -1 bad lattice/size/M/S, -2 a species id outside [0, M), -3 a species
 * with no atoms (c_j = 0 makes Eq. 2 undefined), -4 a shell offset that maps a
 * site onto itself (cell too small along some axis).
 */
int or_validate(int lattice, const int *L, int M, int S, const int8_t *species) {
    if ((lattice != OR_FCC && lattice != OR_BCC) || M < 2 || M > OR_MAX_SPECIES || S < 1 ||
        S > OR_MAX_SHELLS || L[0] < 1 || L[1] < 1 || L[2] < 1)
        return -1;
    int r2[OR_MAX_SHELLS], z[OR_MAX_SHELLS], off[OR_MAX_OFFSETS * 3];
    int n = or_shells(lattice, S, r2, z, off);
    for (int t = 0; t < n; ++t) {
        if (wrap(off[3 * t], 2 * L[0]) == 0 && wrap(off[3 * t + 1], 2 * L[1]) == 0 &&
            wrap(off[3 * t + 2], 2 * L[2]) == 0)
            return -4;
    }
    if (species) {
        int64_t N = or_n_sites(lattice, L);
        int64_t cnt[OR_MAX_SPECIES] = {0};
        for (int64_t p = 0; p < N; ++p) {
            if (species[p] < 0 || species[p] >= M) return -2;
            cnt[species[p]]++;
        }
        for (int i = 0; i < M; ++i)
            if (cnt[i] == 0) return -3;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Pair counts (Sec. 4.3): N[k][i][j] = #{(p, d) : d in shell k, s_p = i,     */
/* s_{p+d} = j}, counted over every site and every offset.                    */
/* ------------------------------------------------------------------------ */

void or_counts(int lattice, const int *L, int M, int S, const int8_t *species,
               int64_t *counts /* [S][M][M] */) {
    int r2[OR_MAX_SHELLS], z[OR_MAX_SHELLS], off[OR_MAX_OFFSETS * 3];
    or_shells(lattice, S, r2, z, off);
    int64_t N = or_n_sites(lattice, L);
    memset(counts, 0, sizeof(int64_t) * S * M * M);
    int t0 = 0;
    for (int k = 0; k < S; ++k) {
        for (int64_t p = 0; p < N; ++p) {
            for (int t = t0; t < t0 + z[k]; ++t) {
                int64_t q = nbr(lattice, L, p, &off[3 * t]);
                counts[(k * M + species[p]) * M + species[q]] += 1;
            }
        }
        t0 += z[k];
    }
}

void or_species_counts(int64_t N, int M, const int8_t *species, int64_t *n_out) {
    for (int i = 0; i < M; ++i) n_out[i] = 0;
    for (int64_t p = 0; p < N; ++p) n_out[species[p]]++;
}

/*
 * Eq. 2 and Eq. 3 in binary64.  With P_ij = N_ij / (n_i z_k) and c_j = n_j / N,
 * alpha_ij = 1 - P_ij / c_j = 1 - N_ij * N / (n_i n_j z_k).  The factor
 * R = N / (n_i n_j z_k) is one IEEE division of two exact integers; then
 * alpha = 1 - N_ij * R and d = alpha - target.  Eq. 3 is evaluated with its own
 * nesting: for each row i the sum over j of d * d (from +0.0), Q_k = the sum of
 * the row sums over i (from +0.0), then S = sum over k of w_k * Q_k (from
 * +0.0), F = sqrt(S).
 */
void or_ratio_table(int64_t N, int M, int S, const int *z, const int64_t *n, double *R) {
    for (int k = 0; k < S; ++k)
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                int64_t den = n[i] * n[j] * (int64_t)z[k];
                R[(k * M + i) * M + j] = (double)N / (double)den;
            }
}

/* squared deviation (alpha - target)^2 of one entry with pair count `count` */
static double sq_dev(int64_t count, double R, double t) {
    double alpha = 1.0 - (double)count * R;
    double d = alpha - t;
    return d * d;
}

/* alpha[S][M][M], sq[S][M][M] = (alpha - target)^2, and S_F[2] = {S, F} */
void or_alpha_objective(int lattice, const int *L, int M, int S, const int8_t *species,
                        const int64_t *counts, const double *target, const double *weight,
                        double *alpha, double *sq, double *S_F) {
    int r2[OR_MAX_SHELLS], z[OR_MAX_SHELLS], off[OR_MAX_OFFSETS * 3];
    or_shells(lattice, S, r2, z, off);
    int64_t N = or_n_sites(lattice, L);
    int64_t n[OR_MAX_SPECIES];
    or_species_counts(N, M, species, n);
    double R[OR_MAX_SHELLS * OR_MAX_SPECIES * OR_MAX_SPECIES];
    or_ratio_table(N, M, S, z, n, R);
    double sum = 0.0;
    for (int k = 0; k < S; ++k) {
        double Q = 0.0;
        for (int i = 0; i < M; ++i) {
            double row = 0.0;
            for (int j = 0; j < M; ++j) {
                int e = (k * M + i) * M + j;
                double a = 1.0 - (double)counts[e] * R[e];
                double d = a - target[e];
                if (alpha) alpha[e] = a;
                if (sq) sq[e] = d * d;
                row = row + d * d;
            }
            Q = Q + row;
        }
        sum = sum + weight[k] * Q;
    }
    S_F[0] = sum;
    S_F[1] = sqrt(sum);
}

/* ------------------------------------------------------------------------ */
/* Incremental update (Sec. 4.5, Eq. 4).  Swapping sites p (species a) and q  */
/* (species b, a != b) changes only the bonds of p and q.  With c_p[j], c_q[j] */
/* the species histograms of the shell-k neighbours of p and q, each          */
/* excluding the partner site, and D = c_q - c_p:                             */
/*   dN[a][j] = dN[j][a] = D[j], dN[b][j] = dN[j][b] = -D[j]  (j not a, b)     */
/*   dN[a][a] = 2 D[a], dN[b][b] = -2 D[b], dN[a][b] = dN[b][a] = D[b] - D[a]  */
/* and every other entry is zero.  The p-q bond itself is unchanged.          */
/* ------------------------------------------------------------------------ */

void or_swap_delta(int lattice, const int *L, int M, int S, const int8_t *species, int64_t p,
                   int64_t q, int64_t *dN /* [S][M][M] */) {
    int r2[OR_MAX_SHELLS], z[OR_MAX_SHELLS], off[OR_MAX_OFFSETS * 3];
    or_shells(lattice, S, r2, z, off);
    memset(dN, 0, sizeof(int64_t) * S * M * M);
    int a = species[p], b = species[q];
    if (a == b) return;
    int t0 = 0;
    for (int k = 0; k < S; ++k) {
        int64_t D[OR_MAX_SPECIES] = {0};
        for (int t = t0; t < t0 + z[k]; ++t) {
            int64_t rp = nbr(lattice, L, p, &off[3 * t]);
            int64_t rq = nbr(lattice, L, q, &off[3 * t]);
            if (rp != q) D[species[rp]] -= 1;
            if (rq != p) D[species[rq]] += 1;
        }
        int64_t *m = dN + (int64_t)k * M * M;
        for (int j = 0; j < M; ++j) {
            if (j == a || j == b) continue;
            m[a * M + j] = D[j];
            m[j * M + a] = D[j];
            m[b * M + j] = -D[j];
            m[j * M + b] = -D[j];
        }
        m[a * M + a] = 2 * D[a];
        m[b * M + b] = -2 * D[b];
        m[a * M + b] = D[b] - D[a];
        m[b * M + a] = D[b] - D[a];
        t0 += z[k];
    }
}

/* dS = sum over k of w_k * dQ_k (from +0.0), with the nesting of Eq. 3:
 * dQ_k = sum over i of (sum over j of sq(N + dN) - sq(N)), each sum from +0.0.
 * Entries with dN = 0 add exactly +0.0. */
static double delta_objective(int M, int S, const int64_t *counts, const int64_t *dN,
                              const double *R, const double *target, const double *weight,
                              const double *sq) {
    double acc = 0.0;
    for (int k = 0; k < S; ++k) {
        double dQ = 0.0;
        for (int i = 0; i < M; ++i) {
            double row = 0.0;
            for (int j = 0; j < M; ++j) {
                int e = (k * M + i) * M + j;
                double sn = sq_dev(counts[e] + dN[e], R[e], target[e]);
                row = row + (sn - sq[e]);
            }
            dQ = dQ + row;
        }
        acc = acc + weight[k] * dQ;
    }
    return acc;
}

/* dS of one swap against a configuration (exported for tests) */
double or_swap_dS(int lattice, const int *L, int M, int S, const int8_t *species, int64_t p,
                  int64_t q, const double *target, const double *weight) {
    int r2[OR_MAX_SHELLS], z[OR_MAX_SHELLS], off[OR_MAX_OFFSETS * 3];
    or_shells(lattice, S, r2, z, off);
    int64_t N = or_n_sites(lattice, L);
    int64_t n[OR_MAX_SPECIES];
    or_species_counts(N, M, species, n);
    int64_t *counts = malloc(sizeof(int64_t) * S * M * M);
    int64_t *dN = malloc(sizeof(int64_t) * S * M * M);
    double R[OR_MAX_SHELLS * OR_MAX_SPECIES * OR_MAX_SPECIES];
    double sq[OR_MAX_SHELLS * OR_MAX_SPECIES * OR_MAX_SPECIES];
    or_ratio_table(N, M, S, z, n, R);
    or_counts(lattice, L, M, S, species, counts);
    for (int k = 0; k < S; ++k)
        for (int e = k * M * M; e < (k + 1) * M * M; ++e)
            sq[e] = sq_dev(counts[e], R[e], target[e]);
    or_swap_delta(lattice, L, M, S, species, p, q, dN);
    double r = delta_objective(M, S, counts, dN, R, target, weight, sq);
    free(counts);
    free(dN);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies by the   */
/* published multipliers, with a Weyl-sequence key schedule.                  */
/* ------------------------------------------------------------------------ */

void or_philox4x32_10(const uint32_t *ctr_in, const uint32_t *key_in, uint32_t *out) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Monte Carlo local search (Sec. 4.2, Algorithms 2 and 3; Sec. 4.6).         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t trials, null_trials, commits, steps;
    int32_t stop_reason; /* 0 = trial budget used, 1 = search depth reached */
    int32_t pad;
    double S, F;
    int64_t log_len;
} or_mc_stats;

typedef struct {
    int64_t p, q;
    int a, b;      /* species of p and q before the swap; a == b means null */
    double dS;
    int improving; /* dS < -tau */
} or_trial;

/* does site y coincide with x or lie in shells 1..S of x? */
static int near_or_equal(int lattice, const int *L, int n_off, const int *off, int64_t x,
                         int64_t y) {
    if (x == y) return 1;
    for (int t = 0; t < n_off; ++t)
        if (nbr(lattice, L, x, &off[3 * t]) == y) return 1;
    return 0;
}

/*
 * One chain.  Per step, B tasks (Algorithm 3) each draw one swap against the
 * same current configuration and compute dS incrementally; the step then
 * ranks the improving tasks by (dS, slot) (Eq. 6) and commits:
 *   mode 1 (BEST): the single best improving swap, as printed in Algorithm 3;
 *   mode 0 (DISJOINT): improving swaps in ranked order, skipping any swap that
 *     shares a site with, or has a site within shells 1..S of, a swap already
 *     committed this step; each survivor's dS is recomputed against the
 *     running state (its dN is unchanged because nothing near it moved) and it
 *     is committed if still < -tau.
 * Trial t of step s uses Philox4x32-10 with counter (slot, step, chain, 0) and
 * key (lo32(seed), hi32(seed)): p = (x0 * N) >> 32, q = (x1 * N) >> 32.  A draw
 * with equal species (including p == q) is a null trial.  The last step runs
 * only the trials left in the budget.  depth_limit > 0 stops the chain after
 * that many consecutive steps without a commit (Sec. 4.6.4).
 * log (optional): 4 uint32 per commit (step, slot, p, q), first log_cap kept.
 * counts_out (optional): the incrementally maintained counts at the end.
 * Returns 0, or the or_validate code.
 */
int or_mc_run(int lattice, const int *L, int M, int S, const double *target,
              const double *weight, uint64_t seed, uint32_t chain_id, int64_t n_trials, int B,
              int mode, int depth_limit, double tau, int8_t *species, uint32_t *log,
              int64_t log_cap, or_mc_stats *stats, int64_t *counts_out) {
    int v = or_validate(lattice, L, M, S, species);
    if (v) return v;
    if (B < 1 || n_trials < 0 || (mode != 0 && mode != 1)) return -1;
    int r2[OR_MAX_SHELLS], z[OR_MAX_SHELLS], off[OR_MAX_OFFSETS * 3];
    int n_off = or_shells(lattice, S, r2, z, off);
    int64_t N = or_n_sites(lattice, L);
    int64_t n[OR_MAX_SPECIES];
    or_species_counts(N, M, species, n);
    const int E = S * M * M;
    double R[OR_MAX_SHELLS * OR_MAX_SPECIES * OR_MAX_SPECIES];
    double sq[OR_MAX_SHELLS * OR_MAX_SPECIES * OR_MAX_SPECIES];
    or_ratio_table(N, M, S, z, n, R);
    int64_t *counts = malloc(sizeof(int64_t) * E);
    int64_t *dN_all = malloc(sizeof(int64_t) * E * (size_t)B);
    or_trial *tr = malloc(sizeof(or_trial) * (size_t)B);
    int *order = malloc(sizeof(int) * (size_t)B);
    int64_t *committed = malloc(sizeof(int64_t) * 2 * (size_t)B);
    or_counts(lattice, L, M, S, species, counts);
    for (int k = 0; k < S; ++k)
        for (int e = k * M * M; e < (k + 1) * M * M; ++e)
            sq[e] = sq_dev(counts[e], R[e], target[e]);

    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    memset(stats, 0, sizeof(*stats));
    int depth = 0;
    int64_t step = 0;
    while (stats->trials < n_trials) {
        int64_t left = n_trials - stats->trials;
        int tasks = left < B ? (int)left : B;
        /* every task draws a swap and evaluates it against the same state */
        int n_impr = 0;
        for (int slot = 0; slot < tasks; ++slot) {
            uint32_t ctr[4] = {(uint32_t)slot, (uint32_t)step, chain_id, 0u};
            uint32_t x[4];
            or_philox4x32_10(ctr, key, x);
            or_trial *t = &tr[slot];
            t->p = (int64_t)(((uint64_t)x[0] * (uint64_t)N) >> 32);
            t->q = (int64_t)(((uint64_t)x[1] * (uint64_t)N) >> 32);
            t->a = species[t->p];
            t->b = species[t->q];
            t->improving = 0;
            t->dS = 0.0;
            if (t->a == t->b) {
                stats->null_trials++;
                continue;
            }
            int64_t *dN = dN_all + (size_t)slot * E;
            or_swap_delta(lattice, L, M, S, species, t->p, t->q, dN);
            t->dS = delta_objective(M, S, counts, dN, R, target, weight, sq);
            if (t->dS < -tau) {
                t->improving = 1;
                order[n_impr++] = slot;
            }
        }
        stats->trials += tasks;
        /* rank improving tasks by (dS, slot): insertion sort, ascending */
        for (int u = 1; u < n_impr; ++u) {
            int s = order[u];
            int w = u - 1;
            while (w >= 0 && (tr[order[w]].dS > tr[s].dS ||
                              (tr[order[w]].dS == tr[s].dS && order[w] > s))) {
                order[w + 1] = order[w];
                --w;
            }
            order[w + 1] = s;
        }
        int n_commit = 0;
        for (int u = 0; u < n_impr; ++u) {
            int s = order[u];
            or_trial *t = &tr[s];
            int64_t *dN = dN_all + (size_t)s * E;
            if (mode == 1 && n_commit > 0) break;
            int conflict = 0;
            for (int c = 0; c < 2 * n_commit && !conflict; ++c)
                conflict = near_or_equal(lattice, L, n_off, off, committed[c], t->p) ||
                           near_or_equal(lattice, L, n_off, off, committed[c], t->q);
            if (conflict) continue;
            double dS = t->dS;
            if (n_commit > 0) {
                dS = delta_objective(M, S, counts, dN, R, target, weight, sq);
                if (!(dS < -tau)) continue;
            }
            /* commit: swap species, update counts and the cached squared deviations */
            species[t->p] = (int8_t)t->b;
            species[t->q] = (int8_t)t->a;
            for (int e = 0; e < E; ++e) counts[e] += dN[e];
            for (int k = 0; k < S; ++k)
                for (int e = k * M * M; e < (k + 1) * M * M; ++e)
                    sq[e] = sq_dev(counts[e], R[e], target[e]);
            if (log && stats->commits < log_cap) {
                uint32_t *rec = log + 4 * stats->commits;
                rec[0] = (uint32_t)step;
                rec[1] = (uint32_t)s;
                rec[2] = (uint32_t)t->p;
                rec[3] = (uint32_t)t->q;
            }
            stats->commits++;
            committed[2 * n_commit] = t->p;
            committed[2 * n_commit + 1] = t->q;
            ++n_commit;
        }
        ++step;
        depth = n_commit > 0 ? 0 : depth + 1;
        if (depth_limit > 0 && depth >= depth_limit) {
            stats->stop_reason = 1;
            break;
        }
    }
    stats->steps = step;
    stats->log_len = log ? (stats->commits < log_cap ? stats->commits : log_cap) : 0;
    /* report from a fresh recount (the maintained counts go to counts_out) */
    int64_t *fresh = malloc(sizeof(int64_t) * E);
    or_counts(lattice, L, M, S, species, fresh);
    double SF[2];
    or_alpha_objective(lattice, L, M, S, species, fresh, target, weight, NULL, NULL, SF);
    stats->S = SF[0];
    stats->F = SF[1];
    if (counts_out) memcpy(counts_out, counts, sizeof(int64_t) * E);
    free(fresh);
    free(counts);
    free(dN_all);
    free(tr);
    free(order);
    free(committed);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* New solutions of the global search (Sec. 4.1, Algorithm 1): a random      */
/* arrangement of a fixed composition.  The paper does not say how a random  */
/* configuration is drawn; here position i of the composition-sorted list    */
/* (species j for c_0 + ... + c_{j-1} <= i < c_0 + ... + c_j) is placed on   */
/* site pi(i), pi a keyed permutation of [0, N):                             */
/*   * a balanced Feistel network on 2h-bit values (h the smallest h >= 1    */
/*     with 4^h >= N), four rounds; round r maps (L, R) to (R, L ^ f) with    */
/*     f = low h bits of word 0 of Philox4x32-10(counter = (R, r, slot,      */
/*     0x80000000 | iteration), key = seed);                                 */
/*   * cycle walking: the network is applied again until the value is < N   */
/*     (it is a permutation of [0, 4^h), so the orbit of i < N returns below */
/*     N, and the map restricted to [0, N) is a permutation).                */
/* ------------------------------------------------------------------------ */

static uint32_t feistel4(uint32_t x, int h, uint32_t slot, uint32_t iteration, const uint32_t *key) {
    const uint32_t mask = (1u << h) - 1u;
    uint32_t l = x >> h, r = x & mask;
    for (uint32_t round = 0; round < 4; ++round) {
        const uint32_t ctr[4] = {r, round, slot, 0x80000000u | iteration};
        uint32_t out[4];
        or_philox4x32_10(ctr, key, out);
        const uint32_t nl = r;
        r = l ^ (out[0] & mask);
        l = nl;
    }
    return (l << h) | r;
}

int or_random_config(int64_t N, int M, const int64_t *composition, uint64_t seed, uint32_t iteration,
                     uint32_t slot, int8_t *out) {
    int64_t total = 0;
    for (int j = 0; j < M; ++j) {
        if (composition[j] < 0) return 1;
        total += composition[j];
    }
    if (total != N || N < 1 || N > (int64_t)1 << 30) return 1;
    int h = 1;
    while (((int64_t)1 << (2 * h)) < N) ++h;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int j = 0;
    int64_t end = composition[0];
    for (int64_t i = 0; i < N; ++i) {
        while (i >= end) end += composition[++j];
        uint32_t x = feistel4((uint32_t)i, h, slot, iteration, key);
        while (x >= (uint64_t)N) x = feistel4(x, h, slot, iteration, key);
        out[x] = (int8_t)j;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Structures from other codes (the application workflow of Sec. 2.3, step  */
/* (3): a relaxed or MD structure is analysed for its SRO).  Each atom is    */
/* assigned to the lattice site nearest to it under periodic minimum-image  */
/* distances, by brute force over all sites; ties go to the lower site id.  */
/* box[3] are the Cartesian edge lengths of the orthorhombic supercell of   */
/* L[0] x L[1] x L[2] conventional cells (site half-unit position h maps to  */
/* h * box / (2 L)).  Returns 0, or 1 if n != number of sites, 2 if some     */
/* atom lies farther than max_disp from every site, 3 if two atoms share a   */
/* site, 4 if a type lies outside [0, M).  species_out[site] = types[atom],  */
/* site_out[atom] = its site.                                                */
/* ------------------------------------------------------------------------ */
int or_map_sites(int lattice, const int *L, int M, const double *box, double max_disp, int64_t n,
                 const double *xyz, const int8_t *types, int8_t *species_out, int64_t *site_out) {
    const int64_t N = or_n_sites(lattice, L);
    if (n != N) return 1;
    int64_t *owner = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    if (!owner) return 5;
    for (int64_t p = 0; p < N; ++p) owner[p] = -1;
    int rc = 0;
    for (int64_t a = 0; a < n && rc == 0; ++a) {
        if (types[a] < 0 || types[a] >= M) {
            rc = 4;
            break;
        }
        int64_t best = -1;
        double best_d2 = 0.0;
        for (int64_t p = 0; p < N; ++p) {
            int pos[3];
            or_site_pos(lattice, L, p, pos);
            double d2 = 0.0;
            for (int ax = 0; ax < 3; ++ax) {
                const double site = (double)pos[ax] * box[ax] / (double)(2 * L[ax]);
                double d = xyz[3 * a + ax] - site;
                d -= box[ax] * floor(d / box[ax] + 0.5); /* minimum image */
                d2 += d * d;
            }
            if (best < 0 || d2 < best_d2) {
                best = p;
                best_d2 = d2;
            }
        }
        if (best_d2 > max_disp * max_disp) {
            rc = 2;
            break;
        }
        if (owner[best] >= 0) {
            rc = 3;
            break;
        }
        owner[best] = a;
        site_out[a] = best;
    }
    if (rc == 0)
        for (int64_t p = 0; p < N; ++p) species_out[p] = types[owner[p]];
    free(owner);
    return rc;
}
