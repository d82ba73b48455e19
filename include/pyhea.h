/*
 * pyhea.h - C ABI of the MI355X (gfx950) library for Warren-Cowley
 * short-range-order (SRO) evaluation and SRO-targeted Monte Carlo structure
 * search, after Niu & Liu, "Short-Range Order Based Ultra Fast Large-Scale
 * Modeling of High-Entropy Alloys" (arXiv:2411.18906).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns a pyhea_status (0 = OK, negative = error) and never
 *    throws.  After an error, pyhea_last_error() returns a message for the
 *    calling thread.
 *  - "_dev" pointers are device (HBM) pointers on the current HIP device, e.g.
 *    torch tensor data_ptr(); "_host" pointers are ordinary host memory.  The
 *    caller owns every buffer it passes; the library keeps no pointer after a
 *    call returns, except the serving API, which copies its inputs.
 *  - `stream` is a hipStream_t (NULL = the default stream); work is ordered on
 *    it.  Calls that return results in host memory synchronise that stream.
 *  - Geometry: a supercell of L[0] x L[1] x L[2] conventional cubic cells of an
 *    FCC (4 sites per cell) or BCC (2 sites per cell) lattice, S = A L^3 sites
 *    (Sec. 2.2, Table 1 caption).  Positions are in half lattice constants:
 *    FCC sites 2c + {(0,0,0),(1,1,0),(1,0,1),(0,1,1)}, BCC 2c + {(0,0,0),(1,1,1)}.
 *    Site id p = ((cz*L[1] + cy)*L[0] + cx)*A + b.  Boundaries are periodic.
 *  - Coordination shell k (k = 1..4) is the set of lattice vectors of the k-th
 *    smallest length: FCC z = 12, 6, 24, 12; BCC z = 8, 6, 12, 24.  Pairs are
 *    counted once per (site, offset), so on cells two cells wide a neighbour
 *    reachable along two offsets counts twice.
 *  - Configurations are int8 species ids in [0, M), one byte per site.
 *  - Pair counts N[k][i][j] = #{(p, d): d in shell k, s_p = i, s_{p+d} = j}
 *    (ordered and symmetric).  alpha and the objective follow Eq. 2-3 in IEEE
 *    binary64 with no fused multiply-add:
 *        R     = (double)N_sites / (double)(n_i * n_j * z_k)
 *        alpha = 1 - N[k][i][j] * R           (P_ij = N_ij/(n_i z_k), c_j = n_j/N)
 *        Q_k   = sum_i (sum_j (alpha - target)^2),   S = sum_k w_k Q_k,
 *        (each sum from +0.0 in increasing index order)
 *        F     = sqrt(S)                      (Eq. 3: F is the fitness)
 *  - Limits: M in [2, 8]; S in [1, 4]; N_sites * max z_k < 2^31; no shell
 *    offset may map a site onto itself (PYHEA_EINVAL otherwise).
 */
#ifndef PYHEA_H
#define PYHEA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pyhea_status;
#define PYHEA_OK 0
#define PYHEA_EINVAL (-1)     /* malformed descriptor or input data            */
#define PYHEA_ENOMEM (-2)     /* device allocation failed / over HBM budget    */
#define PYHEA_EDEVICE (-3)    /* a HIP runtime call failed                     */
#define PYHEA_EBUSY (-4)      /* serving: job not finished yet                 */
#define PYHEA_ECANCELLED (-5) /* serving: job cancelled                        */
#define PYHEA_ENOSYS (-6)     /* not supported by this library                 */
#define PYHEA_ENOENT (-7)     /* serving: unknown job id                       */

#define PYHEA_FCC 0
#define PYHEA_BCC 1

#define PYHEA_MODE_DISJOINT 0 /* commit every non-conflicting improving swap   */
#define PYHEA_MODE_BEST 1     /* commit only the best swap of a step (Eq. 6)   */

#define PYHEA_STOP_TRIALS 0 /* the trial budget was used up                    */
#define PYHEA_STOP_DEPTH 1  /* depth_limit steps in a row committed nothing    */

/* Problem geometry (Sec. 2.2: lattice type and supercell; Sec. 4.3: shells). */
typedef struct {
    int32_t lattice;   /* PYHEA_FCC or PYHEA_BCC                              */
    int32_t L[3];      /* conventional cells along x, y, z (each >= 1)        */
    int32_t n_species; /* M, 2..8                                             */
    int32_t n_shells;  /* S, 1..4                                             */
} pyhea_lattice;

/* Objective of Eq. 3 (Sec. 4.4): user-specified target alphas and weights. */
typedef struct {
    const double *target; /* host, [S][M][M] row-major                        */
    const double *weight; /* host, [S], each finite and >= 0                  */
} pyhea_objective;

/* Monte Carlo local search parameters (Sec. 4.2, Algorithm 3; Sec. 4.6). */
typedef struct {
    uint64_t seed;         /* Philox4x32-10 key = (lo32(seed), hi32(seed))         */
    uint32_t chain_id;     /* Philox counter word 2; independent streams per chain */
    int32_t cand_per_step; /* B, trial swaps evaluated per step ("tasks"), 1..256  */
    int64_t n_trials;      /* T, total trial swaps (the last step may be partial)  */
    int32_t commit_mode;   /* PYHEA_MODE_DISJOINT or PYHEA_MODE_BEST               */
    int32_t depth_limit;   /* stop after this many steps without a commit; 0 = off */
    double accept_tol;     /* tau: a trial swap is accepted iff dS < -tau.  tau = 0:
                              strict improvement; tau > 0: improvement by more
                              than tau; tau < 0: the threshold acceptance of
                              Algorithms 2-3 -- swaps that worsen S by less than
                              -tau are accepted too (null draws never are)       */
} pyhea_mc_params;

/* Per-chain results. */
typedef struct {
    int64_t trials;      /* trial swaps drawn                                  */
    int64_t null_trials; /* draws with equal species at both sites            */
    int64_t commits;     /* swaps applied                                      */
    int64_t steps;       /* steps run                                          */
    int32_t stop_reason; /* PYHEA_STOP_*                                       */
    int32_t status;      /* PYHEA_OK, or the chain's own error                 */
    double S;            /* objective of the final configuration               */
    double F;            /* sqrt(S), Eq. 3                                      */
    int64_t log_len;     /* accepted-swap records written (min(commits, cap))  */
    int32_t shape;       /* launch shape used: store (0 LDS bytes, 1 LDS nibbles,
                            2 HBM) * 10000 + steps per pass * 100 + commit chunk */
    int32_t shape_measured; /* 1 if that shape was chosen by measurement (this
                            call or an earlier one), 0 by the cost model      */
    int32_t graph;       /* 1 if the call's device work ran as a replay of the
                            graph recorded for its structure (pyhea_tune_graphs) */
} pyhea_mc_stats;

/* Global search parameters (Sec. 4.1, Algorithm 1; the parameter study of
 * Sec. 2.1 names the pool size, the global iterations, the tasks and the
 * search depth). */
typedef struct {
    int32_t n_solutions;   /* solutions in the pool, >= 1                          */
    int32_t iterations;    /* global iterations, >= 1                               */
    int32_t n_refine;      /* best solutions refined per iteration, 1..n_solutions  */
    int32_t pad;
    double discard_frac;   /* p_a in [0, 1]: share of the refined solutions dropped;
                              the best n_refine - ceil(p_a n_refine), at most
                              n_refine / 2, seed the next iteration                  */
    pyhea_mc_params local; /* local search of every refined solution: seed (also
                              keys the random solutions), cand_per_step ("tasks"),
                              n_trials (cap per refinement), commit_mode,
                              depth_limit ("search depth"), accept_tol; chain_id is
                              ignored (each refinement uses iteration *
                              n_solutions + pool slot)                              */
} pyhea_global_params;

/* Global search results. */
typedef struct {
    int64_t evaluations; /* full evaluations of pool solutions                   */
    int64_t trials;      /* trial swaps of all local searches                     */
    int64_t commits;     /* swaps applied by all local searches                   */
    double S;            /* objective of the best solution                        */
    double F;            /* sqrt(S) of the best solution                          */
} pyhea_global_stats;

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t pyhea_version(void);

/* Message describing the last error on the calling thread ("" if none). */
const char *pyhea_last_error(void);

/*
 * Full SRO evaluation of one configuration (Sec. 4.3, Eq. 2; Sec. 4.4, Eq. 3).
 *   species_dev  [N] int8, device.
 *   obj          may be NULL: then alpha is still computed, S_F_host untouched.
 *   counts_host  [S][M][M] int64 (may be NULL).
 *   alpha_host   [S][M][M] double (may be NULL).
 *   S_F_host     [2] = {S, F} (ignored when obj is NULL).
 * Counts, alpha, S and F are computed on the device (one counting launch and
 * one objective launch on `stream`), then read back in one copy.
 * Synchronous.  PYHEA_EINVAL if a species id is outside [0, M) or some
 * species is absent (c_j = 0 leaves Eq. 2 undefined).
 */
pyhea_status pyhea_sro_eval(const pyhea_lattice *lat, const int8_t *species_dev,
                            const pyhea_objective *obj, int64_t *counts_host, double *alpha_host,
                            double *S_F_host, void *stream);

/*
 * Full SRO evaluation of K configurations of one geometry in one launch
 * (the fitness evaluation of a solution pool, Algorithm 1).
 *   species_dev  [K][N] int8, device.
 *   counts_dev   [K][S][M][M] int32, device, overwritten.
 *   obj, S_F_dev optional (both or neither): S_F_dev [K][2] double, device;
 *                a configuration with an invalid or absent species gets
 *                {NaN, NaN}.
 * Asynchronous on `stream`.
 */
pyhea_status pyhea_sro_eval_batch(const pyhea_lattice *lat, int64_t n_configs,
                                  const int8_t *species_dev, const pyhea_objective *obj,
                                  int32_t *counts_dev, double *S_F_dev, void *stream);

/*
 * pyhea_sro_eval_batch for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and asynchrony as pyhea_sro_eval_batch;
 * the call allocates nothing (no hipMalloc, hipFree or pool allocation).  Its
 * scratch (per-configuration flags, the target table, partial sums of
 * configurations that span several workgroups) lives in one fixed 16 MiB
 * device array per GPU, held until the process ends; the caller still owns
 * species_dev, counts_dev and S_F_dev.  PYHEA_EINVAL (with a message giving
 * the bytes needed) when n_configs needs more scratch than the array holds --
 * about 4 million configurations of one workgroup each, fewer for
 * configurations split across workgroups.  Calls that overlap on one GPU
 * share the array and race: order them on one stream.
 */
pyhea_status pyhea_sro_eval_batch_noalloc(const pyhea_lattice *lat, int64_t n_configs,
                                          const int8_t *species_dev, const pyhea_objective *obj,
                                          int32_t *counts_dev, double *S_F_dev, void *stream);

/*
 * Nearest-site assignment of a structure from another code (the analysis step
 * of the application workflow, Sec. 2.3: a configuration relaxed or simulated
 * by LAMMPS or DFT is read back onto the lattice so that its SRO can be
 * evaluated with pyhea_sro_eval and used as a target).  Each atom goes to the
 * lattice site nearest to it in the Cartesian metric under periodic minimum
 * images; site half-unit position h lies at h * box / (2 L) per axis.
 *   box_host          [3] edge lengths of the orthorhombic supercell of
 *                     L[0] x L[1] x L[2] conventional cells (same unit as xyz).
 *   max_disp          largest accepted distance of an atom from its site.
 *   n_atoms           must equal the number of sites N.
 *   xyz_dev           [n_atoms][3] double Cartesian positions (any periodic
 *                     image), device.
 *   types_dev         [n_atoms] int8 species ids in [0, M), device.
 *   species_dev       [N] int8 out: the species on each site, device.
 *   atom_of_site_dev  [N] int32 out: the atom on each site, or NULL.
 * Synchronous.  PYHEA_EINVAL when n_atoms != N, an atom lies farther than
 * max_disp from every site, two atoms are nearest to one site (a vacancy
 * elsewhere), or a type lies outside [0, M); the message says which.  Exact
 * ties between two sites (an atom equidistant from both) are resolved by the
 * decoding order, not by site id.
 */
pyhea_status pyhea_map_sites(const pyhea_lattice *lat, const double *box_host, double max_disp,
                             int64_t n_atoms, const double *xyz_dev, const int8_t *types_dev,
                             int8_t *species_dev, int32_t *atom_of_site_dev, void *stream);

/*
 * Incremental evaluation of trial swaps against one configuration (Sec. 4.5,
 * Eq. 4; Sec. 4.6.2, Eq. 5): for each pair (p, q) the count change dN of the
 * swap and dS = S(after) - S(before) in the contract above, without applying
 * the swap.  A pair with equal species gives dS = 0 and dN = 0.
 *   pairs_dev  [n][2] int32 site ids, device.
 *   dS_dev     [n] double, device.
 *   dN_dev     [n][S][M][M] int32, device, or NULL.
 * Asynchronous on `stream`.
 */
pyhea_status pyhea_trial_eval(const pyhea_lattice *lat, const pyhea_objective *obj,
                              const int8_t *species_dev, int64_t n_pairs, const int32_t *pairs_dev,
                              double *dS_dev, int32_t *dN_dev, void *stream);

/*
 * Non-incremental baseline of the same quantity (Sec. 4.5: the full
 * recalculation that Eq. 4 replaces): for each pair (p, q), dS = S(after) -
 * S(before), each S from a full evaluation (Eq. 2-3) -- of the configuration,
 * and of a copy with sites p and q swapped.  A pair with equal species gives
 * dS = 0.  Not bitwise equal to pyhea_trial_eval (a different summation).
 *   pairs_dev  [n][2] int32 site ids in [0, N), device.
 *   dS_dev     [n] double, device.
 * Device scratch of up to 256 MB of swapped copies per call.  Synchronous.
 */
pyhea_status pyhea_trial_eval_full(const pyhea_lattice *lat, const pyhea_objective *obj,
                                   const int8_t *species_dev, int64_t n_pairs, const int32_t *pairs_dev,
                                   double *dS_dev, void *stream);

/*
 * One Monte Carlo chain (Sec. 4.2, Algorithms 2-3; Sec. 4.6), run as one
 * persistent kernel.  Every step draws B trial swaps from Philox4x32-10 with
 * counter (slot, step, chain_id, 0): p = (x0 * N) >> 32, q = (x1 * N) >> 32;
 * all are evaluated against the same configuration; improving swaps
 * (dS < -tau) are ranked by (dS, slot) and committed by the commit mode:
 * BEST commits the first; DISJOINT walks the ranking and commits every swap
 * whose sites are not equal to, nor in shells 1..S of, a site already
 * committed in the step, re-checking its dS against the updated state.
 *   species_dev  [N] int8, device; initial configuration in, final out.
 *   log_dev      [log_cap][4] uint32 (step, slot, p, q) per commit, device,
 *                or NULL.
 *   counts_host  [S][M][M] int64 final pair counts, or NULL.
 * Synchronous.
 */
pyhea_status pyhea_mc_run(const pyhea_lattice *lat, const pyhea_objective *obj,
                          const pyhea_mc_params *params, int8_t *species_dev, uint32_t *log_dev,
                          int64_t log_cap, pyhea_mc_stats *stats_host, int64_t *counts_host,
                          void *stream);

/*
 * Many independent chains of uneven geometry in one persistent launch
 * (Sec. 4.6.1: one workgroup per candidate solution).  Arrays of length
 * n_chains describe each chain; chain c owns species_dev[offsets_host[c] ..
 * offsets_host[c+1]) and, if log_dev is not NULL, the records
 * log_dev[log_offsets_host[c] .. log_offsets_host[c+1]).  Each chain's
 * result is identical to pyhea_mc_run with the same inputs.  Launch shape is
 * chosen by the autotuner (pyhea_tune_*), never the trajectory.  The call
 * uploads its descriptors once and reads results back once; the species
 * totals and ratio tables are formed on the device from the initial counts.
 * A chain with an id outside [0, M) or an absent species makes the call
 * return PYHEA_EINVAL (the message names the first such chain); such chains
 * are left unchanged with stats status PYHEA_EINVAL, and the valid chains
 * still run to completion with status PYHEA_OK.
 * Synchronous.
 */
pyhea_status pyhea_mc_batch(int32_t n_chains, const pyhea_lattice *lats,
                            const pyhea_objective *objs, const pyhea_mc_params *params,
                            int8_t *species_dev, const int64_t *offsets_host, uint32_t *log_dev,
                            const int64_t *log_offsets_host, pyhea_mc_stats *stats_host,
                            void *stream);

/*
 * Serving: a continuous-batching job server.  Jobs are single chains
 * (pyhea_mc_run semantics, chain_id = job id); a worker thread admits queued
 * jobs while free slots and the HBM budget allow, keeps their configurations
 * and count tables resident on the device, advances all resident jobs in
 * rounds of one persistent launch per launch shape (the shapes on up to 16
 * streams, which overlap as far as the HIP runtime's hardware queues allow:
 * GPU_MAX_HW_QUEUES, 4 by default), and retires finished jobs as they end, so
 * jobs that arrive while others run join the next round.
 *   hbm_budget_bytes  device bytes the resident jobs may hold in total.
 *   max_slots         jobs resident at once.
 *   steps_per_round   MC steps per round of the launch shape whose chains take
 *                     longest per step (0 = library default, 256); the other
 *                     shapes run as many steps as their measured time per step
 *                     fits in the same time, at most 16 times as many.  A
 *                     job's result does not depend on where rounds cut it.
 */
pyhea_status pyhea_serve_open(int64_t hbm_budget_bytes, int32_t max_slots,
                              int32_t steps_per_round, void **server);

/* Queue a job.  Inputs are copied; species_host is [N] int8.  The job's
 * params->chain_id is replaced by job_id.  PYHEA_EINVAL for a malformed job or
 * one that can never fit the HBM budget; duplicate ids are rejected. */
pyhea_status pyhea_serve_submit(void *server, uint64_t job_id, const pyhea_lattice *lat,
                                const pyhea_objective *obj, const pyhea_mc_params *params,
                                const int8_t *species_host);

/* Result of a finished job: species_out_host [N] int8 (or NULL) and stats.
 * blocking = 0 returns PYHEA_EBUSY while the job runs; otherwise waits.
 * times_ns_host (or NULL) receives {submit, admit, finish} on a monotonic
 * clock.  A polled job is forgotten. */
pyhea_status pyhea_serve_poll(void *server, uint64_t job_id, int8_t *species_out_host,
                              pyhea_mc_stats *stats_host, int64_t *times_ns_host,
                              int32_t blocking);

/* Cancel a queued or running job (its poll then returns PYHEA_ECANCELLED). */
pyhea_status pyhea_serve_cancel(void *server, uint64_t job_id);

/* Server counters: {submitted, admitted, finished, rejected, resident, queued,
 * rounds, bytes_resident}. */
pyhea_status pyhea_serve_counters(void *server, int64_t *out8_host);

/* Stop the worker, end unfinished jobs as cancelled (a poll blocked on one
 * returns PYHEA_EDEVICE; close waits for it to leave) and free the server.
 * No call may use the handle after close has started. */
pyhea_status pyhea_serve_close(void *server);

/*
 * Global search (Sec. 4.1, Algorithm 1).  Iteration t: solutions without a
 * retained seed are drawn at random (pyhea_random_configs with iteration t);
 * every pool solution is evaluated in full (Eq. 3); the n_refine best (by F,
 * then pool slot) are refined by the Monte Carlo local search of
 * pyhea_mc_batch; the refined ones are ranked by their final F (then by their
 * rank before refinement), the worst fraction p_a is dropped and the best
 * retained ones move to pool slots 0.. as the next iteration's seeds; the best
 * solution so far is replaced only by a strictly lower F.
 *   composition_host  [M] species counts, host; each >= 1, summing to N.
 *   best_dev          [N] int8, device: the best solution found.
 *   history_host      [iterations] best F after each iteration, host, or NULL.
 *   stats_host        results, host.
 * Device memory for the pool is allocated per call.  Synchronous.
 */
pyhea_status pyhea_global_search(const pyhea_lattice *lat, const pyhea_objective *obj,
                                 const int64_t *composition_host, const pyhea_global_params *params,
                                 int8_t *best_dev, double *history_host, pyhea_global_stats *stats_host,
                                 void *stream);

/*
 * Random solutions of the global search (Sec. 4.1: new candidate
 * configurations; the paper does not say how they are drawn).  Configuration
 * c (0 <= c < n_configs) is pool slot slot0 + c of iteration `iteration`: the
 * species list sorted by species (composition_host[j] copies of j) placed on
 * the sites through a keyed permutation -- a four-round Feistel network on
 * 2h-bit values (4^h >= N), round r XOR-ing the low h bits of word 0 of
 * Philox4x32-10(counter = (right half, r, slot, 0x80000000 | iteration), key =
 * seed) into the left half, re-applied until the value is below N.
 *   out_dev  [n_configs][N] int8, device.  Asynchronous.
 */
pyhea_status pyhea_random_configs(int64_t N, int32_t M, const int64_t *composition_host, uint64_t seed,
                                  uint32_t iteration, uint32_t slot0, int32_t n_configs, int8_t *out_dev,
                                  void *stream);

/* Philox4x32-10 (Salmon et al., SC'11) on the device, for checking the
 * library's trial draws: out[i] = philox(ctr[i], key = (lo32(seed), hi32(seed))).
 * ctr_dev and out_dev are [n][4] uint32, device.  Asynchronous. */
pyhea_status pyhea_philox4x32_10(const uint32_t *ctr_dev, uint64_t seed, int64_t n,
                                 uint32_t *out_dev, void *stream);

/* Launch shape of the MC kernels.  The library picks it from the chain's
 * size and the number of chains launched together: of the stores (LDS bytes,
 * LDS nibbles, HBM), steps per pass and speculative commit chunks that fit the
 * LDS, the combination with the best measured rate, one wavefront per shell,
 * and a block small enough that every chain of the call can be resident.
 * This switch forces one shape family process-wide: -1 = automatic, 0 =
 * automatic, 1 = LDS nibbles or HBM, 2 = HBM, 3 = automatic, 4 = offsets
 * spread evenly over the shell wavefronts, 5 = DISJOINT commits decided one by
 * one, 6 = speculative commit chunks of 4 candidates.  Shapes never change
 * results; EINVAL outside -1..6. */
pyhea_status pyhea_tune_force(int32_t variant);

/* Measuring autotuner for the automatic launch shape of single chains
 * (pyhea_mc_run; on by default): the first chain of a kind -- device, lattice,
 * M, S, B, floor(log2 padded sites) -- is counted on a scratch copy, run past
 * its first steps, and from that saved state run again under each candidate
 * shape (per store that fits: the most steps per pass the wave budget allows,
 * about half of that and one, each with the largest commit chunk that fits
 * and with commits one by one, and the cost model's own shape) for two
 * lengths, whose time difference (median of three) is the per-step cost; the
 * cost model's shape is kept unless another is at least 3 % cheaper per step,
 * and the choice is kept in memory and in the text file
 * named by PYHEA_TUNE_CACHE (else $HOME/.cache/pyhea/mc_launch_shapes.txt) for
 * later calls and processes (the server reads it too).  Batches use the cost
 * model, which was fitted to batches.  on = 0 uses the cost model alone.
 * The shape used is reported in pyhea_mc_stats.  Shapes never change results. */
pyhea_status pyhea_tune_measure(int32_t on);

/* Recorded device work of chain calls (pyhea_mc_run, pyhea_mc_batch; on by
 * default).  A call's device work -- the zeroed result block, the initial
 * counts, the ratio tables, the chain launches on up to four streams, the
 * final objective and the recount -- depends only on its structure: the
 * chains' geometries and launch shapes, which fix the device buffer layout.
 * The second call of a structure records that work as a hipGraph on a buffer
 * the library keeps, and it and later calls of the structure upload their
 * descriptors (seeds, trial counts, species and log pointers, targets) and
 * replay the graph: one launch instead of about ten, and no stream forks.  At
 * most 32 structures are recorded per process, each keeping its device
 * buffer (descriptors, counts, ratio tables, padded copies of HBM-store
 * chains) until the process ends; calls of other structures run eagerly.
 * Calls of one structure from several threads take turns.  Results never
 * depend on this.  on = 0 runs every call eagerly. */
pyhea_status pyhea_tune_graphs(int32_t on);

/* Full-evaluation kernel: -1 = automatic (bit-sliced where it covers the
 * geometry, else gather), 0 = gather, 1 = bit-sliced where possible (a
 * configuration whose layers would take more than half of a CU's LDS is cut
 * along z so that two workgroups share each CU), 2 = bit-sliced without that
 * cut, 3 = bit-sliced cut for four workgroups per CU, 4 = streaming where it
 * covers the geometry (persistent workgroups walk whole configurations along
 * z while the next layers load).  All give identical counts. */
pyhea_status pyhea_tune_force_eval(int32_t kernel);

/* Launch shape of the streaming evaluation: centre layers per group (0 =
 * automatic, else 1..8) and workgroup size (0 = automatic, 256 or 512).
 * Process-wide; shapes never change results; EINVAL outside those values. */
pyhea_status pyhea_tune_force_stream(int32_t layers_per_group, int32_t threads);

/* Steps whose candidates one pass of the MC kernel evaluates at once: 0 =
 * automatic (the largest value up to 8 whose block still lets every chain of
 * the call, or every slot of a server, be resident on the GPU at once), or
 * 1..8 (capped so that a block has at most 16 wavefronts).  Candidates are
 * drawn from counters, not from the state, so the candidates of later steps
 * can be evaluated against the current state; a
 * step's evaluation is used only if every earlier step of the pass committed
 * nothing (the state is then unchanged).  Trajectories are bit-identical for
 * every value.  Process-wide; EINVAL outside 0..8. */
pyhea_status pyhea_tune_force_lookahead(int32_t steps);

#ifdef __cplusplus
}
#endif

#endif /* PYHEA_H */
