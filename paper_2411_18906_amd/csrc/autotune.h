// Launch-shape tuning for the MC kernels.  A variant only changes where a
// chain's configuration lives and how launches are shaped, never the
// trajectory: every variant gives bit-identical results.
#pragma once

#include <vector>

#include "geometry.h"

namespace pyhea {

// Launch shape of one chain: where its configuration lives (LDS bytes, LDS
// nibbles or HBM), the wavefronts per slot group (W) and whether the offsets
// are spread evenly over them (bal), and how many steps one pass evaluates
// (K, 1..kMaxLookahead).
struct LaunchShape {
    int store;
    int W;
    int bal;
    int K;
    int CH;   // speculative commit chunk (0: commits one by one)
    int lds;
};

// Variants: 0 = automatic (of LDS bytes, LDS nibbles and HBM, the store whose
// room for steps per pass gives the best measured rate; each wavefront gathers
// its own shell's offsets); 1 = LDS nibbles or HBM, chosen the same way; 2 =
// always HBM; 3 = the automatic shape (kept as an explicit
// name); 4 = automatic store, every wavefront of a slot group gathers an equal
// share of all offsets and the shells' partial histograms meet in LDS;
// 5 = the automatic shape with DISJOINT commits decided one by one; 6 = the
// automatic shape with speculative commit chunks of 4.  The block size follows the
// number of chains launched together (n_chains) so that all can be resident;
// the steps per pass are the largest (up to 8) that fit it and the store, unless
// forced.
// Every variant gives bit-identical results.
constexpr int kNumStoreVariants = 7;

LaunchShape choose_launch(const Geometry &g, int B, int lds_budget, int variant, int n_chains);
int wave_budget(int n_chains);

// Candidate shapes for measurement: for each store that fits, the most steps
// per pass the wave budget allows, about half of that and one step, each with
// the largest commit chunk that fits and with commits one by one.
std::vector<LaunchShape> candidate_launches(const Geometry &g, int B, int lds_budget, int n_chains);
// LDS bytes of shape s for a chain of geometry g (the species store depends on
// the padded size).
int64_t launch_lds_bytes(const Geometry &g, int B, const LaunchShape &s);

// Measured launch shapes.  Key: device (architecture, CU count), lattice, M,
// S, B, floor(log2 padded sites) and the wave budget of the call's residency
// class.  Kept in memory and appended to a text file (PYHEA_TUNE_CACHE, else
// $HOME/.cache/pyhea/mc_launch_shapes.txt) that later processes read.
struct TuneKey {
    int lattice, M, S, B, nbucket, budget;
};
TuneKey tune_key(const Geometry &g, int B, int n_chains);
bool tuned_launch(const TuneKey &k, LaunchShape *s);
void record_tuned_launch(const TuneKey &k, const LaunchShape &s, double us_per_step);
// Whether automatic shapes are measured (pyhea_tune_measure; on by default).
bool measure_enabled();
void set_measure_enabled(bool on);
// Whether repeated chain calls of one structure replay a recorded graph
// (pyhea_tune_graphs; on by default).
bool graphs_enabled();
void set_graphs_enabled(bool on);
// Encoded launch shape reported in the chain statistics:
// store * 10000 + steps per pass * 100 + commit chunk.
inline int32_t shape_code(const LaunchShape &s) { return s.store * 10000 + s.K * 100 + s.CH; }

// Variant forced through pyhea_tune_force (-1 = none).
int forced_variant();
void set_forced_variant(int v);
// Full-evaluation kernel forced through pyhea_tune_force_eval (-1 = automatic,
// 0 = gather, 1-3 = bit-sliced, 4 = streaming).
int forced_eval_kernel();
void set_forced_eval_kernel(int v);
// Streaming evaluation shape forced through pyhea_tune_force_stream (0 = automatic).
void forced_stream_shape(int *layers_per_group, int *threads);
void set_forced_stream_shape(int layers_per_group, int threads);
// Steps per pass forced through pyhea_tune_force_lookahead (0 = automatic).
int forced_lookahead();
void set_forced_lookahead(int k);

}  // namespace pyhea
