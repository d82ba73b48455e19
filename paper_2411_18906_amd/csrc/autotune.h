// Launch-shape tuning for the MC kernels.  A variant only changes where a
// chain's configuration lives and how launches are shaped, never the
// trajectory: every variant gives bit-identical results.
#pragma once

#include "geometry.h"

namespace pyhea {

// Launch shape of one chain: where its configuration lives (LDS bytes, LDS
// nibbles or HBM) and how many wavefronts share each shell (H = 1 or 2).
struct LaunchShape {
    int store;
    int H;
    int lds;
};

// Variants: 0 = automatic (LDS bytes when they fit, else nibbles, else HBM;
// two wavefronts per shell when the block and LDS allow); 1 = LDS nibbles when
// they fit, else HBM; 2 = always HBM; 3 = automatic store, one wavefront per
// shell.  Every variant gives bit-identical results.
constexpr int kNumStoreVariants = 4;

LaunchShape choose_launch(const Geometry &g, int B, int lds_budget, int variant);

// Variant forced through pyhea_tune_force (-1 = none).
int forced_variant();
void set_forced_variant(int v);
// Full-evaluation kernel forced through pyhea_tune_force_eval (-1 = automatic,
// 0 = gather, 1 = bit-sliced).
int forced_eval_kernel();
void set_forced_eval_kernel(int v);
const char *tune_cache_path();
void set_tune_cache_path(const char *p);

}  // namespace pyhea
