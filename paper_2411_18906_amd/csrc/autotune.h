// Launch-shape tuning for the MC kernels.  A variant only changes where a
// chain's configuration lives and how launches are shaped, never the
// trajectory: every variant gives bit-identical results.
#pragma once

#include "geometry.h"

namespace pyhea {

// Variants: 0 = LDS bytes when they fit, else LDS nibbles, else HBM (default);
// 1 = LDS nibbles when they fit, else HBM; 2 = always HBM.
constexpr int kNumStoreVariants = 3;

int tune_store_override(int variant, int default_store, const Geometry &g, int B, int lds_budget,
                        int *lds_bytes);

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
