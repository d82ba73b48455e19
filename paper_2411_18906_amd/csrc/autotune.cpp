// Launch-shape tuning for the MC kernels (see autotune.h).
#include "autotune.h"

#include <mutex>
#include <string>

#include "mc_kernels.h"

namespace pyhea {

namespace {
std::mutex g_mu;
int g_forced = -1;
int g_forced_eval = -1;
std::string g_cache;
}  // namespace

int tune_store_override(int variant, int default_store, const Geometry &g, int B, int lds_budget,
                        int *lds_bytes) {
    const int fixed = mc_lds_bytes(g.S, g.M, B);
    const int64_t b4 = fixed + species_store_bytes(kStoreLds4, g.Npad);
    if (variant == 1 && b4 <= lds_budget) {
        *lds_bytes = (int)b4;
        return kStoreLds4;
    }
    if (variant == 1 || variant == 2) {
        *lds_bytes = fixed;
        return kStoreGlobal;
    }
    return default_store;
}

int forced_variant() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_forced;
}

void set_forced_variant(int v) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_forced = v;
}

int forced_eval_kernel() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_forced_eval;
}

void set_forced_eval_kernel(int v) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_forced_eval = v;
}

const char *tune_cache_path() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_cache.c_str();
}

void set_tune_cache_path(const char *p) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache = p ? p : "";
}

}  // namespace pyhea
