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

LaunchShape choose_launch(const Geometry &g, int B, int lds_budget, int variant) {
    LaunchShape ls;
    const int fixed1 = mc_lds_bytes(g.S, g.M, B, 1);
    const int64_t b8 = fixed1 + species_store_bytes(kStoreLds8, g.Npad);
    const int64_t b4 = fixed1 + species_store_bytes(kStoreLds4, g.Npad);
    if (variant == 2) {
        ls.store = kStoreGlobal;
    } else if (variant == 1) {
        ls.store = b4 <= lds_budget ? kStoreLds4 : kStoreGlobal;
    } else {
        ls.store = b8 <= lds_budget ? kStoreLds8 : (b4 <= lds_budget ? kStoreLds4 : kStoreGlobal);
    }
    ls.H = 1;
    ls.lds = (int)(fixed1 + species_store_bytes(ls.store, g.Npad));
    if (variant != 3 && mc_halves(g.S, B) == 2) {
        const int64_t l2 = mc_lds_bytes(g.S, g.M, B, 2) + species_store_bytes(ls.store, g.Npad);
        if (l2 <= lds_budget) {
            ls.H = 2;
            ls.lds = (int)l2;
        }
    }
    return ls;
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
