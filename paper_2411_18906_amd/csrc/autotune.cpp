// Launch-shape tuning for the MC kernels (see autotune.h).
#include "autotune.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <sys/stat.h>

#include "mc_kernels.h"

namespace pyhea {

namespace {
std::mutex g_mu;
int g_forced = -1;
int g_forced_eval = -1;
int g_stream_G = 0, g_stream_threads = 0;
int g_forced_lookahead = 0;
bool g_measure = true;
bool g_graphs = true;

// measured shapes by key string; loaded from the cache file on first use
std::mutex g_tune_mu;
bool g_tune_loaded = false;
std::map<std::string, LaunchShape> g_tuned;

std::string device_tag() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    return arch + "x" + std::to_string(prop.multiProcessorCount);
}

std::string key_string(const TuneKey &k) {
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%s/%d/%d/%d/%d/%d/%d", device_tag().c_str(), k.lattice, k.M, k.S, k.B,
                  k.nbucket, k.budget);
    return buf;
}

std::string cache_path() {
    if (const char *p = std::getenv("PYHEA_TUNE_CACHE")) return p;
    const char *home = std::getenv("HOME");
    if (!home || !*home) return "";
    return std::string(home) + "/.cache/pyhea/mc_launch_shapes.txt";
}

// lines: key store W bal K CH us_per_step (later lines override earlier ones)
void load_cache_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const std::string path = cache_path();
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char key[160];
    LaunchShape s{};
    double us = 0.0;
    while (std::fscanf(f, "%159s %d %d %d %d %d %lf", key, &s.store, &s.W, &s.bal, &s.K, &s.CH, &us) == 7) {
        if (s.store < 0 || s.store > 2 || s.K < 1 || s.K > kMaxLookahead || s.W < 1 || s.CH < 0) continue;
        s.lds = 0;
        g_tuned[key] = s;
    }
    std::fclose(f);
}
}  // namespace

std::vector<LaunchShape> candidate_launches(const Geometry &g, int B, int lds_budget, int n_chains) {
    std::vector<LaunchShape> out;
    const int Gs = (B + 63) / 64;
    const int W = g.S;
    const int budget = std::max(wave_budget(n_chains), g.S * Gs);
    const int kmax = std::max(1, std::min(kMaxLookahead, budget / (W * Gs)));
    const int E = g.S * g.M * g.M;
    const int chs[3] = {E <= 128 ? 16 : 8, 4, 0};
    int ks[3] = {kmax, (kmax + 1) / 2, 1};
    for (int store : {(int)kStoreLds8, (int)kStoreLds4, (int)kStoreGlobal}) {
        for (int ki = 0; ki < 3; ++ki) {
            const int K = ks[ki];
            if (ki > 0 && K == ks[ki - 1]) continue;
            if (mc_block_waves(B, W, K) > 16) continue;
            bool chunked = false;
            for (int CH : chs) {
                if (CH > 0 && chunked) continue;   // the largest chunk that fits, and none
                const int64_t lds = mc_lds_bytes(g.S, g.M, B, W, 0, K, CH) + species_store_bytes(store, g.Npad);
                if (lds > lds_budget) continue;
                if (CH > 0) chunked = true;
                out.push_back(LaunchShape{store, W, 0, K, CH, (int)lds});
            }
        }
    }
    return out;
}

int64_t launch_lds_bytes(const Geometry &g, int B, const LaunchShape &s) {
    return mc_lds_bytes(g.S, g.M, B, s.W, s.bal, s.K, s.CH) + species_store_bytes(s.store, g.Npad);
}

TuneKey tune_key(const Geometry &g, int B, int n_chains) {
    TuneKey k;
    k.lattice = g.lattice;
    k.M = g.M;
    k.S = g.S;
    k.B = B;
    k.nbucket = g.Npad > 0 ? (int)std::floor(std::log2((double)g.Npad)) : 0;
    k.budget = wave_budget(n_chains);
    return k;
}

bool tuned_launch(const TuneKey &k, LaunchShape *s) {
    const std::string key = key_string(k);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    auto it = g_tuned.find(key);
    if (it == g_tuned.end()) return false;
    *s = it->second;
    return true;
}

void record_tuned_launch(const TuneKey &k, const LaunchShape &s, double us_per_step) {
    const std::string key = key_string(k);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    g_tuned[key] = s;
    const std::string path = cache_path();
    if (path.empty()) return;
    // create the directory chain if needed (best effort; the cache is optional)
    for (size_t i = 1; i < path.size(); ++i)
        if (path[i] == '/') mkdir(path.substr(0, i).c_str(), 0755);
    if (FILE *f = std::fopen(path.c_str(), "a")) {
        std::fprintf(f, "%s %d %d %d %d %d %.4f\n", key.c_str(), s.store, s.W, s.bal, s.K, s.CH, us_per_step);
        std::fclose(f);
    }
}

bool measure_enabled() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_measure;
}

void set_measure_enabled(bool on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_measure = on;
}

bool graphs_enabled() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_graphs;
}

void set_graphs_enabled(bool on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_graphs = on;
}

int wave_budget(int n_chains) {
    // every chain of a launch should be resident at once: 256 CUs x 16 wavefronts
    const int n = n_chains < 1 ? 1 : n_chains;
    return n <= 256 ? 16 : (4096 / n < 1 ? 1 : 4096 / n);
}

LaunchShape choose_launch(const Geometry &g, int B, int lds_budget, int variant, int n_chains) {
    int stores[3], ns = 0;
    if (variant == 2) {
        stores[ns++] = kStoreGlobal;
    } else if (variant == 1) {
        stores[ns++] = kStoreLds4;
        stores[ns++] = kStoreGlobal;
    } else {
        stores[ns++] = kStoreLds8;
        stores[ns++] = kStoreLds4;
        stores[ns++] = kStoreGlobal;
    }
    const int Gs = (B + 63) / 64;
    const int fk = forced_lookahead();
    const int budget = std::max(fk > 0 ? 16 : wave_budget(n_chains), g.S * Gs);
    // one wavefront per shell (gathering its own shell, or with variant 4 an
    // equal share of all offsets), then as many steps per pass as the block allows
    const int W = g.S;
    const int bal = variant == 4 && g.S > 1 ? 1 : 0;
    const int kmax = fk > 0 ? fk : std::max(1, std::min(kMaxLookahead, budget / (W * Gs)));
    // speculative commit chunks: 16 members (8 when a member's table is large),
    // fewer or none when the LDS is short
    const int E = g.S * g.M * g.M;
    int chs[4] = {E <= 128 ? 16 : 8, E <= 128 ? 8 : 4, 4, 0};
    if (variant == 5) chs[0] = chs[1] = chs[2] = 0;   // commits one by one
    if (variant == 6) chs[0] = chs[1] = 4;            // small speculative chunks
    // every (store, steps per pass, commit chunk) that fits, scored by measured
    // rates: steps per pass 1..5 ran the FCC 20^3 chain 1, 1.75, 2.3, 2.75, 2.8
    // times as fast as one step (flat beyond); the configuration as LDS nibbles
    // / in HBM ran at 0.88 / 0.63 of LDS bytes at equal steps per pass; commit
    // chunks of 4 / commits one by one ran the 512 batched chains at 0.92 / 0.83
    // of chunks of 8-16
    static const double kgain[kMaxLookahead + 1] = {0.0, 1.0, 1.75, 2.3, 2.75, 2.8, 2.85, 2.85, 2.85};
    LaunchShape best{kStoreGlobal, W, 0, 1, 0, mc_lds_bytes(g.S, g.M, B, W, 0, 1, 0)};
    double best_score = -1.0;
    for (int si = 0; si < ns; ++si) {
        const double sf = stores[si] == kStoreLds8 ? 1.0 : stores[si] == kStoreLds4 ? 0.88 : 0.63;
        for (int K = kmax; K >= 1; --K) {
            if (mc_block_waves(B, W, K) > 16) continue;
            for (int CH : chs) {
                const double cf = CH >= 8 ? 1.0 : CH >= 4 ? 0.92 : 0.83;
                for (int bl : {bal, 0}) {
                    const int64_t lds =
                        mc_lds_bytes(g.S, g.M, B, W, bl, K, CH) + species_store_bytes(stores[si], g.Npad);
                    if (lds <= lds_budget) {
                        const double score = kgain[K] * sf * cf;
                        if (score > best_score) {
                            best_score = score;
                            best = LaunchShape{stores[si], W, bl, K, CH, (int)lds};
                        }
                        break;
                    }
                    if (bal == 0) break;
                }
            }
        }
    }
    return best;
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

void forced_stream_shape(int *layers_per_group, int *threads) {
    std::lock_guard<std::mutex> lk(g_mu);
    *layers_per_group = g_stream_G;
    *threads = g_stream_threads;
}

void set_forced_stream_shape(int layers_per_group, int threads) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_stream_G = layers_per_group;
    g_stream_threads = threads;
}

int forced_lookahead() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_forced_lookahead;
}

void set_forced_lookahead(int k) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_forced_lookahead = k;
}


}  // namespace pyhea
