// Launch-shape tuning for the MC kernels (see autotune.h).
#include "autotune.h"

#include <algorithm>
#include <mutex>
#include <string>

#include "mc_kernels.h"

namespace pyhea {

namespace {
std::mutex g_mu;
int g_forced = -1;
int g_forced_eval = -1;
int g_stream_G = 0, g_stream_threads = 0;
int g_forced_lookahead = 0;
}  // namespace

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
