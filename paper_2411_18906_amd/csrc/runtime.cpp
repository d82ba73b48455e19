// Host runtime of the pyhea library: validation, the binary64 objective
// contract on the host, and the chain driver behind pyhea_mc_run/pyhea_mc_batch.
#include "runtime.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

#include "autotune.h"
#include "sro_bits.h"

namespace pyhea {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const std::string &last_error() { return g_last_error; }

pyhea_status device_error(hipError_t e, const char *what) {
    set_error(std::string("HIP error in ") + what + ": " + hipGetErrorString(e));
    return PYHEA_EDEVICE;
}

int max_lds_per_block() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
    static int cached[64] = {0};
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
    int v = 64 * 1024;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) v = (int)prop.sharedMemPerBlock;
    if (dev >= 0 && dev < 64) cached[dev] = v;
    return v;
}

pyhea_status check_objective(const Geometry &g, const pyhea_objective *obj) {
    if (!obj || !obj->target || !obj->weight) {
        set_error("objective, target and weight must not be NULL");
        return PYHEA_EINVAL;
    }
    const int E = g.S * g.M * g.M;
    for (int e = 0; e < E; ++e)
        if (!std::isfinite(obj->target[e])) {
            set_error("target alphas must be finite");
            return PYHEA_EINVAL;
        }
    for (int k = 0; k < g.S; ++k)
        if (!std::isfinite(obj->weight[k]) || obj->weight[k] < 0.0) {
            set_error("shell weights must be finite and >= 0");
            return PYHEA_EINVAL;
        }
    return PYHEA_OK;
}

pyhea_status check_params(const pyhea_mc_params *p) {
    if (!p) {
        set_error("params must not be NULL");
        return PYHEA_EINVAL;
    }
    if (p->cand_per_step < 1 || p->cand_per_step > kMaxB) {
        set_error("cand_per_step must be in [1, 256]");
        return PYHEA_EINVAL;
    }
    if (p->n_trials < 0 || p->n_trials / p->cand_per_step >= (int64_t(1) << 32)) {
        set_error("n_trials must be >= 0 and n_trials / cand_per_step < 2^32");
        return PYHEA_EINVAL;
    }
    if (p->commit_mode != PYHEA_MODE_DISJOINT && p->commit_mode != PYHEA_MODE_BEST) {
        set_error("commit_mode must be PYHEA_MODE_DISJOINT or PYHEA_MODE_BEST");
        return PYHEA_EINVAL;
    }
    if (p->depth_limit < 0) {
        set_error("depth_limit must be >= 0");
        return PYHEA_EINVAL;
    }
    if (!std::isfinite(p->accept_tol) || p->accept_tol < 0.0) {
        set_error("accept_tol must be finite and >= 0");
        return PYHEA_EINVAL;
    }
    return PYHEA_OK;
}

bool species_totals(const Geometry &g, const int64_t *counts, int64_t *n) {
    bool ok = true;
    for (int i = 0; i < g.M; ++i) {
        int64_t r = 0;
        for (int j = 0; j < g.M; ++j) r += counts[i * g.M + j];
        n[i] = r / g.z[0];
        ok = ok && n[i] > 0;
    }
    return ok;
}

void ratio_table(const Geometry &g, const int64_t *n, double *R) {
    for (int k = 0; k < g.S; ++k)
        for (int i = 0; i < g.M; ++i)
            for (int j = 0; j < g.M; ++j)
                R[(k * g.M + i) * g.M + j] = (double)g.N / (double)(n[i] * n[j] * (int64_t)g.z[k]);
}

void host_objective(const Geometry &g, const int64_t *counts, const double *target,
                    const double *weight, double *alpha, double *S_F) {
    int64_t n[kMaxSpecies];
    species_totals(g, counts, n);
    std::vector<double> R(g.S * g.M * g.M);
    ratio_table(g, n, R.data());
    double sum = 0.0;
    for (int k = 0; k < g.S; ++k) {
        double Q = 0.0;
        for (int i = 0; i < g.M; ++i) {
            double row = 0.0;
            for (int j = 0; j < g.M; ++j) {
                const int e = (k * g.M + i) * g.M + j;
                const double a = 1.0 - (double)counts[e] * R[e];
                if (alpha) alpha[e] = a;
                if (target) {
                    const double d = a - target[e];
                    row = row + d * d;
                }
            }
            Q = Q + row;
        }
        if (weight) sum = sum + weight[k] * Q;
    }
    if (S_F) {
        S_F[0] = sum;
        S_F[1] = std::sqrt(sum);
    }
}

pyhea_status count_configs(const Geometry &g, int64_t K, const int8_t *species, int32_t *counts,
                           int32_t *bad, hipStream_t stream, const double *tw, double *S_F, bool *fused) {
    if (fused) *fused = false;
    if (K <= 0) return PYHEA_OK;
    const int forced = forced_eval_kernel();
    BitDesc bd;
    if (forced != 0 && fill_bit_desc(g, max_lds_per_block(), K, &bd)) {
        void *partial = nullptr;
        if (bd.nchunks > 1) PYHEA_HIP(hipMallocAsync(&partial, (size_t)K * bd.partial_stride * 4, stream));
        const bool fuse = S_F && bd.nchunks == 1;
        const hipError_t e = launch_count_bits(g, bd, K, species, (int32_t *)partial, counts, bad,
                                               fuse ? tw : nullptr, fuse ? S_F : nullptr, stream);
        if (partial) (void)hipFreeAsync(partial, stream);
        PYHEA_HIP(e);
        if (fused) *fused = fuse;
        return PYHEA_OK;
    }
    EvalDesc ed;
    fill_eval_desc(g, &ed);
    PYHEA_HIP(launch_count_gather(ed, K, species, counts, bad, stream));
    return PYHEA_OK;
}

namespace {

struct DeviceBuffer {
    void *ptr = nullptr;
    ~DeviceBuffer() {
        if (ptr) (void)hipFree(ptr);
    }
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

pyhea_status run_chains(std::vector<ChainJob> &jobs, pyhea_mc_stats *stats,
                        std::vector<std::vector<int64_t>> *final_counts, hipStream_t stream,
                        int variant) {
    const int n = (int)jobs.size();
    if (n == 0) return PYHEA_OK;
    const int lds_budget = max_lds_per_block();

    // device arena: per chain counts, recount, bad flag, R, target, state, padded copy
    struct Slot {
        size_t counts, recount, bad, R, target, state, pad;
        int store, lds, H;
    };
    std::vector<Slot> slot(n);
    size_t total = 0;
    for (int c = 0; c < n; ++c) {
        const Geometry &g = jobs[c].g;
        const size_t E = (size_t)g.S * g.M * g.M;
        Slot &s = slot[c];
        s.counts = total;
        total = align256(total + E * 4);
        s.recount = total;
        total = align256(total + E * 4);
        s.bad = total;
        total = align256(total + 4);
        s.R = total;
        total = align256(total + E * 8);
        s.target = total;
        total = align256(total + E * 8);
        s.state = total;
        total = align256(total + sizeof(ChainState));
        const LaunchShape ls = choose_launch(g, jobs[c].params.cand_per_step, lds_budget, variant < 0 ? 0 : variant);
        s.store = ls.store;
        s.lds = ls.lds;
        s.H = ls.H;
        s.pad = total;
        if (s.store == kStoreGlobal) total = align256(total + (size_t)g.Npad);
    }
    DeviceBuffer arena;
    PYHEA_HIP(hipMalloc(&arena.ptr, total));
    char *base = (char *)arena.ptr;

    // initial pair counts (full evaluation of each chain's configuration)
    std::vector<EvalDesc> eds(n);
    for (int c = 0; c < n; ++c) {
        fill_eval_desc(jobs[c].g, &eds[c]);
        const pyhea_status s = count_configs(jobs[c].g, 1, jobs[c].species_dev, (int32_t *)(base + slot[c].counts),
                                             (int32_t *)(base + slot[c].bad), stream);
        if (s != PYHEA_OK) return s;
    }
    std::vector<std::vector<int32_t>> cnt32(n);
    std::vector<int32_t> bad(n);
    for (int c = 0; c < n; ++c) {
        const Geometry &g = jobs[c].g;
        cnt32[c].resize((size_t)g.S * g.M * g.M);
        PYHEA_HIP(hipMemcpyAsync(cnt32[c].data(), base + slot[c].counts, cnt32[c].size() * 4,
                                 hipMemcpyDeviceToHost, stream));
        PYHEA_HIP(hipMemcpyAsync(&bad[c], base + slot[c].bad, 4, hipMemcpyDeviceToHost, stream));
    }
    PYHEA_HIP(hipStreamSynchronize(stream));

    std::vector<std::vector<double>> Rtab(n);
    for (int c = 0; c < n; ++c) {
        const Geometry &g = jobs[c].g;
        std::vector<int64_t> c64(cnt32[c].begin(), cnt32[c].end());
        int64_t nsp[kMaxSpecies];
        if (bad[c] || !species_totals(g, c64.data(), nsp)) {
            set_error("chain " + std::to_string(c) +
                      ": species ids must lie in [0, n_species) and every species must occur");
            return PYHEA_EINVAL;
        }
        Rtab[c].resize(c64.size());
        ratio_table(g, nsp, Rtab[c].data());
        ChainState st0;
        std::memset(&st0, 0, sizeof(st0));
        PYHEA_HIP(hipMemcpyAsync(base + slot[c].R, Rtab[c].data(), Rtab[c].size() * 8,
                                 hipMemcpyHostToDevice, stream));
        PYHEA_HIP(hipMemcpyAsync(base + slot[c].target, jobs[c].target.data(), jobs[c].target.size() * 8,
                                 hipMemcpyHostToDevice, stream));
        PYHEA_HIP(hipMemcpyAsync(base + slot[c].state, &st0, sizeof(st0), hipMemcpyHostToDevice, stream));
    }

    // descriptors, grouped by launch shape (store, M, S, B, H)
    std::map<std::tuple<int, int, int, int, int>, std::vector<int>> groups;
    std::vector<ChainDesc> descs(n);
    for (int c = 0; c < n; ++c) {
        const ChainJob &j = jobs[c];
        ChainDesc &d = descs[c];
        std::memset(&d, 0, sizeof(d));
        fill_chain_geometry(j.g, &d);
        d.seed = j.params.seed;
        d.chain_id = j.params.chain_id;
        d.B = j.params.cand_per_step;
        d.n_trials = j.params.n_trials;
        d.mode = j.params.commit_mode;
        d.depth_limit = j.params.depth_limit;
        d.tau = j.params.accept_tol;
        for (int k = 0; k < kMaxShells; ++k) d.w[k] = k < j.g.S ? j.weight[k] : 0.0;
        d.species = j.species_dev;
        d.pad_global = slot[c].store == kStoreGlobal ? (int8_t *)(base + slot[c].pad) : nullptr;
        d.R = (const double *)(base + slot[c].R);
        d.target = (const double *)(base + slot[c].target);
        d.counts = (int32_t *)(base + slot[c].counts);
        d.log = j.log_dev;
        d.log_cap = j.log_dev ? j.log_cap : 0;
        d.state = (ChainState *)(base + slot[c].state);
        d.store = slot[c].store;
        d.lds_bytes = slot[c].lds;
        groups[{slot[c].store, j.g.M, j.g.S, d.B, slot[c].H}].push_back(c);
    }
    DeviceBuffer dbuf;
    PYHEA_HIP(hipMalloc(&dbuf.ptr, sizeof(ChainDesc) * n));
    std::vector<ChainDesc> ordered;
    ordered.reserve(n);
    std::vector<std::pair<size_t, std::vector<int>>> launches;
    for (auto &kv : groups) {
        launches.push_back({ordered.size(), kv.second});
        // longest chains first so the tail of the launch is short
        std::vector<int> idx = kv.second;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
            return jobs[a].params.n_trials > jobs[b].params.n_trials;
        });
        launches.back().second = idx;
        for (int c : idx) ordered.push_back(descs[c]);
    }
    PYHEA_HIP(hipMemcpyAsync(dbuf.ptr, ordered.data(), sizeof(ChainDesc) * n, hipMemcpyHostToDevice, stream));
    const ChainDesc *ddev = (const ChainDesc *)dbuf.ptr;
    for (auto &L : launches) {
        const int first = (int)L.first, count = (int)L.second.size();
        const ChainDesc &d0 = descs[L.second[0]];
        int lds = 0;
        for (int c : L.second) lds = std::max(lds, descs[c].lds_bytes);
        if (d0.store == kStoreGlobal) PYHEA_HIP(launch_pad_fill(ddev + first, count, stream));
        PYHEA_HIP(launch_mc(ddev + first, count, d0.store, d0.M, d0.S, d0.B, slot[L.second[0]].H, lds, INT_MAX,
                            stream));
        if (d0.store == kStoreGlobal) PYHEA_HIP(launch_pad_drain(ddev + first, count, stream));
    }

    // results: states, maintained counts, and a fresh recount of the final configuration
    for (int c = 0; c < n; ++c) {
        const pyhea_status s = count_configs(jobs[c].g, 1, jobs[c].species_dev, (int32_t *)(base + slot[c].recount),
                                             (int32_t *)(base + slot[c].bad), stream);
        if (s != PYHEA_OK) return s;
    }
    std::vector<ChainState> sts(n);
    std::vector<std::vector<int32_t>> rec32(n);
    for (int c = 0; c < n; ++c) {
        PYHEA_HIP(hipMemcpyAsync(&sts[c], base + slot[c].state, sizeof(ChainState), hipMemcpyDeviceToHost, stream));
        PYHEA_HIP(hipMemcpyAsync(cnt32[c].data(), base + slot[c].counts, cnt32[c].size() * 4,
                                 hipMemcpyDeviceToHost, stream));
        rec32[c].resize(cnt32[c].size());
        PYHEA_HIP(hipMemcpyAsync(rec32[c].data(), base + slot[c].recount, rec32[c].size() * 4,
                                 hipMemcpyDeviceToHost, stream));
    }
    PYHEA_HIP(hipStreamSynchronize(stream));
    if (final_counts) final_counts->assign(n, {});
    for (int c = 0; c < n; ++c) {
        const Geometry &g = jobs[c].g;
        if (rec32[c] != cnt32[c]) {
            set_error("chain " + std::to_string(c) + ": maintained pair counts differ from a recount");
            return PYHEA_EDEVICE;
        }
        std::vector<int64_t> c64(rec32[c].begin(), rec32[c].end());
        pyhea_mc_stats &s = stats[c];
        std::memset(&s, 0, sizeof(s));
        s.trials = sts[c].trials;
        s.null_trials = sts[c].null_trials;
        s.commits = sts[c].commits;
        s.steps = sts[c].steps;
        s.stop_reason = sts[c].stop_reason;
        s.status = PYHEA_OK;
        double SF[2];
        host_objective(g, c64.data(), jobs[c].target.data(), jobs[c].weight.data(), nullptr, SF);
        s.S = SF[0];
        s.F = SF[1];
        s.log_len = jobs[c].log_dev ? std::min(s.commits, jobs[c].log_cap) : 0;
        if (final_counts) (*final_counts)[c] = c64;
    }
    return PYHEA_OK;
}

}  // namespace pyhea
