// Serving API: continuous batching of Monte Carlo structure-generation jobs.
//
// A worker thread owns the GPU work.  Each round it (1) retires jobs whose
// chains finished in the previous round (results copied to host, device
// memory released), (2) admits queued jobs in arrival order while a slot is
// free and their HBM footprint fits the budget (configuration, padded copy,
// counts and tables stay resident on the device), and (3) advances every
// resident job by up to `steps_per_round` MC steps with one persistent launch
// per launch shape, the shapes on separate streams so they overlap.  A job's
// trajectory depends only on its own inputs (seed, chain id = job id, B,
// budget): rounds are cut at step boundaries and the chain state (step, trial
// and depth counters, counts, configuration) persists between launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "pyhea.h"
#include "autotune.h"
#include "runtime.h"

using namespace pyhea;

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum JobPhase { kQueued, kResident, kDone, kCancelled, kFailed };

struct Job {
    uint64_t id = 0;
    Geometry g;
    pyhea_mc_params params{};
    std::vector<double> target, weight;
    std::vector<int8_t> species;  // input, then the final configuration
    JobPhase phase = kQueued;
    bool cancel = false;
    int32_t status = PYHEA_OK;
    pyhea_mc_stats stats{};
    int64_t t_submit = 0, t_admit = 0, t_finish = 0;
    // device residency
    int64_t footprint = 0;
    void *mem = nullptr;
    ChainDesc desc{};
    int store = kStoreLds8;
    int lds = 0;
    int H = 1;
    size_t off_counts = 0, off_recount = 0, off_bad = 0, off_R = 0, off_t = 0, off_state = 0,
           off_species = 0, off_pad = 0;
};

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

struct Server {
    int device = 0;
    int64_t budget = 0;
    int max_slots = 0;
    int steps_per_round = 256;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
    std::deque<uint64_t> queue;
    std::vector<Job *> resident;
    bool stop = false;
    std::thread worker;
    int64_t n_submitted = 0, n_admitted = 0, n_finished = 0, n_rejected = 0, n_rounds = 0;
    int64_t bytes_resident = 0;
    std::vector<hipStream_t> streams;
    void *desc_dev = nullptr;
    int lds_budget = 0;
    std::string worker_error;

    void run();
    bool admit(Job *j, hipStream_t s);
    void retire(Job *j, hipStream_t s);
    void release(Job *j);
};

int64_t job_footprint(const Geometry &g, int store) {
    const int64_t E = (int64_t)g.S * g.M * g.M;
    int64_t b = 0;
    b += a256(E * 4) * 2 + a256(4) + a256(E * 8) * 2 + a256(sizeof(ChainState));
    b += a256((size_t)g.N);
    if (store == kStoreGlobal) b += a256((size_t)g.Npad);
    return b;
}

bool Server::admit(Job *j, hipStream_t s) {
    const Geometry &g = j->g;
    const size_t E = (size_t)g.S * g.M * g.M;
    size_t off = 0;
    j->off_counts = off;
    off = a256(off + E * 4);
    j->off_recount = off;
    off = a256(off + E * 4);
    j->off_bad = off;
    off = a256(off + 4);
    j->off_R = off;
    off = a256(off + E * 8);
    j->off_t = off;
    off = a256(off + E * 8);
    j->off_state = off;
    off = a256(off + sizeof(ChainState));
    j->off_species = off;
    off = a256(off + (size_t)g.N);
    j->off_pad = off;
    if (j->store == kStoreGlobal) off = a256(off + (size_t)g.Npad);
    if (hipMalloc(&j->mem, off) != hipSuccess) {
        j->mem = nullptr;
        return false;
    }
    char *base = (char *)j->mem;
    // n_i from the host copy (same integers the counts give), then R
    int64_t n[kMaxSpecies] = {0};
    for (int8_t v : j->species) n[v]++;
    std::vector<double> R(E);
    ratio_table(g, n, R.data());
    ChainState st0;
    std::memset(&st0, 0, sizeof(st0));
    bool ok = hipMemcpyAsync(base + j->off_species, j->species.data(), g.N, hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(base + j->off_R, R.data(), E * 8, hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(base + j->off_t, j->target.data(), E * 8, hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(base + j->off_state, &st0, sizeof(st0), hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && count_configs(g, 1, (const int8_t *)(base + j->off_species), (int32_t *)(base + j->off_counts),
                             (int32_t *)(base + j->off_bad), s) == PYHEA_OK;
    ChainDesc &d = j->desc;
    std::memset(&d, 0, sizeof(d));
    fill_chain_geometry(g, &d);
    d.seed = j->params.seed;
    d.chain_id = j->params.chain_id;
    d.B = j->params.cand_per_step;
    d.n_trials = j->params.n_trials;
    d.mode = j->params.commit_mode;
    d.depth_limit = j->params.depth_limit;
    d.tau = j->params.accept_tol;
    for (int k = 0; k < kMaxShells; ++k) d.w[k] = k < g.S ? j->weight[k] : 0.0;
    d.species = (int8_t *)(base + j->off_species);
    d.pad_global = j->store == kStoreGlobal ? (int8_t *)(base + j->off_pad) : nullptr;
    d.R = (const double *)(base + j->off_R);
    d.target = (const double *)(base + j->off_t);
    d.counts = (int32_t *)(base + j->off_counts);
    d.log = nullptr;
    d.log_cap = 0;
    d.state = (ChainState *)(base + j->off_state);
    d.store = j->store;
    d.lds_bytes = j->lds;
    if (ok && j->store == kStoreGlobal) {
        // one-chain descriptor copy for the padding kernel
        void *tmp = nullptr;
        ok = hipMalloc(&tmp, sizeof(ChainDesc)) == hipSuccess;
        ok = ok && hipMemcpyAsync(tmp, &d, sizeof(d), hipMemcpyHostToDevice, s) == hipSuccess;
        ok = ok && launch_pad_fill((const ChainDesc *)tmp, 1, s) == hipSuccess;
        ok = ok && hipStreamSynchronize(s) == hipSuccess;
        if (tmp) (void)hipFree(tmp);
    }
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    return ok;
}

void Server::retire(Job *j, hipStream_t s) {
    const Geometry &g = j->g;
    char *base = (char *)j->mem;
    const size_t E = (size_t)g.S * g.M * g.M;
    bool ok = true;
    if (j->store == kStoreGlobal) {
        void *tmp = nullptr;
        ok = hipMalloc(&tmp, sizeof(ChainDesc)) == hipSuccess;
        ok = ok && hipMemcpyAsync(tmp, &j->desc, sizeof(ChainDesc), hipMemcpyHostToDevice, s) == hipSuccess;
        ok = ok && launch_pad_drain((const ChainDesc *)tmp, 1, s) == hipSuccess;
        ok = ok && hipStreamSynchronize(s) == hipSuccess;
        if (tmp) (void)hipFree(tmp);
    }
    ok = ok && count_configs(g, 1, (const int8_t *)(base + j->off_species), (int32_t *)(base + j->off_recount),
                             (int32_t *)(base + j->off_bad), s) == PYHEA_OK;
    ChainState st;
    std::vector<int32_t> cm(E), cr(E);
    ok = ok && hipMemcpyAsync(&st, base + j->off_state, sizeof(st), hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(cm.data(), base + j->off_counts, E * 4, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(cr.data(), base + j->off_recount, E * 4, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(j->species.data(), base + j->off_species, g.N, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    std::memset(&j->stats, 0, sizeof(j->stats));
    if (!ok || cm != cr) {
        j->status = PYHEA_EDEVICE;
    } else {
        std::vector<int64_t> c64(cr.begin(), cr.end());
        double SF[2];
        host_objective(g, c64.data(), j->target.data(), j->weight.data(), nullptr, SF);
        j->stats.trials = st.trials;
        j->stats.null_trials = st.null_trials;
        j->stats.commits = st.commits;
        j->stats.steps = st.steps;
        j->stats.stop_reason = st.stop_reason;
        j->stats.S = SF[0];
        j->stats.F = SF[1];
        j->stats.status = PYHEA_OK;
    }
    j->stats.status = j->status;
}

void Server::release(Job *j) {
    if (j->mem) (void)hipFree(j->mem);
    j->mem = nullptr;
    bytes_resident -= j->footprint;
}

void Server::run() {
    (void)hipSetDevice(device);
    hipStream_t s0 = streams[0];
    std::vector<ChainState> states;
    for (;;) {
        std::vector<Job *> to_admit;
        {
            std::unique_lock<std::mutex> lk(mu);
            // admit in arrival order while slots and budget allow
            for (auto it = queue.begin(); it != queue.end();) {
                Job *j = jobs.count(*it) ? jobs[*it].get() : nullptr;
                if (!j || j->phase != kQueued) {
                    it = queue.erase(it);
                    continue;
                }
                if ((int)(resident.size() + to_admit.size()) >= max_slots) break;
                if (bytes_resident + j->footprint > budget) {
                    ++it;
                    continue;
                }
                bytes_resident += j->footprint;
                to_admit.push_back(j);
                it = queue.erase(it);
            }
            if (resident.empty() && to_admit.empty()) {
                if (stop) return;
                cv_work.wait(lk, [&] { return stop || !queue.empty(); });
                if (stop && queue.empty()) return;
                continue;
            }
        }
        for (Job *j : to_admit) {
            const bool ok = admit(j, s0);
            std::lock_guard<std::mutex> lk(mu);
            if (!ok) {
                release(j);
                j->status = PYHEA_ENOMEM;
                j->phase = kFailed;
                j->t_finish = now_ns();
                ++n_finished;
                cv_done.notify_all();
                continue;
            }
            j->phase = kResident;
            j->t_admit = now_ns();
            resident.push_back(j);
            ++n_admitted;
        }
        std::vector<Job *> run_set;
        {
            std::lock_guard<std::mutex> lk(mu);
            run_set = resident;
            if (stop) run_set.clear();
        }
        if (run_set.empty()) {
            std::lock_guard<std::mutex> lk(mu);
            if (stop) return;
            continue;
        }
        // one round: group by launch shape, one stream per group
        std::map<std::tuple<int, int, int, int, int>, std::vector<Job *>> groups;
        for (Job *j : run_set)
            groups[{j->store, j->g.M, j->g.S, j->params.cand_per_step, j->H}].push_back(j);
        std::vector<ChainDesc> descs;
        std::vector<std::pair<size_t, std::vector<Job *>>> launches;
        for (auto &kv : groups) {
            launches.push_back({descs.size(), kv.second});
            for (Job *j : kv.second) descs.push_back(j->desc);
        }
        bool ok = hipMemcpyAsync(desc_dev, descs.data(), descs.size() * sizeof(ChainDesc), hipMemcpyHostToDevice,
                                 s0) == hipSuccess;
        ok = ok && hipStreamSynchronize(s0) == hipSuccess;
        for (size_t gi = 0; ok && gi < launches.size(); ++gi) {
            auto &L = launches[gi];
            const Job *j0 = L.second[0];
            int lds = 0;
            for (Job *j : L.second) lds = std::max(lds, j->lds);
            hipStream_t s = streams[gi % streams.size()];
            ok = launch_mc((const ChainDesc *)desc_dev + L.first, (int)L.second.size(), j0->store, j0->g.M,
                           j0->g.S, j0->params.cand_per_step, j0->H, lds, steps_per_round, s) == hipSuccess;
        }
        for (hipStream_t s : streams) ok = ok && hipStreamSynchronize(s) == hipSuccess;
        // done flags
        states.resize(run_set.size());
        for (size_t i = 0; ok && i < run_set.size(); ++i)
            ok = hipMemcpyAsync(&states[i], run_set[i]->desc.state, sizeof(ChainState), hipMemcpyDeviceToHost, s0) ==
                 hipSuccess;
        ok = ok && hipStreamSynchronize(s0) == hipSuccess;
        std::vector<Job *> finished, cancelled;
        {
            std::lock_guard<std::mutex> lk(mu);
            ++n_rounds;
            for (size_t i = 0; i < run_set.size(); ++i) {
                Job *j = run_set[i];
                if (!ok) {
                    j->status = PYHEA_EDEVICE;
                    finished.push_back(j);
                } else if (j->cancel) {
                    cancelled.push_back(j);
                } else if (states[i].done) {
                    finished.push_back(j);
                }
            }
        }
        for (Job *j : finished)
            if (j->status == PYHEA_OK) retire(j, s0);
        {
            std::lock_guard<std::mutex> lk(mu);
            for (Job *j : finished) {
                j->phase = j->status == PYHEA_OK ? kDone : kFailed;
                j->stats.status = j->status;
                j->t_finish = now_ns();
                release(j);
                resident.erase(std::find(resident.begin(), resident.end(), j));
                ++n_finished;
            }
            for (Job *j : cancelled) {
                release(j);
                j->phase = kCancelled;
                j->status = PYHEA_ECANCELLED;
                j->t_finish = now_ns();
                resident.erase(std::find(resident.begin(), resident.end(), j));
                ++n_finished;
            }
            if (!ok) worker_error = "device error during a serving round";
        }
        cv_done.notify_all();
    }
}

Server *as_server(void *p) { return static_cast<Server *>(p); }

}  // namespace

extern "C" {

pyhea_status pyhea_serve_open(int64_t hbm_budget_bytes, int32_t max_slots, int32_t steps_per_round,
                              void **server) {
    if (!server || hbm_budget_bytes <= 0 || max_slots < 1 || max_slots > 65535 || steps_per_round < 0) {
        set_error("serve_open: need server != NULL, budget > 0, 1 <= max_slots <= 65535, steps_per_round >= 0");
        return PYHEA_EINVAL;
    }
    auto *s = new Server();
    PYHEA_HIP(hipGetDevice(&s->device));
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->steps_per_round = steps_per_round > 0 ? steps_per_round : 256;
    s->lds_budget = max_lds_per_block();
    s->streams.resize(4);
    for (auto &st : s->streams) {
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            set_error("serve_open: stream creation failed");
            return PYHEA_EDEVICE;
        }
    }
    if (hipMalloc(&s->desc_dev, sizeof(ChainDesc) * (size_t)max_slots) != hipSuccess) {
        for (auto st : s->streams) (void)hipStreamDestroy(st);
        delete s;
        set_error("serve_open: descriptor table allocation failed");
        return PYHEA_ENOMEM;
    }
    s->worker = std::thread([s] { s->run(); });
    *server = s;
    set_error("");
    return PYHEA_OK;
}

pyhea_status pyhea_serve_submit(void *server, uint64_t job_id, const pyhea_lattice *lat, const pyhea_objective *obj,
                                const pyhea_mc_params *params, const int8_t *species_host) {
    Server *s = as_server(server);
    if (!s || !species_host) {
        set_error("serve_submit: server and species_host must not be NULL");
        return PYHEA_EINVAL;
    }
    auto j = std::make_unique<Job>();
    std::string err;
    if (build_geometry(lat, &j->g, &err) != PYHEA_OK) {
        set_error("serve_submit: " + err);
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->n_rejected;
        return PYHEA_EINVAL;
    }
    pyhea_status st = check_objective(j->g, obj);
    if (st == PYHEA_OK) st = check_params(params);
    if (st != PYHEA_OK) {
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->n_rejected;
        return st;
    }
    const Geometry &g = j->g;
    j->species.assign(species_host, species_host + g.N);
    int64_t n[kMaxSpecies] = {0};
    for (int8_t v : j->species) {
        if (v < 0 || v >= g.M) {
            set_error("serve_submit: species ids must lie in [0, n_species)");
            std::lock_guard<std::mutex> lk(s->mu);
            ++s->n_rejected;
            return PYHEA_EINVAL;
        }
        n[v]++;
    }
    for (int i = 0; i < g.M; ++i)
        if (n[i] == 0) {
            set_error("serve_submit: every species must occur");
            std::lock_guard<std::mutex> lk(s->mu);
            ++s->n_rejected;
            return PYHEA_EINVAL;
        }
    j->id = job_id;
    j->params = *params;
    j->params.chain_id = (uint32_t)job_id;
    const int E = g.S * g.M * g.M;
    j->target.assign(obj->target, obj->target + E);
    j->weight.assign(obj->weight, obj->weight + g.S);
    const LaunchShape ls = choose_launch(g, params->cand_per_step, s->lds_budget, 0);
    j->store = ls.store;
    j->lds = ls.lds;
    j->H = ls.H;
    j->footprint = job_footprint(g, j->store);
    std::lock_guard<std::mutex> lk(s->mu);
    if (j->footprint > s->budget) {
        set_error("serve_submit: the job's HBM footprint exceeds the server budget");
        ++s->n_rejected;
        return PYHEA_ENOMEM;
    }
    if (s->jobs.count(job_id)) {
        set_error("serve_submit: duplicate job id");
        ++s->n_rejected;
        return PYHEA_EINVAL;
    }
    j->t_submit = now_ns();
    s->queue.push_back(job_id);
    s->jobs[job_id] = std::move(j);
    ++s->n_submitted;
    s->cv_work.notify_all();
    set_error("");
    return PYHEA_OK;
}

pyhea_status pyhea_serve_poll(void *server, uint64_t job_id, int8_t *species_out_host, pyhea_mc_stats *stats_host,
                              int64_t *times_ns_host, int32_t blocking) {
    Server *s = as_server(server);
    if (!s) {
        set_error("serve_poll: server must not be NULL");
        return PYHEA_EINVAL;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) {
        set_error("serve_poll: unknown job id");
        return PYHEA_ENOENT;
    }
    Job *j = it->second.get();
    auto finished = [&] { return j->phase == kDone || j->phase == kCancelled || j->phase == kFailed; };
    if (!finished()) {
        if (!blocking) return PYHEA_EBUSY;
        s->cv_done.wait(lk, [&] { return finished() || (s->stop && s->worker_error.size()); });
        if (!finished()) {
            set_error("serve_poll: server stopped");
            return PYHEA_EDEVICE;
        }
    }
    if (stats_host) *stats_host = j->stats;
    if (times_ns_host) {
        times_ns_host[0] = j->t_submit;
        times_ns_host[1] = j->t_admit;
        times_ns_host[2] = j->t_finish;
    }
    const int32_t status = j->phase == kCancelled ? PYHEA_ECANCELLED : j->status;
    if (species_out_host && j->phase == kDone) std::memcpy(species_out_host, j->species.data(), j->g.N);
    s->jobs.erase(it);
    if (status != PYHEA_OK) set_error("serve_poll: job ended with an error");
    return status;
}

pyhea_status pyhea_serve_cancel(void *server, uint64_t job_id) {
    Server *s = as_server(server);
    if (!s) return PYHEA_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) {
        set_error("serve_cancel: unknown job id");
        return PYHEA_ENOENT;
    }
    Job *j = it->second.get();
    if (j->phase == kQueued) {
        j->phase = kCancelled;
        j->status = PYHEA_ECANCELLED;
        j->t_finish = now_ns();
        ++s->n_finished;
        s->cv_done.notify_all();
    } else if (j->phase == kResident) {
        j->cancel = true;
    }
    return PYHEA_OK;
}

pyhea_status pyhea_serve_counters(void *server, int64_t *out8_host) {
    Server *s = as_server(server);
    if (!s || !out8_host) return PYHEA_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    int64_t queued = 0;
    for (auto &kv : s->jobs) queued += kv.second->phase == kQueued;
    out8_host[0] = s->n_submitted;
    out8_host[1] = s->n_admitted;
    out8_host[2] = s->n_finished;
    out8_host[3] = s->n_rejected;
    out8_host[4] = (int64_t)s->resident.size();
    out8_host[5] = queued;
    out8_host[6] = s->n_rounds;
    out8_host[7] = s->bytes_resident;
    return PYHEA_OK;
}

pyhea_status pyhea_serve_close(void *server) {
    Server *s = as_server(server);
    if (!s) return PYHEA_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->queue.clear();
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->device);
    for (Job *j : s->resident) {
        if (j->mem) (void)hipFree(j->mem);
        j->mem = nullptr;
    }
    if (s->desc_dev) (void)hipFree(s->desc_dev);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return PYHEA_OK;
}

}  // extern "C"
